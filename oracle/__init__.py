"""Python access to the FP64 CPU oracle (``oracle/liboracle.so``).

TEST INFRASTRUCTURE ONLY: used by ``tests/``, the smoke check and the CPU
baseline leg of ``bench.py``.  The product library never loads it.

The oracle is a plain sequential C transcription of the scheme of
"AVIP: a low temperature plasma code" (arXiv 2201.01291); see ``oracle.c`` for
the passages each function follows.  ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
MAXSP = 16

# model / flux / limiter codes of the oracle
GAS, DRIFT_DIFFUSION, NAVIER_STOKES = 0, 1, 2
HLLC, ROE = 0, 1
LLW, SG = 0, 2   # drift-diffusion schemes
FIRST_ORDER, MINMOD, VANLEER, SWEBY, UNLIMITED = 0, 1, 2, 3, 4


def build(verbose: bool = False) -> str:
    """Compile liboracle.so (plain gcc, -O2, no fast-math, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", LIB_PATH, os.path.join(HERE, "oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB_PATH


class _Phys(C.Structure):
    _fields_ = [("model", C.c_int32), ("flux", C.c_int32), ("limiter", C.c_int32),
                ("rk", C.c_int32), ("nspecies", C.c_int32), ("closure", C.c_int32),
                ("predictor", C.c_int32), ("beta", C.c_double), ("cfl", C.c_double), ("fourier", C.c_double),
                ("gamma", C.c_double), ("entropy_fix", C.c_double),
                ("z", C.c_double * MAXSP), ("mu", C.c_double * MAXSP),
                ("D", C.c_double * MAXSP),
                ("Wk", C.c_double * MAXSP), ("cpa", C.c_double * MAXSP),
                ("cpb", C.c_double * MAXSP), ("cpc", C.c_double * MAXSP),
                ("Sc", C.c_double * MAXSP), ("mu_ref", C.c_double), ("T_ref", C.c_double),
                ("Pr", C.c_double), ("diel", C.c_double)]


@dataclass
class Phys:
    model: int = GAS
    flux: int = HLLC
    limiter: int = MINMOD
    rk: int = 2
    nspecies: int = 0
    closure: int = 1         # 0 none, 1 node flux, 2 interpolated (2D)
    predictor: int = 0       # gas, plane meshes, rk 1: MUSCL-Hancock half-step predictor
    beta: float = 1.0
    cfl: float = 0.5
    fourier: float = 0.25
    gamma: float = 1.4
    entropy_fix: float = 0.1
    z: list = field(default_factory=list)
    mu: list = field(default_factory=list)
    D: list = field(default_factory=list)
    mixture: object = None   # workloads.Mixture for the Navier-Stokes model
    diel: float = 0.0        # drift-diffusion: dielectric time-step constant A_D (0: off)

    def to_c(self) -> _Phys:
        p = _Phys()
        p.model, p.flux, p.limiter, p.rk = self.model, self.flux, self.limiter, self.rk
        p.nspecies, p.closure = self.nspecies, int(self.closure)
        p.predictor = int(self.predictor)
        p.beta, p.cfl, p.fourier = self.beta, self.cfl, self.fourier
        p.gamma, p.entropy_fix = self.gamma, self.entropy_fix
        p.diel = self.diel
        for k, (z, mu, D) in enumerate(zip(self.z, self.mu, self.D)):
            p.z[k], p.mu[k], p.D[k] = z, mu, D
        if self.mixture is not None:
            mx = self.mixture
            for k in range(mx.n):
                p.Wk[k], p.cpa[k], p.cpb[k] = mx.W[k], mx.cp_a[k], mx.cp_b[k]
                p.cpc[k], p.Sc[k] = mx.cp_c[k], mx.Sc[k]
            p.mu_ref, p.T_ref, p.Pr = mx.mu_ref, mx.T_ref, mx.Pr
        return p

    def nvar(self, nd: int) -> int:
        return self.nspecies if self.model == DRIFT_DIFFUSION else 2 + nd + self.nspecies


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int64)
        L.om_mesh_create.restype = C.c_void_p
        L.om_mesh_create.argtypes = [C.c_int, C.c_int64, dp, C.c_int64, C.c_int, ip, dp,
                                     C.POINTER(C.c_int)]
        L.om_mesh_create_axi.restype = C.c_void_p
        L.om_mesh_create_axi.argtypes = [C.c_int, C.c_int64, dp, C.c_int64, C.c_int, ip, dp, C.c_int,
                                         C.POINTER(C.c_int)]
        L.om_axi_geometry.argtypes = [C.c_void_p, dp, dp]
        L.om_mesh_destroy.argtypes = [C.c_void_p]
        L.om_mesh_counts.argtypes = [C.c_void_p, ip]
        L.om_geometry.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.om_edge_normals.argtypes = [C.c_void_p, dp, ip]
        L.om_gradient.argtypes = [C.c_void_p, C.c_int, dp, dp]
        L.om_slope_limiter.restype = C.c_double
        L.om_slope_limiter.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double]
        L.om_psi_limiter.restype = C.c_double
        L.om_psi_limiter.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double]
        L.om_euler_flux.argtypes = [C.c_int, C.c_int, dp, dp, dp]
        L.om_hllc.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, dp, dp, dp, dp]
        L.om_roe.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, dp, dp, dp, dp]
        L.om_flux_branches.argtypes = [ip, C.c_int]
        L.om_hancock_rate.argtypes = [C.c_int, C.c_int, C.c_double, dp, dp, dp]
        L.om_sg_flux.restype = C.c_double
        L.om_sg_flux.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp, dp, C.c_double, dp]
        L.om_ns_conserved.argtypes = [C.c_int, C.POINTER(_Phys), dp, dp]
        pp = C.POINTER(_Phys)
        L.om_residual.argtypes = [C.c_void_p, pp, dp, dp, C.c_double, dp]
        L.om_flux_scale.argtypes = [C.c_void_p, pp, dp, dp, C.c_double, dp]
        L.om_timestep.argtypes = [C.c_void_p, pp, dp, dp, dp]
        L.om_step.argtypes = [C.c_void_p, pp, dp, dp, C.c_int, C.c_double, dp, dp,
                              C.POINTER(C.c_int)]
        L.om_sums.argtypes = [C.c_void_p, C.c_int, dp, dp, dp]
        L.om_poisson_coo.argtypes = [C.c_void_p, ip, ip, dp]
        L.om_boundary_measure.argtypes = [C.c_void_p, dp]
        L.om_ns_node.argtypes = [C.c_int, pp, dp, dp]
        L.om_viscous_flux.argtypes = [C.c_int, C.c_int, dp, dp, C.c_double, C.c_double, dp, dp,
                                      dp, dp, dp, dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


class OracleMesh:
    """FP64 oracle view of a mesh (geometry computed once at construction)."""

    def __init__(self, mesh, axisymmetric: bool = False):
        L = lib()
        self.axi = bool(axisymmetric)
        self.nd, self.nn = mesh.ndim, mesh.nnodes
        self.nc, self.nv = mesh.ncells, mesh.nv
        self.ne = 3 if self.nv == 3 else (4 if self.nd == 2 else 6)
        xyz = _c64(mesh.xyz)
        cells = np.ascontiguousarray(mesh.cells, dtype=np.int64)
        per = None if mesh.period is None else _c64(mesh.period)
        st = C.c_int(0)
        h = L.om_mesh_create_axi(self.nd, self.nn, _d(xyz), self.nc, self.nv,
                                 cells.ctypes.data_as(C.POINTER(C.c_int64)),
                                 _d(per) if per is not None else None, int(self.axi), C.byref(st))
        if not h:
            raise OracleError(st.value, "mesh_create")
        self._h = C.c_void_p(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.om_mesh_destroy(h)
            self._h = None

    def counts(self):
        out = np.zeros(4, dtype=np.int64)
        lib().om_mesh_counts(self._h, out.ctypes.data_as(C.POINTER(C.c_int64)))
        return dict(nn=int(out[0]), nc=int(out[1]), nbfaces=int(out[2]), nbnodes=int(out[3]))

    def geometry(self):
        S = np.zeros((self.nc, self.nv, self.nd))
        Vc = np.zeros(self.nc)
        Vn = np.zeros(self.nn)
        Sb = np.zeros((self.nd, self.nn))
        lib().om_geometry(self._h, _d(S), _d(Vc), _d(Vn), _d(Sb))
        return dict(S=S, Vc=Vc, Vn=Vn, Sb=Sb)

    def axi_geometry(self):
        """Axisymmetric meshes: node volumes int r dA over 2 pi and the
        radius-weighted boundary normals [nd][nn]."""
        Vp = np.zeros(self.nn)
        Sbr = np.zeros((self.nd, self.nn))
        lib().om_axi_geometry(self._h, _d(Vp), _d(Sbr))
        return Vp, Sbr

    def edge_normals(self):
        Sij = np.zeros((self.nc, self.ne, self.nd))
        ends = np.zeros((self.nc, self.ne, 2), dtype=np.int64)
        lib().om_edge_normals(self._h, _d(Sij), ends.ctypes.data_as(C.POINTER(C.c_int64)))
        return Sij, ends

    def gradient(self, W):
        W = _c64(W)
        nvar = W.shape[0]
        G = np.zeros((nvar, self.nd, self.nn))
        lib().om_gradient(self._h, nvar, _d(W), _d(G))
        return G

    def residual(self, phys: Phys, U, E=None, dt: float = 0.0):
        U = _c64(U)
        r = np.zeros_like(U)
        Ec = None if E is None else _c64(E)
        p = phys.to_c()
        st = lib().om_residual(self._h, C.byref(p), _d(U), _d(Ec) if Ec is not None else None,
                               float(dt), _d(r))
        if st:
            raise OracleError(st, "residual")
        return r

    def flux_scale(self, phys: Phys, U, E=None, dt: float = 0.0):
        """Per node and variable, the sum of |F.S| over its cell-edges."""
        U = _c64(U)
        r = np.zeros_like(U)
        Ec = None if E is None else _c64(E)
        p = phys.to_c()
        st = lib().om_flux_scale(self._h, C.byref(p), _d(U), _d(Ec) if Ec is not None else None,
                                 float(dt), _d(r))
        if st:
            raise OracleError(st, "flux_scale")
        return r

    def timestep(self, phys: Phys, U, E=None) -> float:
        U = _c64(U)
        Ec = None if E is None else _c64(E)
        dt = C.c_double(0.0)
        p = phys.to_c()
        st = lib().om_timestep(self._h, C.byref(p), _d(U), _d(Ec) if Ec is not None else None,
                               C.byref(dt))
        if st:
            raise OracleError(st, "timestep")
        return dt.value

    def step(self, phys: Phys, U, E=None, nsteps: int = 1, t_end: float = 0.0, t0: float = 0.0,
             check: bool = True):
        U = _c64(U).copy()
        Ec = None if E is None else _c64(E)
        t, dtl, done = C.c_double(t0), C.c_double(0.0), C.c_int(0)
        p = phys.to_c()
        st = lib().om_step(self._h, C.byref(p), _d(U), _d(Ec) if Ec is not None else None,
                           int(nsteps), float(t_end), C.byref(t), C.byref(dtl), C.byref(done))
        if st and check:
            raise OracleError(st, "step")
        return U, t.value, dtl.value, done.value

    def poisson_matrix(self):
        """Matrix of -lap phi integrated over the nodal volumes (Sec.
        "Integrating the Poisson equation"), scipy CSR [nn x nn]."""
        import scipy.sparse as sp
        n = self.nc * self.nv * self.nv
        I = np.zeros(n, dtype=np.int64)
        K = np.zeros(n, dtype=np.int64)
        v = np.zeros(n)
        lib().om_poisson_coo(self._h, I.ctypes.data_as(C.POINTER(C.c_int64)),
                             K.ctypes.data_as(C.POINTER(C.c_int64)), _d(v))
        return sp.coo_matrix((v, (I, K)), shape=(self.nn, self.nn)).tocsr()

    def boundary_measure(self):
        out = np.zeros(self.nn)
        lib().om_boundary_measure(self._h, _d(out))
        return out

    def poisson_solve(self, q, dirichlet=None, phi_D=None, En=None):
        """Potential phi of -lap phi = q (q = rho / eps0 at the nodes),
        integrated over the nodal volumes:

          sum_k L_ik phi_k = q_i V_i - E_n,i |S_i^b|   (free node i)
          phi_i = phi_D,i                              (Dirichlet node i)

        (Sec. "Boundary conditions": Dirichlet rows replaced by the imposed
        value, Neumann data on the right-hand side, zero Neumann where
        nothing is imposed).  On axisymmetric meshes V_i and |S_i^b| are the
        revolved ones over 2 pi and the matrix is not symmetric (Sec.
        "Axisymmetric configuration").  Without Dirichlet nodes the matrix is
        singular: a uniform background charge makes the right-hand side
        compatible (q minus its volume mean) and phi is returned with zero
        volume mean.  Solved by a sparse direct factorisation."""
        import scipy.sparse as sp
        import scipy.sparse.linalg as spla
        L = self.poisson_matrix()
        Vn = self.axi_geometry()[0] if self.axi else self.geometry()["Vn"]
        b = np.asarray(q, dtype=np.float64) * Vn
        if En is not None:
            b = b - np.asarray(En, dtype=np.float64) * self.boundary_measure()
        if dirichlet is not None and np.any(dirichlet):
            dmask = np.asarray(dirichlet, dtype=bool)
            free = ~dmask
            phi = np.zeros(self.nn)
            phi[dmask] = np.asarray(phi_D, dtype=np.float64)[dmask]
            rhs = b[free] - L[free][:, dmask] @ phi[dmask]
            phi[free] = spla.spsolve(L[free][:, free].tocsc(), rhs)
            return phi
        b = b - Vn * (b.sum() / Vn.sum())
        one = np.ones((self.nn, 1))
        B = sp.bmat([[L, sp.csr_matrix(one)], [sp.csr_matrix(one.T), None]]).tocsc()
        sol = spla.spsolve(B, np.concatenate([b, [0.0]]))
        phi = sol[:self.nn]
        return phi - (Vn @ phi) / Vn.sum()

    def electric_field(self, phi):
        """E = -grad phi with the nodal gradient of the scheme (volume-weighted
        mean of the cell gradients), [nd][nn]."""
        return -self.gradient(np.asarray(phi, dtype=np.float64)[None, :])[0]

    def sums(self, U):
        U = _c64(U)
        nvar = U.shape[0]
        s, a = np.zeros(nvar), np.zeros(nvar)
        lib().om_sums(self._h, nvar, _d(U), _d(s), _d(a))
        return s, a


def slope_limiter(kind, beta, a, b) -> float:
    return lib().om_slope_limiter(int(kind), float(beta), float(a), float(b))


def psi_limiter(kind, beta, a, b) -> float:
    return lib().om_psi_limiter(int(kind), float(beta), float(a), float(b))


def euler_flux(nd, nsp, W, S):
    W, S = _c64(W), _c64(S)
    F = np.zeros(2 + nd + nsp)
    lib().om_euler_flux(nd, nsp, _d(W), _d(S), _d(F))
    return F


def hllc(nd, nsp, WL, WR, S, gL=1.4, gR=None):
    WL, WR, S = _c64(WL), _c64(WR), _c64(S)
    F = np.zeros(2 + nd + nsp)
    lib().om_hllc(nd, nsp, float(gL), float(gL if gR is None else gR), _d(WL), _d(WR), _d(S), _d(F))
    return F


def flux_branches(reset: bool = True) -> dict:
    """Counts of the Riemann-flux branches taken since the last reset (test
    instrumentation of the oracle), and reset them."""
    out = np.zeros(6, dtype=np.int64)
    lib().om_flux_branches(out.ctypes.data_as(C.POINTER(C.c_int64)), int(reset))
    keys = ("hllc_left_supersonic", "hllc_right_supersonic", "hllc_star_left",
            "hllc_star_right", "roe_calls", "roe_entropy_fix")
    return dict(zip(keys, (int(v) for v in out)))


def hancock_rate(nd, nsp, w, g, gamma=1.4):
    """MUSCL-Hancock half-step rate of one node: the time derivative of
    (rho, rho u, rho E, rho Y, p) from the node state w [nr] and its gradients
    g [nr][nd]."""
    w, g = _c64(w), _c64(g)
    out = np.zeros(3 + nd + nsp)
    lib().om_hancock_rate(nd, nsp, float(gamma), _d(w), _d(g), _d(out))
    return out


def sg_flux(ui, uj, V, S, dx, D, gbar):
    """Scharfetter-Gummel flux of one species through S on the edge i -> j."""
    V, S, dx, gbar = _c64(V), _c64(S), _c64(dx), _c64(gbar)
    return lib().om_sg_flux(len(S), float(ui), float(uj), _d(V), _d(S), _d(dx), float(D), _d(gbar))


def roe(nd, nsp, WL, WR, S, gamma=1.4, fix=0.1):
    WL, WR, S = _c64(WL), _c64(WR), _c64(S)
    F = np.zeros(2 + nd + nsp)
    lib().om_roe(nd, nsp, float(gamma), float(fix), _d(WL), _d(WR), _d(S), _d(F))
    return F


def ns_node(nd, phys: Phys, Ui):
    """(T, p, gamma, mu, lambda, D_k..., hs_k...) of one multi-species node state."""
    Ui = _c64(Ui)
    out = np.zeros(5 + 2 * phys.nspecies)
    p = phys.to_c()
    lib().om_ns_node(nd, C.byref(p), _d(Ui), _d(out))
    return out


def ns_conserved(nd, phys: Phys, prim):
    """Conserved multi-species state from (rho, u, T, Y) at one node."""
    prim = np.ascontiguousarray(prim, dtype=np.float64)
    U = np.zeros(2 + nd + phys.nspecies)
    p = phys.to_c()
    lib().om_ns_conserved(nd, C.byref(p), _d(prim), _d(U))
    return U


def conserved_from_primitive(nd, phys: Phys, P):
    """Conserved state [nvar][nn] from primitive rows [nvar][nn]: gas (rho, u,
    p, Y) with the constant-gamma ideal gas, multi-species (rho, u, T, Y) with
    the mixture's sensible energy, drift-diffusion densities unchanged."""
    P = np.asarray(P, dtype=np.float64)
    if phys.model == DRIFT_DIFFUSION:
        return P.copy()
    if phys.model == NAVIER_STOKES:
        return np.stack([ns_conserved(nd, phys, P[:, i]) for i in range(P.shape[1])], axis=1)
    rho, u, p = P[0], P[1:1 + nd], P[1 + nd]
    rows = [rho] + [rho * v for v in u] + [p / (phys.gamma - 1.0) + 0.5 * rho * np.sum(u * u, axis=0)]
    rows += [rho * y for y in P[2 + nd:]]
    return np.stack(rows)


def viscous_flux(nd, nsp, prim_i, prim_j, rho_i, rho_j, aux_i, aux_j, gprim_i, gprim_j, S):
    args = [_c64(a) for a in (prim_i, prim_j)]
    aux = [_c64(a) for a in (aux_i, aux_j)]
    g = [_c64(a) for a in (gprim_i, gprim_j)]
    S = _c64(S)
    Fv = np.zeros(2 + nd + nsp)
    lib().om_viscous_flux(nd, nsp, _d(args[0]), _d(args[1]), float(rho_i), float(rho_j),
                          _d(aux[0]), _d(aux[1]), _d(g[0]), _d(g[1]), _d(S), _d(Fv))
    return Fv


def prim_to_W(rho, vel, p, gamma=1.4, Y=()):
    """Reconstructed-variable vector (rho, rho u, rho E, rho Y, p) of one
    state, for the point-wise flux functions."""
    vel = np.asarray(vel, dtype=np.float64)
    rE = p / (gamma - 1.0) + 0.5 * rho * float(vel @ vel)
    return np.concatenate([[rho], rho * vel, [rE], rho * np.asarray(Y, dtype=np.float64), [p]])
