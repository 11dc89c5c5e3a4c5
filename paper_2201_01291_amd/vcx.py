"""Thin Python binding of ``libvcx.so`` (the C ABI in ``include/vcx.h``).

Argument marshalling only: every step of the residual, the update and the
time step runs in the library's HIP kernels.  Device memory and streams may
come from PyTorch (CUDA/HIP tensors are passed by pointer with
``is_device = 1``); host arrays are numpy.

There is no CPU fallback: if the library is missing, importing the binding
raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libvcx.so")

OK, E_ARG, E_MESH, E_OOM, E_HIP, E_UNSTABLE, E_BUSY, E_STATE = 0, -1, -2, -3, -4, -5, -6, -7
MODEL_GAS, MODEL_DRIFT_DIFFUSION, MODEL_NAVIER_STOKES = 0, 1, 2
FLUX_HLLC, FLUX_ROE = 0, 1
FLUX_LLW, FLUX_SG = 0, 2   # drift-diffusion schemes
LIM_FIRST_ORDER, LIM_MINMOD, LIM_VANLEER, LIM_SWEBY, LIM_NONE = 0, 1, 2, 3, 4
PREC_FP64, PREC_MIXED = 0, 1
MAX_SPECIES = 16

# every symbol declared in include/vcx.h
EXPORTS = (
    "vcx_mesh_create", "vcx_mesh_create_tiled", "vcx_mesh_destroy", "vcx_mesh_info", "vcx_mesh_geometry",
    "vcx_mesh_preprocess", "vcx_solver_create", "vcx_solver_destroy", "vcx_solver_nvar",
    "vcx_state_upload", "vcx_state_upload_primitive", "vcx_state_download", "vcx_state_set_time", "vcx_gradient",
    "vcx_residual", "vcx_timestep", "vcx_step", "vcx_steps_done", "vcx_state_time", "vcx_solve_batch",
    "vcx_solve_batch_eager", "vcx_solver_footprint", "vcx_server_create", "vcx_server_submit",
    "vcx_server_poll", "vcx_server_wait", "vcx_server_stats", "vcx_server_destroy",
    "vcx_conservation_sums", "vcx_profile_enable", "vcx_profile_query", "vcx_last_error",
    "vcx_solver_set_field", "vcx_poisson_create", "vcx_poisson_destroy", "vcx_poisson_solve",
    "vcx_poisson_field", "vcx_poisson_field_add", "vcx_poisson_info", "vcx_solver_charge",
    "vcx_mesh_create_axisymmetric", "vcx_mesh_create_axisymmetric_nv", "vcx_residual_noalloc",
    "vcx_noalloc_scratch_bytes",
)


class VcxError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__(f"{what} failed ({code}): {msg}")
        self.code = code


class Physics(C.Structure):
    _fields_ = [("model", C.c_int32), ("flux", C.c_int32), ("limiter", C.c_int32),
                ("rk_stages", C.c_int32), ("nspecies", C.c_int32), ("closure", C.c_int32),
                ("precision", C.c_int32), ("predictor", C.c_int32),
                ("beta", C.c_double), ("cfl", C.c_double), ("fourier", C.c_double),
                ("gamma", C.c_double), ("entropy_fix", C.c_double),
                ("z", C.c_double * MAX_SPECIES), ("mu", C.c_double * MAX_SPECIES),
                ("D", C.c_double * MAX_SPECIES),
                ("Wk", C.c_double * MAX_SPECIES), ("cpa", C.c_double * MAX_SPECIES),
                ("cpb", C.c_double * MAX_SPECIES), ("cpc", C.c_double * MAX_SPECIES),
                ("Sc", C.c_double * MAX_SPECIES), ("mu_ref", C.c_double), ("T_ref", C.c_double),
                ("Pr", C.c_double), ("diel", C.c_double)]


def physics(model=MODEL_GAS, flux=FLUX_HLLC, limiter=LIM_MINMOD, rk_stages=2, nspecies=0,
            closure=True, precision=PREC_FP64, beta=1.0, cfl=0.5, fourier=0.25, gamma=1.4,
            entropy_fix=0.1, z=(), mu=(), D=(), mixture=None, diel=0.0, predictor=0) -> Physics:
    p = Physics()
    p.model, p.flux, p.limiter, p.rk_stages = model, flux, limiter, rk_stages
    p.nspecies, p.closure, p.precision = nspecies, int(closure), precision
    p.predictor = int(predictor)
    p.beta, p.cfl, p.fourier, p.gamma, p.entropy_fix = beta, cfl, fourier, gamma, entropy_fix
    p.diel = diel
    for k, (a, b, c) in enumerate(zip(z, mu, D)):
        p.z[k], p.mu[k], p.D[k] = a, b, c
    if mixture is not None:
        for k in range(mixture.n):
            p.Wk[k], p.cpa[k], p.cpb[k] = mixture.W[k], mixture.cp_a[k], mixture.cp_b[k]
            p.cpc[k], p.Sc[k] = mixture.cp_c[k], mixture.Sc[k]
        p.mu_ref, p.T_ref, p.Pr = mixture.mu_ref, mixture.T_ref, mixture.Pr
    return p


_lib = None


def lib():
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2201_01291_amd.build`")
        # PyTorch, where installed, loads its own copy of the HIP runtime by
        # path; loaded first, it is the copy the library binds to (a second
        # copy loaded after the library's would hold the device, and the
        # library's first call would find none)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, dp, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)
        L.vcx_mesh_create.argtypes = [C.c_int, C.c_int64, dp, C.c_int64, C.c_int, i64p, dp, vp,
                                      C.POINTER(vp)]
        L.vcx_mesh_create_tiled.argtypes = [C.c_int, C.c_int64, dp, C.c_int64, C.c_int, i64p, dp,
                                            C.c_int, C.c_int, vp, C.POINTER(vp)]
        L.vcx_mesh_destroy.argtypes = [vp]
        L.vcx_mesh_info.argtypes = [vp, i64p]
        L.vcx_mesh_geometry.argtypes = [vp, dp, dp]
        L.vcx_mesh_preprocess.argtypes = [C.c_int, C.c_int64, dp, C.c_int64, C.c_int, i64p, dp,
                                          i64p]
        L.vcx_solver_create.argtypes = [vp, C.POINTER(Physics), dp, C.POINTER(vp)]
        L.vcx_solver_destroy.argtypes = [vp]
        L.vcx_solver_nvar.argtypes = [vp]
        L.vcx_solver_nvar.restype = C.c_int
        L.vcx_state_upload.argtypes = [vp, vp, C.c_int]
        L.vcx_state_upload_primitive.argtypes = [vp, vp, C.c_int]
        L.vcx_state_download.argtypes = [vp, vp, C.c_int]
        L.vcx_state_set_time.argtypes = [vp, C.c_double]
        L.vcx_gradient.argtypes = [vp, vp, C.c_int]
        L.vcx_residual.argtypes = [vp, C.c_double, vp, C.c_int]
        L.vcx_timestep.argtypes = [vp, dp]
        L.vcx_step.argtypes = [vp, C.c_int, C.c_double, dp, dp]
        L.vcx_steps_done.argtypes = [vp]
        L.vcx_steps_done.restype = C.c_int64
        L.vcx_state_time.argtypes = [vp, dp, dp]
        L.vcx_solve_batch.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(C.c_int), dp]
        L.vcx_solve_batch_eager.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(C.c_int), dp]
        L.vcx_solver_footprint.argtypes = [vp, C.POINTER(Physics), C.POINTER(C.c_size_t)]
        L.vcx_server_create.argtypes = [C.c_size_t, C.c_int, C.c_int, C.c_int, C.POINTER(vp)]
        L.vcx_server_submit.argtypes = [vp, vp, C.POINTER(Physics), dp, dp, C.c_int, C.c_double,
                                        i64p]
        L.vcx_server_poll.argtypes = [vp, C.c_int64, C.POINTER(C.c_int), C.POINTER(C.c_int), dp, dp]
        L.vcx_server_wait.argtypes = [vp, C.c_int64, C.c_double, C.POINTER(C.c_int)]
        L.vcx_server_stats.argtypes = [vp, dp]
        L.vcx_server_destroy.argtypes = [vp]
        L.vcx_conservation_sums.argtypes = [vp, dp]
        L.vcx_profile_enable.argtypes = [vp, C.c_int]
        L.vcx_profile_query.argtypes = [vp, C.c_char_p, i64p, dp]
        L.vcx_last_error.restype = C.c_char_p
        L.vcx_solver_set_field.argtypes = [vp, vp, C.c_int]
        L.vcx_mesh_create_axisymmetric.argtypes = [C.c_int64, dp, C.c_int64, i64p, C.c_double, C.c_int,
                                                   C.c_int, vp, C.POINTER(vp)]
        L.vcx_mesh_create_axisymmetric_nv.argtypes = [C.c_int64, dp, C.c_int64, C.c_int, i64p, C.c_double,
                                                      C.c_int, C.c_int, vp, C.POINTER(vp)]
        L.vcx_poisson_create.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(vp)]
        L.vcx_poisson_destroy.argtypes = [vp]
        L.vcx_poisson_solve.argtypes = [vp, vp, vp, vp, vp, C.c_int, C.c_double, C.c_int,
                                        C.POINTER(C.c_int), dp]
        L.vcx_poisson_field.argtypes = [vp, vp, vp, C.c_int]
        L.vcx_poisson_field_add.argtypes = [vp, vp, vp, vp, C.c_int]
        L.vcx_poisson_info.argtypes = [vp, i64p]
        L.vcx_solver_charge.argtypes = [vp, vp, C.c_int]
        L.vcx_residual_noalloc.argtypes = [vp, C.POINTER(Physics), vp, vp, C.c_double, vp]
        L.vcx_noalloc_scratch_bytes.argtypes = []
        L.vcx_noalloc_scratch_bytes.restype = C.c_size_t
        for name in EXPORTS:
            if name not in ("vcx_solver_nvar", "vcx_steps_done", "vcx_last_error",
                            "vcx_noalloc_scratch_bytes"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(code, what):
    if code != OK:
        raise VcxError(code, what, lib().vcx_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _is_device_tensor(x) -> bool:
    return hasattr(x, "is_cuda") and bool(getattr(x, "is_cuda"))


def _ptr(x):
    """(pointer, is_device) of a numpy array or a torch tensor."""
    if _is_device_tensor(x):
        import torch
        if x.dtype != torch.float64 or not x.is_contiguous():
            raise ValueError("device arrays must be contiguous float64 tensors")
        return C.c_void_p(x.data_ptr()), 1
    if not (isinstance(x, np.ndarray) and x.dtype == np.float64 and x.flags["C_CONTIGUOUS"]):
        raise ValueError("host arrays must be C-contiguous float64 numpy arrays")
    return C.c_void_p(x.ctypes.data), 0


def current_stream():
    """Handle of PyTorch's current HIP stream (0 if torch has no GPU)."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return 0


def mesh_preprocess(mesh) -> dict:
    """Host-only dry run of the library's mesh preprocessing."""
    xyz, cells = _f64(mesh.xyz), np.ascontiguousarray(mesh.cells, dtype=np.int64)
    per = None if mesh.period is None else _f64(mesh.period)
    st = np.zeros(10, dtype=np.int64)
    _check(lib().vcx_mesh_preprocess(mesh.ndim, mesh.nnodes, _dptr(xyz), mesh.ncells, mesh.nv,
                                     cells.ctypes.data_as(C.POINTER(C.c_int64)),
                                     _dptr(per) if per is not None else None,
                                     st.ctypes.data_as(C.POINTER(C.c_int64))),
           "vcx_mesh_preprocess")
    out = dict(zip(("nnodes", "ncells", "nfaces", "ntiles", "nslots", "nbnd", "max_tile_cells",
                    "max_tile_nodes"), map(int, st[:8])))
    out["vol_cells"] = float(st[8:9].view(np.float64)[0])
    out["vol_nodes"] = float(st[9:10].view(np.float64)[0])
    return out


class Mesh:
    def __init__(self, mesh, stream=None, tile_cells: int = 0, tile_nodes: int = 0,
                 axisymmetric: bool = False):
        """axisymmetric: mesh of the (x, r) half-plane (second coordinate the
        radius; only x may be periodic)."""
        L = lib()
        self.src = mesh
        self.ndim, self.nnodes, self.ncells = mesh.ndim, mesh.nnodes, mesh.ncells
        self.stream = current_stream() if stream is None else stream
        xyz, cells = _f64(mesh.xyz), np.ascontiguousarray(mesh.cells, dtype=np.int64)
        per = None if mesh.period is None else _f64(mesh.period)
        h = C.c_void_p()
        cp = cells.ctypes.data_as(C.POINTER(C.c_int64))
        if axisymmetric:
            px = float(per[0]) if per is not None else 0.0
            _check(L.vcx_mesh_create_axisymmetric_nv(mesh.nnodes, _dptr(xyz), mesh.ncells, mesh.nv, cp, px,
                                                     int(tile_cells), int(tile_nodes),
                                                     C.c_void_p(self.stream), C.byref(h)),
                   "vcx_mesh_create_axisymmetric_nv")
        else:
            _check(L.vcx_mesh_create_tiled(mesh.ndim, mesh.nnodes, _dptr(xyz), mesh.ncells, mesh.nv, cp,
                                           _dptr(per) if per is not None else None, int(tile_cells),
                                           int(tile_nodes), C.c_void_p(self.stream), C.byref(h)),
                   "vcx_mesh_create_tiled")
        self.h = h

    def info(self) -> dict:
        out = np.zeros(8, dtype=np.int64)
        _check(lib().vcx_mesh_info(self.h, out.ctypes.data_as(C.POINTER(C.c_int64))), "vcx_mesh_info")
        return dict(zip(("nnodes", "ncells", "nfaces", "ntiles", "nslots", "nbnd",
                         "max_tile_cells", "max_tile_nodes"), map(int, out)))

    def geometry(self):
        Vn = np.zeros(self.nnodes)
        Sb = np.zeros((self.ndim, self.nnodes))
        _check(lib().vcx_mesh_geometry(self.h, _dptr(Vn), _dptr(Sb)), "vcx_mesh_geometry")
        return Vn, Sb

    def close(self):
        if getattr(self, "h", None):
            lib().vcx_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    def __init__(self, mesh: Mesh, phys: Physics, E=None):
        self.mesh, self.phys = mesh, phys
        Ec = None if E is None else _f64(E)
        h = C.c_void_p()
        _check(lib().vcx_solver_create(mesh.h, C.byref(phys), _dptr(Ec) if Ec is not None else None,
                                       C.byref(h)), "vcx_solver_create")
        self.h = h
        self.nvar = lib().vcx_solver_nvar(h)
        self.nr = self.nvar if phys.model == MODEL_DRIFT_DIFFUSION else self.nvar + 1

    def upload(self, U):
        if not _is_device_tensor(U):
            U = _f64(U)
        p, dev = _ptr(U)
        _check(lib().vcx_state_upload(self.h, p, dev), "vcx_state_upload")

    def charge(self, out=None):
        """Space charge (e/eps0) sum_s z_s n_s of a drift-diffusion state
        (vcx_solver_charge), host array or into a device tensor."""
        if out is None:
            out = np.zeros(self.mesh.nnodes)
        p, dev = _ptr(out)
        _check(lib().vcx_solver_charge(self.h, p, dev), "vcx_solver_charge")
        return out

    def upload_primitive(self, P):
        """State from primitive rows (gas: rho, u, p, Y; Navier-Stokes: rho,
        u, T, Y), converted by the library's equation of state."""
        if not _is_device_tensor(P):
            P = _f64(P)
        p, dev = _ptr(P)
        _check(lib().vcx_state_upload_primitive(self.h, p, dev), "vcx_state_upload_primitive")

    def set_field(self, E):
        """Replace the drift-diffusion field E [ndim][nnodes] (host or device)."""
        if not _is_device_tensor(E):
            E = _f64(E)
        p, dev = _ptr(E)
        _check(lib().vcx_solver_set_field(self.h, p, dev), "vcx_solver_set_field")

    def set_time(self, t: float):
        _check(lib().vcx_state_set_time(self.h, float(t)), "vcx_state_set_time")

    def download(self, out=None):
        if out is None:
            out = np.zeros((self.nvar, self.mesh.nnodes))
        p, dev = _ptr(out)
        _check(lib().vcx_state_download(self.h, p, dev), "vcx_state_download")
        return out

    def gradient(self, out=None):
        if out is None:
            out = np.zeros((self.nr, self.mesh.ndim, self.mesh.nnodes))
        p, dev = _ptr(out)
        _check(lib().vcx_gradient(self.h, p, dev), "vcx_gradient")
        return out

    def residual(self, dt: float = 0.0, out=None):
        if out is None:
            out = np.zeros((self.nvar, self.mesh.nnodes))
        p, dev = _ptr(out)
        _check(lib().vcx_residual(self.h, float(dt), p, dev), "vcx_residual")
        return out

    def timestep(self) -> float:
        dt = C.c_double()
        _check(lib().vcx_timestep(self.h, C.byref(dt)), "vcx_timestep")
        return dt.value

    def step(self, nsteps: int, t_end: float = 0.0):
        t, dl = C.c_double(), C.c_double()
        _check(lib().vcx_step(self.h, int(nsteps), float(t_end), C.byref(t), C.byref(dl)), "vcx_step")
        return t.value, dl.value

    def steps_done(self) -> int:
        return int(lib().vcx_steps_done(self.h))

    def time(self):
        """(t, dt_last) after the last step / batch call."""
        t, d = C.c_double(), C.c_double()
        _check(lib().vcx_state_time(self.h, C.byref(t), C.byref(d)), "vcx_state_time")
        return t.value, d.value

    def sums(self):
        out = np.zeros(self.nvar)
        _check(lib().vcx_conservation_sums(self.h, _dptr(out)), "vcx_conservation_sums")
        return out

    def profile(self, enable: bool = True):
        _check(lib().vcx_profile_enable(self.h, int(enable)), "vcx_profile_enable")

    def profile_query(self, kernel: str):
        n, ms = C.c_int64(), C.c_double()
        _check(lib().vcx_profile_query(self.h, kernel.encode(), C.byref(n), C.byref(ms)),
               "vcx_profile_query")
        return n.value, ms.value

    def close(self):
        if getattr(self, "h", None):
            lib().vcx_solver_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def footprint(mesh: Mesh, phys: Physics) -> int:
    """Device bytes a solver of this physics on this mesh allocates."""
    b = C.c_size_t()
    _check(lib().vcx_solver_footprint(mesh.h, C.byref(phys), C.byref(b)), "vcx_solver_footprint")
    return int(b.value)


SERVER_STATS = ("submitted", "completed", "failed", "queued", "running", "member_steps", "chunks",
                "mean_running", "latency_p50_ms", "latency_p99_ms", "step_p50_ms", "step_p99_ms",
                "resident_bytes", "peak_resident_bytes", "peak_running", "device_error",
                "idle_bytes")


class Server:
    """Continuous-batching request server (scheduler thread in the library)."""

    def __init__(self, hbm_budget: int, max_slots: int = 64, chunk_steps: int = 16, graphs=True):
        h = C.c_void_p()
        _check(lib().vcx_server_create(int(hbm_budget), int(max_slots), int(chunk_steps),
                                       int(bool(graphs)), C.byref(h)), "vcx_server_create")
        self.h = h
        self._req = {}    # id -> (mesh, nvar): meshes stay alive while their requests run

    def submit(self, mesh: Mesh, phys: Physics, U0, E=None, nsteps: int = 1, t_end: float = 0.0):
        U0 = _f64(U0)
        Ec = None if E is None else _f64(E)
        rid = C.c_int64()
        _check(lib().vcx_server_submit(self.h, mesh.h, C.byref(phys), _dptr(U0),
                                       _dptr(Ec) if Ec is not None else None, int(nsteps),
                                       float(t_end), C.byref(rid)), "vcx_server_submit")
        self._req[rid.value] = (mesh, U0.shape)
        return rid.value

    def poll(self, rid: int, take: bool = True):
        """(done, status, U or None, t).  With take, a finished request's
        state is returned and the request is forgotten."""
        done, st, t = C.c_int(), C.c_int(), C.c_double()
        mesh, shape = self._req.get(rid, (None, None))
        U = np.zeros(shape) if take and shape is not None else None
        _check(lib().vcx_server_poll(self.h, int(rid), C.byref(done), C.byref(st),
                                     _dptr(U) if U is not None else None, C.byref(t)),
               "vcx_server_poll")
        if not done.value:
            return False, None, None, None
        if take:
            del self._req[rid]
        return True, st.value, U, t.value

    def wait(self, rid: int, timeout: float = -1.0) -> bool:
        done = C.c_int()
        _check(lib().vcx_server_wait(self.h, int(rid), float(timeout), C.byref(done)),
               "vcx_server_wait")
        return bool(done.value)

    def stats(self) -> dict:
        out = np.zeros(17)
        _check(lib().vcx_server_stats(self.h, _dptr(out)), "vcx_server_stats")
        return dict(zip(SERVER_STATS, out.tolist()))

    def close(self):
        if getattr(self, "h", None):
            _check(lib().vcx_server_destroy(self.h), "vcx_server_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Poisson:
    """Poisson operator of a mesh: potential of -lap phi = q (q = rho/eps0)
    and the field E = -grad phi (vcx_poisson_*)."""

    def __init__(self, mesh: Mesh, dirichlet=None):
        self.mesh = mesh
        h = C.c_void_p()
        dm = None
        if dirichlet is not None:
            dm = np.ascontiguousarray(np.asarray(dirichlet) != 0, dtype=np.int32)
        _check(lib().vcx_poisson_create(mesh.h, dm.ctypes.data_as(C.POINTER(C.c_int32))
                                        if dm is not None else None, C.byref(h)), "vcx_poisson_create")
        self.h = h

    def solve(self, q, phiD=None, En=None, phi0=None, tol: float = 1e-12, max_iter: int = 10000,
              out=None):
        """Returns (phi, iterations, relative residual); all arrays host or all
        device tensors."""
        dev = _is_device_tensor(q)
        n = self.mesh.nnodes

        def arr(x):
            if x is None:
                return None, None
            if dev:
                return x, C.c_void_p(x.data_ptr())
            a = _f64(x)
            return a, C.c_void_p(a.ctypes.data)

        qa, qp = arr(q)
        Da, Dp = arr(phiD)
        Ea, Ep = arr(En)
        if out is None:
            if dev:
                import torch
                out = torch.zeros(n, dtype=torch.float64, device=q.device)
            else:
                out = np.zeros(n)
        if phi0 is not None:
            if dev:
                out.copy_(phi0)
            else:
                out[:] = phi0
        op = C.c_void_p(out.data_ptr()) if dev else C.c_void_p(out.ctypes.data)
        it, rel = C.c_int(), C.c_double()
        _check(lib().vcx_poisson_solve(self.h, qp, Dp, Ep, op, int(dev), float(tol), int(max_iter),
                                       C.byref(it), C.byref(rel)), "vcx_poisson_solve")
        return out, it.value, rel.value

    def field(self, phi, out=None, background=None):
        """E = -grad phi, or E = background - grad phi (vcx_poisson_field_add)."""
        dev = _is_device_tensor(phi)
        n, nd = self.mesh.nnodes, self.mesh.ndim
        if out is None:
            if dev:
                import torch
                out = torch.zeros((nd, n), dtype=torch.float64, device=phi.device)
            else:
                out = np.zeros((nd, n))
        if dev:
            pp, op = C.c_void_p(phi.data_ptr()), C.c_void_p(out.data_ptr())
            bp = C.c_void_p(background.data_ptr()) if background is not None else None
        else:
            phi = _f64(phi)
            pp, op = C.c_void_p(phi.ctypes.data), C.c_void_p(out.ctypes.data)
            if background is not None:
                background = _f64(background)
            bp = C.c_void_p(background.ctypes.data) if background is not None else None
        if background is None:
            _check(lib().vcx_poisson_field(self.h, pp, op, int(dev)), "vcx_poisson_field")
        else:
            _check(lib().vcx_poisson_field_add(self.h, pp, bp, op, int(dev)), "vcx_poisson_field_add")
        return out

    def info(self) -> dict:
        out = np.zeros(4, dtype=np.int64)
        _check(lib().vcx_poisson_info(self.h, out.ctypes.data_as(C.POINTER(C.c_int64))), "vcx_poisson_info")
        return dict(rows=int(out[0]), nnz=int(out[1]), coarse=int(out[2]),
                    solver="BiCGStab" if out[3] else "CG")

    def close(self):
        if getattr(self, "h", None):
            lib().vcx_poisson_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def residual_noalloc(mesh: "Mesh", phys: Physics, U, E=None, dt: float = 0.0, out=None):
    """vcx_residual_noalloc: residual of the device state U (torch tensor,
    [nvar][nnodes]) without a solver and without device allocation in the
    library; E a device [ndim][nnodes] field for drift-diffusion; out a
    device tensor like U (allocated here by torch when None)."""
    import torch
    if out is None:
        out = torch.empty_like(U)
    ep = C.c_void_p(E.data_ptr()) if E is not None else None
    _check(lib().vcx_residual_noalloc(mesh.h, C.byref(phys), C.c_void_p(U.data_ptr()), ep, float(dt),
                                      C.c_void_p(out.data_ptr())), "vcx_residual_noalloc")
    return out


def noalloc_scratch_bytes() -> int:
    return int(lib().vcx_noalloc_scratch_bytes())


def solve_batch(solvers, nsteps, t_end=None, graphs=True):
    """Advance independent solvers together (batched kernels); nsteps and
    t_end are per solver (t_end None or <= 0: no end time)."""
    n = len(solvers)
    if np.isscalar(nsteps):
        nsteps = [nsteps] * n
    if t_end is None:
        t_end = [0.0] * n
    elif np.isscalar(t_end):
        t_end = [t_end] * n
    hs = (C.c_void_p * n)(*[s.h for s in solvers])
    ns = (C.c_int * n)(*[int(x) for x in nsteps])
    te = (C.c_double * n)(*[float(x) for x in t_end])
    fn = lib().vcx_solve_batch if graphs else lib().vcx_solve_batch_eager
    _check(fn(hs, n, ns, te), "vcx_solve_batch")
