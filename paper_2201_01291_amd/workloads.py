"""Seeded synthetic meshes and initial states.

This module produces inputs only: node coordinates, simplex connectivity and
initial nodal states.  It contains none of the finite-volume arithmetic (no
normals, volumes, gradients, fluxes or time steps), so both the HIP library
and the CPU oracle can be fed from it without sharing any of the method.

Conventions shared by every generator
-------------------------------------
* coordinates ``xyz``: float64 array ``[ndim][nnodes]``;
* connectivity ``cells``: int64 array ``[nv][ncells]`` (``nv`` = 3 triangles,
  4 tetrahedra), vertices listed counter-clockwise / positively oriented on
  the unjittered lattice;
* ``period``: float64 ``[ndim]`` for a fully periodic box, else ``None``.
  Periodic meshes store each node once; cells that straddle the seam refer to
  the wrapped node indices.
* every random draw comes from ``numpy.random.default_rng(seed)`` (PCG64).

The workload recipes (domain sizes, jitter, blob counts) are the synthetic
stand-ins for the paper's test problems: the shock tube (Sec. "One-dimensional
shock tube"), drift-diffusion streamer meshes (Sec. "Bagheri benchmark") and
3D/multi-species transport, which the paper runs but does not benchmark.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    xyz: np.ndarray          # [ndim][nnodes] float64
    cells: np.ndarray        # [nv][ncells] int64
    period: np.ndarray | None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def ndim(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nnodes(self) -> int:
        return int(self.xyz.shape[1])

    @property
    def nv(self) -> int:
        return int(self.cells.shape[0])

    @property
    def ncells(self) -> int:
        return int(self.cells.shape[1])

    @property
    def nfaces(self) -> int:
        """Cell-edges: 3 per triangle, 4 per quadrilateral, 6 per tetrahedron."""
        return self.ncells * {3: 3, 4: 4 if self.ndim == 2 else 6}[self.nv]


# ---------------------------------------------------------------------------
# meshes
# ---------------------------------------------------------------------------

def tri_rect_mesh(nx: int, ny: int, lx: float = 1.0, ly: float = 1.0, *,
                  jitter: float = 0.0, seed: int = 0, periodic=False,
                  origin=(0.0, 0.0)) -> Mesh:
    """``nx`` x ``ny`` quads on ``[0,lx]x[0,ly]``, each split in two triangles
    along its (0,0)->(1,1) diagonal.

    ``periodic`` is a bool (both axes) or a pair of bools (per axis); the
    returned ``period`` holds the box length for periodic axes and 0 for open
    ones.  ``jitter`` moves each node by U(-jitter*h, jitter*h) per axis
    (h = spacing of that axis); nodes on an open boundary do not move
    normal to it, so the boundary stays straight.
    """
    if nx < 1 or ny < 1:
        raise ValueError("need at least one quad per direction")
    perx, pery = (periodic, periodic) if isinstance(periodic, bool) else tuple(periodic)
    if (perx and nx < 3) or (pery and ny < 3):
        raise ValueError("periodic axes need >= 3 quads")
    hx, hy = lx / nx, ly / ny
    px = nx if perx else nx + 1
    py = ny if pery else ny + 1
    I, J = np.meshgrid(np.arange(px), np.arange(py), indexing="ij")
    x = origin[0] + I.astype(np.float64) * hx
    y = origin[1] + J.astype(np.float64) * hy
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        dx = rng.uniform(-jitter * hx, jitter * hx, size=x.shape)
        dy = rng.uniform(-jitter * hy, jitter * hy, size=y.shape)
        if not perx:
            dx = np.where((I > 0) & (I < nx), dx, 0.0)
        if not pery:
            dy = np.where((J > 0) & (J < ny), dy, 0.0)
        x = x + dx
        y = y + dy
        if perx:
            x = origin[0] + np.mod(x - origin[0], lx)
        if pery:
            y = origin[1] + np.mod(y - origin[1], ly)

    def nid(i, j):
        return (i % px) * py + (j % py)

    qi, qj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    qi, qj = qi.ravel(), qj.ravel()
    n00, n10 = nid(qi, qj), nid(qi + 1, qj)
    n01, n11 = nid(qi, qj + 1), nid(qi + 1, qj + 1)
    ta = np.stack([n00, n10, n11])
    tb = np.stack([n00, n11, n01])
    cells = np.empty((3, 2 * qi.size), dtype=np.int64)
    cells[:, 0::2] = ta
    cells[:, 1::2] = tb
    xyz = np.stack([x.ravel(), y.ravel()]).astype(np.float64)
    period = np.array([lx if perx else 0.0, ly if pery else 0.0]) if (perx or pery) else None
    return Mesh(xyz, cells, period, name=f"tri{nx}x{ny}",
                meta=dict(nx=nx, ny=ny, lx=lx, ly=ly, jitter=jitter, seed=seed))


def quad_rect_mesh(nx: int, ny: int, lx: float = 1.0, ly: float = 1.0, *,
                   jitter: float = 0.0, seed: int = 0, periodic=False,
                   origin=(0.0, 0.0)) -> Mesh:
    """``nx`` x ``ny`` quadrilaterals on ``[0,lx]x[0,ly]``, vertices in
    counter-clockwise order; node layout, ``periodic`` and ``jitter`` as
    :func:`tri_rect_mesh` (the same seed moves the nodes the same way)."""
    t = tri_rect_mesh(nx, ny, lx, ly, jitter=jitter, seed=seed, periodic=periodic, origin=origin)
    perx, pery = (periodic, periodic) if isinstance(periodic, bool) else tuple(periodic)
    px = nx if perx else nx + 1
    py = ny if pery else ny + 1

    def nid(i, j):
        return (i % px) * py + (j % py)

    qi, qj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    qi, qj = qi.ravel(), qj.ravel()
    cells = np.stack([nid(qi, qj), nid(qi + 1, qj), nid(qi + 1, qj + 1), nid(qi, qj + 1)]).astype(np.int64)
    return Mesh(t.xyz, cells, t.period, name=f"quad{nx}x{ny}", meta=dict(t.meta))


_KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def kuhn_tet_mesh(nx: int, ny: int, nz: int, lx: float = 1.0, ly: float = 1.0,
                  lz: float = 1.0, *, jitter: float = 0.0, seed: int = 0,
                  periodic: bool = True) -> Mesh:
    """Cube lattice, each cube split into the 6 Kuhn tetrahedra
    (corner 000 -> +e_a -> +e_a+e_b -> corner 111 for every axis order a,b,c).
    The split is conforming across cubes and across the periodic seam."""
    if min(nx, ny, nz) < 1:
        raise ValueError("need at least one cube per direction")
    if periodic and min(nx, ny, nz) < 3:
        raise ValueError("periodic meshes need >= 3 cubes per direction")
    n = (nx, ny, nz)
    h = (lx / nx, ly / ny, lz / nz)
    L = (lx, ly, lz)
    p = tuple(k if periodic else k + 1 for k in n)
    I, J, K = np.meshgrid(np.arange(p[0]), np.arange(p[1]), np.arange(p[2]), indexing="ij")
    coords = [I.astype(np.float64) * h[0], J.astype(np.float64) * h[1], K.astype(np.float64) * h[2]]
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        deltas = [rng.uniform(-jitter * h[a], jitter * h[a], size=I.shape) for a in range(3)]
        if not periodic:
            interior = ((I > 0) & (I < nx) & (J > 0) & (J < ny) & (K > 0) & (K < nz))
            deltas = [np.where(interior, d, 0.0) for d in deltas]
        coords = [c + d for c, d in zip(coords, deltas)]
        if periodic:
            coords = [np.mod(c, L[a]) for a, c in enumerate(coords)]

    def nid(i, j, k):
        if periodic:
            return ((i % p[0]) * p[1] + (j % p[1])) * p[2] + (k % p[2])
        return (i * p[1] + j) * p[2] + k

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    base = np.stack([ci.ravel(), cj.ravel(), ck.ravel()])
    tets = []
    for perm in _KUHN_PERMS:
        verts = [base.copy()]
        cur = base.copy()
        for a in perm:
            cur = cur.copy()
            cur[a] += 1
            verts.append(cur)
        tets.append(np.stack([nid(*v) for v in verts]))
    # interleave the 6 tets of each cube so a cube's tets are consecutive
    cells = np.stack(tets, axis=2).reshape(4, -1).astype(np.int64)
    xyz = np.stack([c.ravel() for c in coords]).astype(np.float64)
    period = np.array(L, dtype=np.float64) if periodic else None
    return Mesh(xyz, cells, period, name=f"kuhn{nx}x{ny}x{nz}",
                meta=dict(nx=nx, ny=ny, nz=nz, L=L, jitter=jitter, seed=seed))


def fix_orientation_free(mesh: Mesh) -> Mesh:
    """Return the mesh with the vertex order of every odd cell reversed.

    Used by tests to check that consumers do not rely on a particular vertex
    orientation.  (Pure relabelling, no geometry.)"""
    cells = mesh.cells.copy()
    odd = np.arange(mesh.ncells) % 2 == 1
    cells[[1, 2]] = np.where(odd, cells[[2, 1]], cells[[1, 2]])
    return Mesh(mesh.xyz, cells, mesh.period, mesh.name + "-flip", dict(mesh.meta))


def shuffled(mesh: Mesh, seed: int = 0):
    """Randomly renumber nodes and cells; returns (mesh, node_perm) where
    ``node_perm[new] = old``."""
    rng = np.random.default_rng(seed)
    nperm = rng.permutation(mesh.nnodes)
    inv = np.empty_like(nperm)
    inv[nperm] = np.arange(mesh.nnodes)
    cperm = rng.permutation(mesh.ncells)
    cells = inv[mesh.cells[:, cperm]]
    return Mesh(mesh.xyz[:, nperm].copy(), cells, mesh.period, mesh.name + "-shuf",
                dict(mesh.meta)), nperm


# ---------------------------------------------------------------------------
# states
# ---------------------------------------------------------------------------

def _min_image(d: np.ndarray, L: float | None) -> np.ndarray:
    if L is None:
        return d
    return d - L * np.round(d / L)


def conserved_from_primitive(rho, vel, p, gamma, Y=None):
    """Conserved gas state [rho, rho*u_1..rho*u_nd, rho*E, rho*Y_1..] from
    primitives, ideal gas with constant gamma (input preparation only)."""
    vel = np.atleast_2d(vel)
    ke = 0.5 * rho * np.sum(vel * vel, axis=0)
    rows = [rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + ke]
    if Y is not None:
        rows += [rho * y for y in np.atleast_2d(Y)]
    return np.stack(rows).astype(np.float64)


def sod_state(mesh: Mesh, gamma: float = 1.4, x0: float = 0.5,
              left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1)) -> np.ndarray:
    """Shock-tube initial data (rho, u, p) split at x = x0, zero transverse velocity."""
    x = mesh.xyz[0]
    L = x < x0
    rho = np.where(L, left[0], right[0])
    u = np.where(L, left[1], right[1])
    p = np.where(L, left[2], right[2])
    vel = np.zeros((mesh.ndim, mesh.nnodes))
    vel[0] = u
    return conserved_from_primitive(rho, vel, p, gamma)


def euler_blob_state(mesh: Mesh, *, nblobs: int = 8, amp: float = 0.1, sigma: float = 0.08,
                     mach: float = 0.3, gamma: float = 1.4, seed: int = 1,
                     nspecies: int = 0) -> np.ndarray:
    """Uniform flow at the given Mach number along x (rho0 = 1, p0 = 1/gamma so
    the sound speed is 1) with ``nblobs`` seeded Gaussian bumps multiplying
    rho and p by (1 + amp*exp(-|x-c|^2/sigma^2)); periodic minimum image.
    Optional passive species get seeded smooth mass fractions summing to 1."""
    rng = np.random.default_rng(seed)
    nd = mesh.ndim
    lengths = mesh.period if mesh.period is not None else (mesh.xyz.max(1) - mesh.xyz.min(1))
    lo = mesh.xyz.min(1)
    centres = lo[:, None] + rng.uniform(0.0, 1.0, size=(nd, nblobs)) * np.asarray(lengths)[:, None]
    bump = np.zeros(mesh.nnodes)
    for b in range(nblobs):
        r2 = np.zeros(mesh.nnodes)
        for a in range(nd):
            L = None if mesh.period is None else float(mesh.period[a])
            d = _min_image(mesh.xyz[a] - centres[a, b], L)
            r2 += d * d
        bump += amp * np.exp(-r2 / (sigma * sigma))
    rho = 1.0 * (1.0 + bump)
    p = (1.0 / gamma) * (1.0 + bump)
    vel = np.zeros((nd, mesh.nnodes))
    vel[0] = mach
    Y = None
    if nspecies > 0:
        w = rng.uniform(0.5, 1.5, size=(nspecies, nblobs))
        raw = np.ones((nspecies, mesh.nnodes))
        for b in range(nblobs):
            r2 = np.zeros(mesh.nnodes)
            for a in range(nd):
                L = None if mesh.period is None else float(mesh.period[a])
                d = _min_image(mesh.xyz[a] - centres[a, b], L)
                r2 += d * d
            raw += w[:, b:b + 1] * np.exp(-r2 / (4 * sigma * sigma))[None, :]
        Y = raw / raw.sum(0, keepdims=True)
    return conserved_from_primitive(rho, vel, p, gamma, Y)


def explosion_state(mesh: Mesh, *, centre=(1.0, 1.0), radius: float = 0.4,
                    inside=(1.0, 1.0), outside=(0.125, 0.1), width: float | None = None,
                    gamma: float = 1.4) -> np.ndarray:
    """Cylindrical (2D) or spherical (3D) explosion at rest (Sec.
    "Explosions", after Toro Ch. 17.1): density and pressure ``inside`` =
    (rho, p) within ``radius`` of ``centre`` and ``outside`` beyond it, blended
    by 0.5 (1 - tanh((r - radius)/width)) so the interface has no staircase;
    ``width`` defaults to one mean mesh spacing."""
    nd = mesh.ndim
    if width is None:
        ext = mesh.xyz.max(1) - mesh.xyz.min(1)
        width = float(np.prod(ext) / max(mesh.ncells, 1) * math.factorial(nd)) ** (1.0 / nd)
    r = np.sqrt(sum((mesh.xyz[a] - centre[a]) ** 2 for a in range(nd)))
    w = 0.5 * (1.0 - np.tanh((r - radius) / width))
    rho = outside[0] + (inside[0] - outside[0]) * w
    p = outside[1] + (inside[1] - outside[1]) * w
    return conserved_from_primitive(rho, np.zeros((nd, mesh.nnodes)), p, gamma)


# Velocity directions of the four quadrant states of the paper's 2D Riemann
# problems (figure of the four cases; quadrants 1..4 = top-left, top-right,
# bottom-right, bottom-left), as signs of (u_x, u_y).
QUADRANT_SIGNS = {
    1: ((+1, +1), (+1, -1), (-1, -1), (-1, +1)),   # clockwise turn (mixing interfaces)
    2: ((-1, +1), (-1, -1), (+1, -1), (+1, +1)),   # shock / expansion diagonals
    3: ((-1, +1), (+1, +1), (+1, -1), (-1, -1)),   # every state moving outward
    4: ((+1, -1), (-1, -1), (-1, +1), (+1, +1)),   # every state moving inward
}


def quadrant_state(mesh: Mesh, case: int, *, centre=(0.0, 0.0), rho=(2.0, 1.0, 3.0, 1.0),
                   p: float = 1.0, speeds=(0.75, 0.5), gamma: float = 1.4) -> np.ndarray:
    """Initial data of the paper's 2D Riemann problems (Sec. "2D Riemann
    problems"): four constant states in the quadrants around ``centre``,
    densities 2, 1, 3, 1 (quadrants 1..4), pressure 1 everywhere, velocity
    components of magnitude 0.75 (x) and 0.5 (y) with the signs of
    ``QUADRANT_SIGNS[case]``."""
    x, y = mesh.xyz[0] - centre[0], mesh.xyz[1] - centre[1]
    q = np.where(y >= 0, np.where(x < 0, 0, 1), np.where(x >= 0, 2, 3))
    sg = np.array(QUADRANT_SIGNS[case], dtype=np.float64)
    r = np.asarray(rho, dtype=np.float64)[q]
    vel = np.stack([speeds[0] * sg[q, 0], speeds[1] * sg[q, 1]])
    return conserved_from_primitive(r, vel, np.full(mesh.nnodes, p), gamma)


@dataclass
class DDSpecies:
    z: float      # charge sign (-1 electrons, +1 positive ions)
    mu: float     # mobility [m^2/(V s)]
    D: float      # diffusion coefficient [m^2/s]


def dd_fields(mesh: Mesh, *, seed: int = 2, peak: float = 1e18, sigma: float = 5e-4,
              nblobs: int = 4, e0: float = 1e6, bump_amp: float = 700.0,
              bump_sigma: float = 2e-3, nspecies: int = 2):
    """Drift-diffusion inputs: densities [nspecies][nnodes] made of ``nblobs``
    seeded Gaussians (same for every species) and the electric field
    E = -grad(phi) [ndim][nnodes] of phi = -e0*x + A*exp(-|x-xb|^2/sb^2)
    (periodic image sum), evaluated analytically at the nodes."""
    rng = np.random.default_rng(seed)
    nd = mesh.ndim
    lengths = mesh.period if mesh.period is not None else (mesh.xyz.max(1) - mesh.xyz.min(1))
    lo = mesh.xyz.min(1)
    centres = lo[:, None] + rng.uniform(0.0, 1.0, size=(nd, nblobs)) * np.asarray(lengths)[:, None]
    xb = lo + rng.uniform(0.0, 1.0, size=nd) * np.asarray(lengths)
    dens = np.zeros(mesh.nnodes)
    for b in range(nblobs):
        r2 = np.zeros(mesh.nnodes)
        for a in range(nd):
            L = None if mesh.period is None else float(mesh.period[a])
            d = _min_image(mesh.xyz[a] - centres[a, b], L)
            r2 += d * d
        dens += peak * np.exp(-r2 / (sigma * sigma))
    n = np.stack([dens.copy() for _ in range(nspecies)])
    E = np.zeros((nd, mesh.nnodes))
    E[0] = e0
    shifts = [(-1, 0, 1) if mesh.period is not None else (0,)] * nd
    for img in np.array(np.meshgrid(*shifts, indexing="ij")).reshape(nd, -1).T:
        d = np.stack([mesh.xyz[a] - xb[a] - (img[a] * lengths[a] if mesh.period is not None else 0.0)
                      for a in range(nd)])
        g = bump_amp * np.exp(-np.sum(d * d, axis=0) / (bump_sigma ** 2))
        # E = -grad(phi_bump) = A*exp(..)*2*d/sb^2
        E += g[None, :] * 2.0 * d / (bump_sigma ** 2)
    return n.astype(np.float64), E.astype(np.float64)


DD_STREAMER_SPECIES = (DDSpecies(z=-1.0, mu=0.04, D=0.1), DDSpecies(z=+1.0, mu=0.04, D=0.1))


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

def sod_tube(nx: int = 100, ny: int = 10) -> Mesh:
    """Shock tube: [0,1]x[0,0.1] with nx x ny quads split in two triangles,
    periodic across the tube (y) and open at both ends (x)."""
    return tri_rect_mesh(nx, ny, 1.0, 0.1, periodic=(False, True))


def dd_streamer_mesh(nx: int = 400, ny: int = 250, jitter: float = 0.2, seed: int = 7) -> Mesh:
    """Periodic [0,0.02]x[0,0.0125] m box (h = 50 um at 400x250), jittered
    triangles: 2*nx*ny cells, nx*ny nodes."""
    return tri_rect_mesh(nx, ny, 0.02 * nx / 400, 0.0125 * ny / 250, jitter=jitter,
                         seed=seed, periodic=True)


def euler3d_mesh(nx: int = 70, ny: int = 70, nz: int = 68, jitter: float = 0.1,
                 seed: int = 11) -> Mesh:
    """Periodic unit cube (for the default sizes), Kuhn-split, jittered."""
    return kuhn_tet_mesh(nx, ny, nz, 1.0 * nx / 70, 1.0 * ny / 70, 1.0 * nz / 68,
                         jitter=jitter, seed=seed, periodic=True)


def ns3d_mesh(n: int = 110, jitter: float = 0.1, seed: int = 13) -> Mesh:
    """Periodic cube of side 1 cm, Kuhn-split n^3 cubes (6 n^3 tets), jittered."""
    return kuhn_tet_mesh(n, n, n, 0.01, 0.01, 0.01, jitter=jitter, seed=seed, periodic=True)


def serving_requests(n: int = 256, *, seed: int = 5, npool: int = 16, cell_min: float = 5e3,
                     cell_max: float = 2e6):
    """Request stream of the serving workload.

    Returns ``(pool, requests)``.  ``pool`` holds ``npool`` cell counts,
    log-uniform in [cell_min, cell_max]; each pool entry is meshed twice: a
    periodic unit square for gas requests (side = sqrt(cells / 2)) and the
    drift-diffusion box of ``dd_streamer_mesh`` at the matching resolution.
    Each request picks a pool entry uniformly; even ids are gas, odd ids
    drift-diffusion; ``scale`` (log-uniform in [0.5, 2]) multiplies the pool
    entry's initial state, so requests on one mesh differ; ``gap`` is the
    unit-rate exponential inter-arrival time (divide by the arrival rate).
    """
    rng = np.random.default_rng(seed)
    cells = np.exp(rng.uniform(math.log(cell_min), math.log(cell_max), size=npool))
    pool = []
    for c in cells:
        side = max(3, int(round(math.sqrt(c / 2.0))))
        nx = max(3, int(round(math.sqrt(c / 2.0 * 1.6))))
        ny = max(3, int(round(nx / 1.6)))
        pool.append(dict(cells=float(c), gas_side=side, dd_nx=nx, dd_ny=ny))
    which = rng.integers(npool, size=n)
    scale = np.exp(rng.uniform(math.log(0.5), math.log(2.0), size=n))
    gaps = rng.exponential(1.0, size=n)
    reqs = [dict(id=k, kind="gas" if k % 2 == 0 else "dd", pool=int(which[k]),
                 scale=float(scale[k]), gap=float(gaps[k])) for k in range(n)]
    return pool, reqs


# ---------------------------------------------------------------------------
# synthetic multi-species mixture (no thermochemical tables are available)
# ---------------------------------------------------------------------------

R_GAS = 8.314462618  # J/(mol K)


@dataclass
class Mixture:
    """Seeded synthetic species data for the multi-species transport model.

    W      molar masses [kg/mol]
    cp_a, cp_b, cp_c   c_p,k(T) = (R/W_k)(a + b tau + c tau^2), tau = T/1000
    Sc     Schmidt numbers (D_k = mu / (rho Sc_k))
    mu_ref, T_ref, Pr  mu = mu_ref (T/T_ref)^0.7, lambda = mu c_p / Pr
    """
    W: np.ndarray
    cp_a: np.ndarray
    cp_b: np.ndarray
    cp_c: np.ndarray
    Sc: np.ndarray
    mu_ref: float = 1.8e-5
    T_ref: float = 300.0
    Pr: float = 0.72

    @property
    def n(self) -> int:
        return int(self.W.size)


def synthetic_mixture(nspecies: int = 9, seed: int = 3) -> Mixture:
    rng = np.random.default_rng(seed)
    W = np.sort(rng.uniform(0.002, 0.044, size=nspecies))
    return Mixture(W=W, cp_a=rng.uniform(2.5, 4.0, size=nspecies),
                   cp_b=rng.uniform(0.0, 1.0, size=nspecies),
                   cp_c=rng.uniform(-0.2, 0.2, size=nspecies),
                   Sc=rng.uniform(0.4, 1.2, size=nspecies))


def _lattice_fields(mesh: Mesh, nfields_y: int, lattice: int, rng, ranges):
    """Dirichlet(1) fractions and uniform scalar fields drawn on a periodic
    lattice^nd lattice and interpolated (multi)linearly to the nodes."""
    nd = mesh.ndim
    shape = (lattice,) * nd
    Yl = rng.dirichlet(np.ones(nfields_y), size=shape)
    Sl = [rng.uniform(lo, hi, size=shape) for lo, hi in ranges]
    lengths = mesh.period if mesh.period is not None else (mesh.xyz.max(1) - mesh.xyz.min(1))
    lo = mesh.xyz.min(1)
    t = [(mesh.xyz[a] - lo[a]) / lengths[a] * lattice for a in range(nd)]
    i0 = [np.floor(ta).astype(np.int64) for ta in t]
    fr = [ta - ia for ta, ia in zip(t, i0)]
    Y = np.zeros((nfields_y, mesh.nnodes))
    S = [np.zeros(mesh.nnodes) for _ in ranges]
    for corner in np.ndindex(*(2,) * nd):
        w = np.ones(mesh.nnodes)
        idx = []
        for a in range(nd):
            w = w * (fr[a] if corner[a] else 1.0 - fr[a])
            idx.append((i0[a] + corner[a]) % lattice)
        Y += w[None, :] * Yl[tuple(idx)].T
        for f, fl in zip(S, Sl):
            f += w * fl[tuple(idx)]
    return Y / Y.sum(axis=0, keepdims=True), S


def ns_primitive_state(mesh: Mesh, mix: Mixture, *, seed: int = 4, lattice: int = 8,
                       T_range=(300.0, 2000.0), p: float = 101325.0,
                       vel=(100.0, 50.0, 25.0)) -> np.ndarray:
    """Primitive multi-species state [rho, u_1..u_nd, T, Y_1..Y_n] of the 3D
    multi-species workload: Dirichlet(1) mass fractions and T ~ U(300, 2000)
    K drawn on a periodic lattice^nd lattice and interpolated to the nodes
    (Y stays on the simplex, T inside the range), pressure 101325 Pa, so
    rho = p W_mix / (R T) with the mixture molar mass of the drawn Y, and a
    uniform velocity.  The library or the oracle turns it into conserved
    variables with its own equation of state."""
    rng = np.random.default_rng(seed)
    Y, (T,) = _lattice_fields(mesh, mix.n, lattice, rng, [T_range])
    r_mix = R_GAS * np.sum(Y / mix.W[:, None], axis=0)   # specific gas constant of the draw
    rho = p / (r_mix * T)
    nd = mesh.ndim
    velv = np.tile(np.asarray(vel[:nd], dtype=np.float64)[:, None], (1, mesh.nnodes))
    return np.stack([rho, *velv, T, *Y])


def ns_state(mesh: Mesh, mix: Mixture, *, seed: int = 4, lattice: int = 8,
             theta_range=(300.0, 2000.0), rho_range=(0.2, 1.2),
             vel=(100.0, 50.0, 25.0), cv_scale: float = 718.0) -> np.ndarray:
    """Conserved multi-species state [rho, rho u, rho E, rho Y_1..rho Y_n].

    Dirichlet(1) mass fractions, a temperature-like field theta ~ U(theta_range)
    and a density ~ U(rho_range), each drawn on a periodic lattice^nd lattice
    and interpolated (multi)linearly to the nodes (so Y stays on the simplex);
    uniform velocity.  The sensible energy is set to cv_scale*(theta - 298.15)
    J/kg -- a fixed species-independent scale, not the mixture model: the
    temperature and pressure follow from each solver's own mixture
    thermodynamics."""
    rng = np.random.default_rng(seed)
    nd = mesh.ndim
    shape = (lattice,) * nd
    Yl = rng.dirichlet(np.ones(mix.n), size=shape)          # [..., n]
    Tl = rng.uniform(theta_range[0], theta_range[1], size=shape)
    Rl = rng.uniform(rho_range[0], rho_range[1], size=shape)
    lengths = mesh.period if mesh.period is not None else (mesh.xyz.max(1) - mesh.xyz.min(1))
    lo = mesh.xyz.min(1)
    t = [(mesh.xyz[a] - lo[a]) / lengths[a] * lattice for a in range(nd)]
    i0 = [np.floor(ta).astype(np.int64) for ta in t]
    fr = [ta - ia for ta, ia in zip(t, i0)]
    Y = np.zeros((mix.n, mesh.nnodes))
    theta = np.zeros(mesh.nnodes)
    rho = np.zeros(mesh.nnodes)
    for corner in np.ndindex(*(2,) * nd):
        w = np.ones(mesh.nnodes)
        idx = []
        for a in range(nd):
            w = w * (fr[a] if corner[a] else 1.0 - fr[a])
            idx.append((i0[a] + corner[a]) % lattice)
        Y += w[None, :] * Yl[tuple(idx)].T
        theta += w * Tl[tuple(idx)]
        rho += w * Rl[tuple(idx)]
    Y = Y / Y.sum(axis=0, keepdims=True)
    velv = np.tile(np.asarray(vel[:nd], dtype=np.float64)[:, None], (1, mesh.nnodes))
    es = cv_scale * (theta - 298.15)
    rows = [rho] + [rho * v for v in velv] + [rho * (es + 0.5 * np.sum(velv ** 2, axis=0))]
    rows += [rho * y for y in Y]
    return np.stack(rows)
