"""Parity cases shared by the GPU tests and the smoke check: a seeded mesh, a
seeded state, and one scheme description translated into both the oracle's
and the library's parameter structs."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import oracle
from paper_2201_01291_amd import workloads as wl

LIMNAMES = {"first": 0, "minmod": 1, "vanleer": 2, "sweby": 3, "none": 4}


@dataclass
class Case:
    name: str
    mesh: object
    U: np.ndarray
    E: np.ndarray | None
    scheme: dict
    tiles: tuple = (0, 0)     # (max cells, max nodes) per tile; 0 = library default

    @property
    def model(self):
        return {"gas": 0, "dd": 1, "ns": 2}[self.scheme["model"]]

    def oracle_phys(self):
        s = self.scheme
        return oracle.Phys(model=self.model, flux={"roe": 1, "sg": 2}.get(s.get("flux"), 0),
                           limiter=LIMNAMES[s["limiter"]], rk=s.get("rk", 2),
                           nspecies=s.get("nspecies", 0), closure=int(s.get("closure", 1)),
                           beta=s.get("beta", 1.0), cfl=s.get("cfl", 0.5),
                           fourier=s.get("fourier", 0.25), gamma=1.4,
                           entropy_fix=s.get("fix", 0.1), z=s.get("z", []), mu=s.get("mu", []),
                           D=s.get("D", []), mixture=s.get("mixture"), diel=s.get("diel", 0.0),
                           predictor=s.get("predictor", 0))

    def vcx_phys(self, precision=0):
        from paper_2201_01291_amd import vcx
        s = self.scheme
        return vcx.physics(model=self.model, flux={"roe": 1, "sg": 2}.get(s.get("flux"), 0),
                           limiter=LIMNAMES[s["limiter"]], rk_stages=s.get("rk", 2),
                           nspecies=s.get("nspecies", 0), closure=int(s.get("closure", 1)),
                           precision=precision, beta=s.get("beta", 1.0), cfl=s.get("cfl", 0.5),
                           fourier=s.get("fourier", 0.25), gamma=1.4,
                           entropy_fix=s.get("fix", 0.1), z=s.get("z", []), mu=s.get("mu", []),
                           D=s.get("D", []), mixture=s.get("mixture"), diel=s.get("diel", 0.0),
                           predictor=s.get("predictor", 0))


DD2 = dict(model="dd", limiter="minmod", rk=1, nspecies=2, z=[-1.0, 1.0], mu=[0.04, 0.04],
           D=[0.1, 0.1])


def make_case(name: str) -> Case:
    if name == "dd2d-streamer":
        m = wl.dd_streamer_mesh(40, 25)
        n, E = wl.dd_fields(m, sigma=2e-3)
        return Case(name, m, n, E, dict(DD2))
    if name == "dd2d-diel":
        # dense plasma: the dielectric limit sets the time step
        m = wl.dd_streamer_mesh(40, 25, seed=3)
        n, E = wl.dd_fields(m, sigma=2e-3, seed=8, peak=2e19)
        return Case(name, m, n, E, dict(DD2, diel=0.8))
    if name == "dd2d-open-closure2":
        # second boundary-closure option: interpolated half-edge fluxes
        m = wl.tri_rect_mesh(23, 17, 0.02, 0.015, jitter=0.2, seed=12)
        n, E = wl.dd_fields(m, sigma=3e-3, seed=6)
        return Case(name, m, n, E, dict(DD2, limiter="vanleer", closure=2))
    if name == "euler2d-open-closure2":
        m = wl.tri_rect_mesh(18, 14, jitter=0.2, seed=13)
        U = wl.euler_blob_state(m, nblobs=3, amp=0.3, sigma=0.2, mach=0.5)
        return Case(name, m, U, None, dict(model="gas", flux="hllc", limiter="minmod", rk=2, closure=2))
    if name == "dd2d-open-vanleer":
        m = wl.tri_rect_mesh(23, 17, 0.02, 0.015, jitter=0.2, seed=9)
        n, E = wl.dd_fields(m, sigma=3e-3, seed=4)
        return Case(name, m, n, E, dict(DD2, limiter="vanleer"))
    if name == "dd3d-sweby":
        m = wl.kuhn_tet_mesh(5, 5, 6, 1e-3, 1e-3, 1.2e-3, jitter=0.1, seed=3)
        n, E = wl.dd_fields(m, sigma=3e-4, bump_sigma=2e-4, bump_amp=50.0, nspecies=1)
        return Case(name, m, n, E, dict(model="dd", limiter="sweby", beta=1.5, rk=1, nspecies=1,
                                        z=[-1.0], mu=[0.04], D=[0.1]))
    if name == "sod-hllc":
        m = wl.sod_tube(100, 10)
        return Case(name, m, wl.sod_state(m), None,
                    dict(model="gas", flux="hllc", limiter="minmod", rk=2))
    if name == "euler2d-roe-sp2":
        m = wl.tri_rect_mesh(20, 16, jitter=0.2, seed=5, periodic=True)
        U = wl.euler_blob_state(m, nblobs=4, amp=0.3, sigma=0.15, nspecies=2)
        return Case(name, m, U, None,
                    dict(model="gas", flux="roe", limiter="vanleer", rk=2, nspecies=2))
    if name == "euler3d-roe":
        m = wl.kuhn_tet_mesh(7, 6, 6, jitter=0.1, seed=11)
        U = wl.euler_blob_state(m, nblobs=8, amp=0.1, sigma=0.2)
        return Case(name, m, U, None, dict(model="gas", flux="roe", limiter="vanleer", rk=2))
    if name == "euler3d-hllc-open-sp2":
        m = wl.kuhn_tet_mesh(4, 4, 5, jitter=0.15, seed=2, periodic=False)
        U = wl.euler_blob_state(m, nblobs=3, amp=0.4, sigma=0.3, nspecies=2, mach=0.6)
        return Case(name, m, U, None, dict(model="gas", flux="hllc", limiter="sweby", beta=1.5,
                                           rk=3, nspecies=2))
    if name == "euler3d-hllc-sp9":
        m = wl.kuhn_tet_mesh(5, 5, 5, jitter=0.1, seed=6)
        U = wl.euler_blob_state(m, nblobs=4, amp=0.2, sigma=0.25, nspecies=9)
        return Case(name, m, U, None, dict(model="gas", flux="hllc", limiter="minmod", rk=4,
                                           nspecies=9))
    if name == "ns3d-sp9":
        mix = wl.synthetic_mixture(9, seed=3)
        m = wl.kuhn_tet_mesh(5, 4, 5, 0.01, 0.008, 0.01, jitter=0.1, seed=8)
        U = wl.ns_state(m, mix, lattice=4, seed=6)
        return Case(name, m, U, None, dict(model="ns", flux="hllc", limiter="vanleer", rk=2,
                                           nspecies=9, mixture=mix), tiles=(64, 48))
    if name == "ns3d-sp2-smalltile":
        # small flux tiles: the gradient pass's tiles (four times larger)
        # still split the mesh, so its shared-node completion runs
        mix = wl.synthetic_mixture(2, seed=7)
        mix.mu_ref = 2e-3
        m = wl.kuhn_tet_mesh(4, 4, 3, 0.008, 0.008, 0.006, jitter=0.15, seed=12)
        U = wl.ns_state(m, mix, lattice=3, seed=13, vel=(25.0, -10.0, 5.0))
        return Case(name, m, U, None, dict(model="ns", flux="hllc", limiter="minmod", rk=3,
                                           nspecies=2, mixture=mix), tiles=(24, 20))
    if name == "ns2d-sp2-open":
        mix = wl.synthetic_mixture(2, seed=5)
        mix.mu_ref = 2e-3    # visible diffusive fluxes at this resolution
        m = wl.tri_rect_mesh(14, 11, 0.01, 0.008, jitter=0.2, seed=4)
        U = wl.ns_state(m, mix, lattice=3, seed=9, vel=(30.0, -10.0))
        return Case(name, m, U, None, dict(model="ns", flux="hllc", limiter="minmod", rk=3,
                                           nspecies=2, mixture=mix))
    if name == "ns2d-sp2-bigtile":
        # tiles of more cells than a block has threads: the multi-species
        # flux pass keeps the cells' vertex parts apart from the staged fields
        mix = wl.synthetic_mixture(2, seed=6)
        mix.mu_ref = 2e-3
        m = wl.tri_rect_mesh(24, 17, 0.012, 0.009, jitter=0.2, seed=21)
        U = wl.ns_state(m, mix, lattice=3, seed=10, vel=(20.0, 15.0))
        return Case(name, m, U, None, dict(model="ns", flux="hllc", limiter="vanleer", rk=2,
                                           nspecies=2, mixture=mix), tiles=(320, 200))
    # -- cases that drive faces transonic or supersonic ------------------
    if name == "shock1d-roe-vanleer":
        # the paper's modified shock tube (table shock_1d): its left
        # rarefaction is transonic, where Roe's entropy fix acts
        m = wl.sod_tube(100, 10)
        U = wl.sod_state(m, left=(1.0, 0.75, 1.0), right=(0.125, 0.0, 0.1))
        return Case(name, m, U, None, dict(model="gas", flux="roe", limiter="vanleer", rk=2))
    if name == "euler2d-mach2.5-hllc":
        # supersonic stream: both fully upwind HLLC branches (0 <= S_L, S_R < 0)
        m = wl.tri_rect_mesh(20, 16, jitter=0.2, seed=14, periodic=True)
        U = wl.euler_blob_state(m, nblobs=4, amp=0.4, sigma=0.15, mach=2.5, seed=3)
        return Case(name, m, U, None, dict(model="gas", flux="hllc", limiter="minmod", rk=2))
    if name == "euler2d-mach2.5-roe-sp2":
        m = wl.tri_rect_mesh(18, 17, jitter=0.2, seed=15, periodic=True)
        U = wl.euler_blob_state(m, nblobs=4, amp=0.4, sigma=0.15, mach=2.5, seed=4, nspecies=2)
        return Case(name, m, U, None, dict(model="gas", flux="roe", limiter="vanleer", rk=3,
                                           nspecies=2))
    if name == "explosion2d":
        # cylindrical explosion (Sec. "Explosions"): [0,2]^2, circle of radius
        # 0.4, HLLC-MUSCL RK2 with the Sweby limiter at beta = 1.7
        m = wl.tri_rect_mesh(40, 40, 2.0, 2.0)
        U = wl.explosion_state(m)
        return Case(name, m, U, None, dict(model="gas", flux="hllc", limiter="sweby", beta=1.7,
                                           rk=2))
    if name == "riemann2d-c3-hllc":
        # 2D Riemann problem, every quadrant moving outward (the rho = 3
        # quadrant is supersonic, Mach 1.3)
        m = wl.tri_rect_mesh(30, 30, 1.0, 1.0, origin=(-0.5, -0.5))
        U = wl.quadrant_state(m, 3)
        return Case(name, m, U, None, dict(model="gas", flux="hllc", limiter="minmod", rk=2))
    if name == "riemann2d-c4-roe":
        # every quadrant moving inward: colliding shocks
        m = wl.tri_rect_mesh(30, 30, 1.0, 1.0, origin=(-0.5, -0.5))
        U = wl.quadrant_state(m, 4)
        return Case(name, m, U, None, dict(model="gas", flux="roe", limiter="vanleer", rk=2))
    if name == "euler3d-mach2-roe":
        m = wl.kuhn_tet_mesh(6, 6, 6, jitter=0.1, seed=16)
        U = wl.euler_blob_state(m, nblobs=6, amp=0.4, sigma=0.2, mach=2.0, seed=5)
        return Case(name, m, U, None, dict(model="gas", flux="roe", limiter="vanleer", rk=2))
    if name == "euler3d-mach2-hllc-sp2":
        m = wl.kuhn_tet_mesh(5, 6, 5, jitter=0.1, seed=17)
        U = wl.euler_blob_state(m, nblobs=6, amp=0.4, sigma=0.2, mach=2.0, seed=6, nspecies=2)
        return Case(name, m, U, None, dict(model="gas", flux="hllc", limiter="minmod", rk=2,
                                           nspecies=2))
    if name == "explosion3d-hllc":
        # spherical explosion (Sec. "Explosions"), open cube
        m = wl.kuhn_tet_mesh(8, 8, 8, 2.0, 2.0, 2.0, periodic=False)
        U = wl.explosion_state(m, centre=(1.0, 1.0, 1.0), radius=0.5)
        return Case(name, m, U, None, dict(model="gas", flux="hllc", limiter="sweby", beta=1.7,
                                           rk=2))
    # -- MUSCL-Hancock predictor (one forward-Euler stage) ---------------
    if name == "euler2d-hancock-hllc":
        m = wl.tri_rect_mesh(20, 16, jitter=0.2, seed=23, periodic=True)
        U = wl.euler_blob_state(m, nblobs=4, amp=0.3, sigma=0.15, mach=0.8, seed=7)
        return Case(name, m, U, None, dict(model="gas", flux="hllc", limiter="vanleer", rk=1,
                                           predictor=1))
    if name == "sod-hancock-roe":
        m = wl.sod_tube(100, 10)
        return Case(name, m, wl.sod_state(m), None,
                    dict(model="gas", flux="roe", limiter="minmod", rk=1, predictor=1))
    if name == "euler2d-open-closure2-hancock":
        m = wl.tri_rect_mesh(18, 14, jitter=0.2, seed=24)
        U = wl.euler_blob_state(m, nblobs=3, amp=0.3, sigma=0.2, mach=0.5, seed=8, nspecies=2)
        return Case(name, m, U, None, dict(model="gas", flux="hllc", limiter="sweby", beta=1.5,
                                           rk=1, closure=2, nspecies=2, predictor=1))
    if name == "euler3d-hancock-roe-sp2":
        m = wl.kuhn_tet_mesh(6, 5, 6, jitter=0.1, seed=25, periodic=False)
        U = wl.euler_blob_state(m, nblobs=5, amp=0.3, sigma=0.25, mach=0.7, seed=9, nspecies=2)
        return Case(name, m, U, None, dict(model="gas", flux="roe", limiter="vanleer", rk=1,
                                           nspecies=2, predictor=1))
    if name == "euler3d-hancock-hllc-sp9":
        m = wl.kuhn_tet_mesh(5, 5, 5, jitter=0.1, seed=26)
        U = wl.euler_blob_state(m, nblobs=4, amp=0.2, sigma=0.25, nspecies=9, mach=1.2, seed=10)
        # the predictor's increments take more LDS than the default 3D tile
        # leaves with nine species in FP64
        return Case(name, m, U, None, dict(model="gas", flux="hllc", limiter="minmod", rk=1,
                                           nspecies=9, predictor=1), tiles=(96, 72))
    # -- Scharfetter-Gummel drift-diffusion flux --------------------------
    if name == "dd2d-sg":
        m = wl.dd_streamer_mesh(40, 25, seed=4)
        n, E = wl.dd_fields(m, sigma=2e-3, seed=11)
        return Case(name, m, n, E, dict(DD2, flux="sg", rk=2))
    if name == "dd2d-open-sg":
        m = wl.tri_rect_mesh(23, 17, 0.02, 0.015, jitter=0.2, seed=27)
        n, E = wl.dd_fields(m, sigma=3e-3, seed=12)
        return Case(name, m, n, E, dict(DD2, flux="sg"))
    if name == "dd3d-sg":
        m = wl.kuhn_tet_mesh(5, 5, 6, 1e-3, 1e-3, 1.2e-3, jitter=0.1, seed=28)
        n, E = wl.dd_fields(m, sigma=3e-4, bump_sigma=2e-4, bump_amp=50.0, nspecies=1, seed=13)
        return Case(name, m, n, E, dict(model="dd", flux="sg", limiter="minmod", rk=2, nspecies=1,
                                        z=[-1.0], mu=[0.04], D=[0.1]))
    # -- 2D quadrilateral meshes -----------------------------------------
    if name == "quad-dd-llw":
        m = wl.quad_rect_mesh(36, 22, 2e-3, 1.2e-3, jitter=0.2, seed=31, periodic=True)
        n, E = wl.dd_fields(m, sigma=2e-4, seed=14)
        return Case(name, m, n, E, dict(DD2, limiter="vanleer", rk=2), tiles=(96, 120))
    if name == "quad-dd-sg-open":
        m = wl.quad_rect_mesh(23, 17, 0.02, 0.015, jitter=0.2, seed=32)
        n, E = wl.dd_fields(m, sigma=3e-3, seed=15)
        return Case(name, m, n, E, dict(DD2, flux="sg"))
    if name == "quad-euler-hllc":
        m = wl.quad_rect_mesh(24, 18, jitter=0.2, seed=33, periodic=True)
        U = wl.euler_blob_state(m, nblobs=4, amp=0.3, sigma=0.15, mach=0.8, seed=11)
        return Case(name, m, U, None, dict(model="gas", flux="hllc", limiter="vanleer", rk=2))
    if name == "quad-euler-roe-sp2-closure2":
        m = wl.quad_rect_mesh(18, 14, jitter=0.2, seed=34)
        U = wl.euler_blob_state(m, nblobs=3, amp=0.4, sigma=0.2, mach=1.5, seed=12, nspecies=2)
        return Case(name, m, U, None, dict(model="gas", flux="roe", limiter="minmod", rk=3, nspecies=2,
                                           closure=2))
    if name == "quad-explosion-hancock":
        m = wl.quad_rect_mesh(40, 40, 2.0, 2.0)
        U = wl.explosion_state(m)
        return Case(name, m, U, None, dict(model="gas", flux="hllc", limiter="sweby", beta=1.5, rk=1,
                                           predictor=1))
    raise KeyError(name)


# Cases on 2D quadrilateral meshes (gas and drift-diffusion)
QUAD_CASES = ["quad-dd-llw", "quad-dd-sg-open", "quad-euler-hllc", "quad-euler-roe-sp2-closure2",
              "quad-explosion-hancock"]

# Drift-diffusion cases with the Scharfetter-Gummel flux
SG_CASES = ["dd2d-sg", "dd2d-open-sg", "dd3d-sg"]

# Gas cases with the MUSCL-Hancock predictor (plane meshes, one stage)
HANCOCK_CASES = ["euler2d-hancock-hllc", "sod-hancock-roe", "euler2d-open-closure2-hancock",
                 "euler3d-hancock-roe-sp2", "euler3d-hancock-hllc-sp9"]

# Gas cases built to reach the transonic and supersonic branches of the
# Riemann fluxes, with the branches each must reach (oracle branch counters)
BRANCH_CASES = {
    "shock1d-roe-vanleer": ("roe_entropy_fix",),
    "euler2d-mach2.5-hllc": ("hllc_left_supersonic", "hllc_right_supersonic"),
    "euler2d-mach2.5-roe-sp2": ("roe_entropy_fix",),
    "explosion2d": ("hllc_star_left", "hllc_star_right"),
    "riemann2d-c3-hllc": ("hllc_left_supersonic", "hllc_right_supersonic"),
    "riemann2d-c4-roe": ("roe_entropy_fix",),
    "euler3d-mach2-roe": ("roe_entropy_fix",),
    "euler3d-mach2-hllc-sp2": ("hllc_left_supersonic", "hllc_right_supersonic"),
    "explosion3d-hllc": ("hllc_star_left", "hllc_star_right"),
}

CASE_NAMES = ["dd2d-streamer", "dd2d-diel", "dd2d-open-vanleer", "dd2d-open-closure2",
              "euler2d-open-closure2", "dd3d-sweby", "sod-hllc", "euler2d-roe-sp2",
              "euler3d-roe", "euler3d-hllc-open-sp2", "euler3d-hllc-sp9", "ns3d-sp9", "ns3d-sp2-smalltile",
              "ns2d-sp2-open", "ns2d-sp2-bigtile", *BRANCH_CASES, *HANCOCK_CASES, *SG_CASES,
              *QUAD_CASES]


def reconstructed(case: Case) -> np.ndarray:
    """W = (U, p) for gas, U for drift-diffusion (test-side input preparation;
    the multi-species pressure comes from the oracle's node state)."""
    if case.model == 1:
        return case.U
    if case.model == 2:
        ph = case.oracle_phys()
        p = np.array([oracle.ns_node(case.mesh.ndim, ph, case.U[:, i])[1]
                      for i in range(case.mesh.nnodes)])
        return np.vstack([case.U, p[None]])
    nd = case.mesh.ndim
    rho = case.U[0]
    ke = 0.5 * np.sum(case.U[1:1 + nd] ** 2, axis=0) / rho
    p = 0.4 * (case.U[1 + nd] - ke)
    return np.vstack([case.U, p[None]])


def normwise(a, b, scale):
    """max_i |a - b| / max_i scale, per variable (rows)."""
    num = np.abs(a - b).reshape(a.shape[0], -1).max(axis=1)
    den = np.abs(scale).reshape(scale.shape[0], -1).max(axis=1)
    den = np.where(den > 0, den, np.abs(scale).max())   # rows that are zero everywhere
    return num / den


def state_err(case: Case, Ua, Ub):
    """Norm-wise state difference per variable, max_i |Ua - Ub| / max_i |Ub|,
    with the momentum components normalised by the largest momentum
    component (a vector quantity: its scale does not depend on the axes)."""
    den = np.abs(Ub).max(axis=1)
    if case.model != 1:
        nd = case.mesh.ndim
        den[1:1 + nd] = den[1:1 + nd].max()
    den = np.where(den > 0, den, np.abs(Ub).max())
    return np.abs(Ua - Ub).max(axis=1) / den
