"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Bar: FP64 path within 1e-12 norm-wise -- max_i |r_gpu - r_oracle| divided by
max_i sum_f |F_f . S_f| (per variable), a residual norm scaled by the face
fluxes, since a residual is a difference of face fluxes and can vanish where
the fluxes do not.  States after N steps: max |dU| / max |U| <= 1e-12 per variable.
Mixed precision (FP32 flux) errors are measured and printed; the bound
asserted for them is stated in each test.
"""
import os

import numpy as np
import pytest

import oracle
from cases import CASE_NAMES, make_case, normwise, reconstructed, state_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2201_01291_amd import vcx  # noqa: E402

FP64_TOL = 1e-12


def _setup(case, precision=0):
    print(f"[case] {case.name} prec={precision} nn={case.mesh.nnodes} nc={case.mesh.ncells}",
          flush=True)
    om = oracle.OracleMesh(case.mesh)
    gm = vcx.Mesh(case.mesh, tile_cells=case.tiles[0], tile_nodes=case.tiles[1])
    s = vcx.Solver(gm, case.vcx_phys(precision), case.E)
    s.upload(case.U)
    return om, gm, s


@pytest.mark.parametrize("name", CASE_NAMES)
def test_gradient_parity(name):
    case = make_case(name)
    om, gm, s = _setup(case)
    W = reconstructed(case)
    Go = om.gradient(W)
    Gg = s.gradient()
    h = (case.mesh.ncells / om.geometry()["Vc"].sum()) ** (1.0 / case.mesh.ndim)
    scale = np.abs(W).max(axis=1) * h
    scale = np.where(scale > 0, scale, np.abs(W).max() * h)   # rows that are zero everywhere
    err = np.abs(Gg - Go).max(axis=(1, 2)) / scale
    print("gradient err", err)
    assert err.max() <= FP64_TOL


@pytest.mark.parametrize("name", ["ns3d-sp9", "ns2d-sp2-open"])
def test_gradient_query_of_a_mixed_solver_is_fp64(name):
    """The multi-species FP32 path keeps G in FP32 between its passes; the
    gradient query still runs the FP64 pass, so a mixed solver returns the
    FP64 solver's gradient exactly."""
    case = make_case(name)
    _, _, s64 = _setup(case)
    _, _, s32 = _setup(case, precision=1)
    G64, G32 = s64.gradient(), s32.gradient()
    assert np.array_equal(G64, G32)
    # after a step (whose gradient passes stored FP32 rows) the query is the
    # FP64 gradient of the stepped state
    s32.step(1)
    s64.upload(s32.download())
    assert np.array_equal(s32.gradient(), s64.gradient())


@pytest.mark.parametrize("name", CASE_NAMES)
def test_residual_parity_fp64(name):
    case = make_case(name)
    om, gm, s = _setup(case)
    ph = case.oracle_phys()
    dt = om.timestep(ph, case.U, case.E)
    ro = om.residual(ph, case.U, case.E, dt)
    rg = s.residual(dt)
    err = normwise(rg, ro, om.flux_scale(ph, case.U, case.E, dt))
    print("residual err", err)
    assert err.max() <= FP64_TOL


@pytest.mark.parametrize("name", CASE_NAMES)
def test_residual_mixed_precision_error_stated(name):
    """FP32 reconstruction/limiter/flux with FP64 accumulation: error against
    the FP64 oracle is printed; asserted bound 1e-4 norm-wise (FP32 epsilon
    1.2e-7 times the flux cancellation of a few cell-edges)."""
    case = make_case(name)
    om, gm, s = _setup(case, precision=1)
    ph = case.oracle_phys()
    dt = om.timestep(ph, case.U, case.E)
    ro = om.residual(ph, case.U, case.E, dt)
    rg = s.residual(dt)
    err = normwise(rg, ro, om.flux_scale(ph, case.U, case.E, dt))
    print(f"MIXED residual err {name}: {err}")
    assert err.max() <= 1e-4


@pytest.mark.parametrize("name", CASE_NAMES)
def test_timestep_parity(name):
    case = make_case(name)
    om, gm, s = _setup(case)
    assert s.timestep() == pytest.approx(om.timestep(case.oracle_phys(), case.U, case.E), rel=1e-13)


@pytest.mark.parametrize("name", CASE_NAMES)
def test_step_parity_fp64(name):
    case = make_case(name)
    om, gm, s = _setup(case)
    ph = case.oracle_phys()
    Uo, to, dto, no = om.step(ph, case.U, case.E, nsteps=5)
    tg, dtg = s.step(5)
    Ug = s.download()
    assert s.steps_done() == 5 and no == 5
    assert tg == pytest.approx(to, rel=1e-12) and dtg == pytest.approx(dto, rel=1e-12)
    err = state_err(case, Ug, Uo)
    print("state err", err)
    assert err.max() <= FP64_TOL


@pytest.mark.parametrize("name", ["euler3d-roe", "dd2d-streamer", "euler2d-roe-sp2"])
def test_conservation_sums(name):
    case = make_case(name)
    om, gm, s = _setup(case)
    so, ao = om.sums(case.U)
    sg = s.sums()
    np.testing.assert_allclose(sg, so, rtol=0, atol=1e-13 * ao.max())
    s.step(10)
    sg2 = s.sums()
    drift = np.abs(sg2 - sg) / np.maximum(ao, 1e-300)
    print("conservation drift", drift)
    assert np.all((drift <= 1e-13) | (ao == 0))


@pytest.mark.parametrize("name", ["euler3d-roe", "dd2d-streamer", "sod-hllc"])
def test_bitwise_determinism(name):
    case = make_case(name)
    om, gm, s = _setup(case)
    r1 = s.residual(1e-12)
    r2 = s.residual(1e-12)
    assert np.array_equal(r1, r2)
    s.step(3)
    U1 = s.download()
    s.upload(case.U)
    s.step(3)
    assert np.array_equal(s.download(), U1)
    # an independent solver on an independent mesh object gives the same bits
    s2 = vcx.Solver(vcx.Mesh(case.mesh), case.vcx_phys(), case.E)
    s2.upload(case.U)
    s2.step(3)
    assert np.array_equal(s2.download(), U1)


def test_device_pointer_io():
    case = make_case("euler3d-roe")
    om, gm, s = _setup(case)
    r_host = s.residual()
    Ud = torch.tensor(case.U, device="cuda", dtype=torch.float64)
    s.upload(Ud)
    rd = torch.empty_like(Ud)
    s.residual(out=rd)
    torch.cuda.synchronize()
    assert np.array_equal(rd.cpu().numpy(), r_host)
    out = torch.zeros_like(Ud)
    s.download(out=out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), case.U)


def test_shock_tube_to_t_end_matches_oracle():
    """The shock-tube workload (100x10 tube, HLLC-minmod-RK2, CFL 0.5) run to
    t = 0.2 on the GPU: every step's dt and the final state against the oracle."""
    case = make_case("sod-hllc")
    om, gm, s = _setup(case)
    ph = case.oracle_phys()
    Uo, to, _, no = om.step(ph, case.U, nsteps=100000, t_end=0.2)
    tg, _ = s.step(100000, t_end=0.2)
    assert s.steps_done() == no and tg == pytest.approx(0.2, abs=1e-14)
    err = state_err(case, s.download(), Uo)
    print("sod state err", err, "steps", no)
    assert err.max() <= FP64_TOL


def test_unstable_state_is_reported_and_state_kept():
    case = make_case("euler2d-roe-sp2")
    U = case.U.copy()
    U[3, 17] = 1e-3  # energy below kinetic energy: negative pressure
    om, gm, s = _setup(case)
    s.upload(U)
    with pytest.raises(vcx.VcxError) as e:
        s.step(2)
    assert e.value.code == vcx.E_UNSTABLE
    assert s.steps_done() == 0
    assert np.array_equal(s.download(), U)


def test_unstable_after_good_steps_keeps_last_good_state():
    """A blow-up in a later step leaves the state of the last good step."""
    case = make_case("dd2d-streamer")
    om, gm, s = _setup(case)
    s.step(2)
    U2 = s.download()
    bad = U2.copy()
    bad[0, 5] = np.nan
    s.upload(bad)
    with pytest.raises(vcx.VcxError):
        s.step(3)
    assert s.steps_done() == 0
    np.testing.assert_array_equal(np.isnan(s.download()), np.isnan(bad))


def test_full_size_drift_diffusion_residual_and_steps():
    """The 200k-cell jittered drift-diffusion workload at full size: residual
    and 3 steps against the oracle (the oracle handles 6e5 faces quickly)."""
    from paper_2201_01291_amd import workloads as wl
    import cases
    m = wl.dd_streamer_mesh()
    n, E = wl.dd_fields(m)
    case = cases.Case("dd2d-full", m, n, E, dict(cases.DD2))
    om, gm, s = _setup(case)
    ph = case.oracle_phys()
    dt = om.timestep(ph, n, E)
    assert s.timestep() == pytest.approx(dt, rel=1e-13)
    err = normwise(s.residual(dt), om.residual(ph, n, E, dt), om.flux_scale(ph, n, E, dt))
    assert err.max() <= FP64_TOL
    Uo, *_ = om.step(ph, n, E, nsteps=3)
    s.step(3)
    assert state_err(case, s.download(), Uo).max() <= FP64_TOL


def test_binding_first_in_a_fresh_process():
    """A process whose first GPU work goes through the binding (PyTorch not
    imported before it) creates a mesh and a solver and takes a step: the
    library and PyTorch share one copy of the HIP runtime."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("from paper_2201_01291_amd import vcx, workloads as wl\n"
            "m = wl.tri_rect_mesh(16, 12, periodic=True)\n"
            "n, E = wl.dd_fields(m, sigma=2e-3)\n"
            "gm = vcx.Mesh(m)\n"
            "s = vcx.Solver(gm, vcx.physics(model=vcx.MODEL_DRIFT_DIFFUSION, nspecies=2, z=[1.0, -1.0],"
            " mu=[0.03, 0.05], D=[0.1, 0.2]), E)\n"
            "s.upload(n)\n"
            "s.step(2)\n"
            "print('ok', s.download().shape)\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    print(out.stdout, out.stderr[-2000:])
    assert out.returncode == 0 and "ok" in out.stdout


def test_large_drift_diffusion_mesh_on_the_separate_passes():
    """A drift-diffusion mesh above 2^20 cells (the size family of the
    workload, 1.2M cells) takes the separate gradient and flux passes, its
    gradient from the node-gradient tables: time step, residual and 2 steps
    against the oracle, and the gradient against the oracle's."""
    from paper_2201_01291_amd import workloads as wl
    import cases
    m = wl.dd_streamer_mesh(800, 750)
    assert m.ncells > 1 << 20
    n, E = wl.dd_fields(m)
    case = cases.Case("dd2d-large", m, n, E, dict(cases.DD2))
    print(f"[case] {case.name} nc={m.ncells}", flush=True)
    om, gm, s = _setup(case)
    s.profile(True)
    ph = case.oracle_phys()
    dt = om.timestep(ph, n, E)
    assert s.timestep() == pytest.approx(dt, rel=1e-13)
    err = normwise(s.residual(dt), om.residual(ph, n, E, dt), om.flux_scale(ph, n, E, dt))
    assert err.max() <= FP64_TOL
    assert s.profile_query("gradient")[0] >= 1     # the separate passes ran
    assert s.profile_query("gradient_shared")[0] == 0   # with no completion pass
    W = reconstructed(case)
    h = (m.ncells / om.geometry()["Vc"].sum()) ** 0.5
    gerr = np.abs(s.gradient() - om.gradient(W)).max(axis=(1, 2)) / (np.abs(W).max(axis=1) * h)
    assert gerr.max() <= FP64_TOL
    Uo, *_ = om.step(ph, n, E, nsteps=2)
    s.step(2)
    assert state_err(case, s.download(), Uo).max() <= FP64_TOL


def test_full_size_euler3d_residual_and_steps():
    """The 2M-tet periodic 3D Euler workload (Roe + van Leer, RK2) at full
    size and in the benchmark's tiling: time step, FP64 residual and two
    steps against the oracle (about 15 s of oracle work)."""
    from paper_2201_01291_amd import workloads as wl
    import cases
    m = wl.euler3d_mesh()
    U = wl.euler_blob_state(m)
    case = cases.Case("euler3d-full", m, U, None,
                      dict(model="gas", flux="roe", limiter="vanleer", rk=2))
    om, gm, s = _setup(case)
    ph = case.oracle_phys()
    dt = om.timestep(ph, U, None)
    assert s.timestep() == pytest.approx(dt, rel=1e-13)
    err = normwise(s.residual(dt), om.residual(ph, U, None, dt), om.flux_scale(ph, U, None, dt))
    print("euler3d full residual err", err)
    assert err.max() <= FP64_TOL
    Uo, to, _, _ = om.step(ph, U, None, nsteps=2)
    tg, _ = s.step(2)
    assert tg == pytest.approx(to, rel=1e-12)
    assert state_err(case, s.download(), Uo).max() <= FP64_TOL


def test_full_size_ns3d_properties():
    """The 8M-tet, 9-species Navier-Stokes workload at full size, in the
    benchmark's 64-cell tiling (the oracle needs minutes here, so properties
    that hold at any size): the residual of a periodic mesh sums to zero per
    variable, the mixed-precision residual stays within its stated bound of
    the FP64 one, two steps conserve every total, and FP64 and mixed states
    agree after them."""
    from paper_2201_01291_amd import workloads as wl
    import cases
    mix = wl.synthetic_mixture(9, seed=3)
    m = wl.ns3d_mesh()
    U = wl.ns_state(m, mix, lattice=8, seed=4)
    case = cases.Case("ns3d-full", m, U, None,
                      dict(model="ns", flux="hllc", limiter="vanleer", rk=2, nspecies=9,
                           mixture=mix), tiles=(64, 48))
    print(f"[case] {case.name} nn={m.nnodes} nc={m.ncells}", flush=True)
    gm = vcx.Mesh(m, tile_cells=64, tile_nodes=48)
    s64 = vcx.Solver(gm, case.vcx_phys(0), None)
    s32 = vcx.Solver(gm, case.vcx_phys(1), None)
    s64.upload(U)
    s32.upload(U)
    dt = s64.timestep()
    assert dt > 0 and s32.timestep() == dt      # the time step is FP64 on both paths
    r64, r32 = s64.residual(dt), s32.residual(dt)
    mag = np.abs(r64).sum(axis=1)
    assert np.all(np.abs(r64.sum(axis=1)) <= 1e-11 * mag)
    mixed = np.abs(r32 - r64).max(axis=1) / np.abs(r64).max(axis=1)
    print("ns3d full: mixed residual vs FP64", mixed)
    assert mixed.max() <= 1e-3
    Vn, _ = gm.geometry()
    absum = (np.abs(U) * Vn[None, :]).sum(axis=1)
    t0 = s64.sums()
    s64.step(2)
    s32.step(2)
    drift = np.abs(s64.sums() - t0) / absum
    print("ns3d full: conservation drift", drift)
    assert np.all(drift <= 1e-13)
    U64, U32 = s64.download(), s32.download()
    assert np.all(np.isfinite(U64))
    dev = np.abs(U32 - U64).max(axis=1) / np.abs(U64).max(axis=1)
    print("ns3d full: mixed state vs FP64 after 2 steps", dev)
    assert dev.max() <= 1e-5


@pytest.mark.parametrize("kind", ["ns3d", "gas2d-sp2"])
def test_primitive_upload_matches_the_oracle_conversion(kind):
    """vcx_state_upload_primitive converts (rho, u, T, Y) or (rho, u, p, Y)
    with the library's equation of state: the conserved state equals the
    oracle's conversion of the same primitives to 1e-14, and the residual of
    that state matches the oracle's within the FP64 bar."""
    from paper_2201_01291_amd import workloads as wl
    import cases
    if kind == "ns3d":
        mix = wl.synthetic_mixture(9, seed=3)
        m = wl.kuhn_tet_mesh(5, 5, 4, 0.01, 0.01, 0.008, jitter=0.1, seed=9)
        P = wl.ns_primitive_state(m, mix, lattice=3, seed=2)
        scheme = dict(model="ns", flux="hllc", limiter="vanleer", rk=2, nspecies=9, mixture=mix)
    else:
        m = wl.tri_rect_mesh(16, 12, jitter=0.2, seed=3, periodic=True)
        rng = np.random.default_rng(4)
        Y = rng.dirichlet(np.ones(2), size=m.nnodes).T
        P = np.stack([rng.uniform(0.5, 1.5, m.nnodes), rng.uniform(-0.3, 0.3, m.nnodes),
                      rng.uniform(-0.3, 0.3, m.nnodes), rng.uniform(0.5, 1.0, m.nnodes), *Y])
        scheme = dict(model="gas", flux="hllc", limiter="minmod", rk=2, nspecies=2)
    case = cases.Case(f"prim-{kind}", m, None, None, scheme)
    ph = case.oracle_phys()
    Uo = oracle.conserved_from_primitive(m.ndim, ph, P)
    case.U = Uo
    print(f"[case] {case.name} nn={m.nnodes} T range "
          f"{P[1 + m.ndim].min():.1f}..{P[1 + m.ndim].max():.1f}", flush=True)
    gm = vcx.Mesh(m)
    s = vcx.Solver(gm, case.vcx_phys(), None)
    s.upload_primitive(P)
    Ug = s.download()
    rel = np.abs(Ug - Uo).max(axis=1) / np.abs(Uo).max(axis=1)
    print("conversion rel err", rel)
    assert rel.max() <= 1e-14
    om = oracle.OracleMesh(m)
    dt = om.timestep(ph, Uo)
    err = normwise(s.residual(dt), om.residual(ph, Uo, None, dt), om.flux_scale(ph, Uo, None, dt))
    print("residual err", err)
    assert err.max() <= FP64_TOL
