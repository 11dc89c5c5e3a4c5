"""GPU trajectories against the FP64 oracle: the paper's modified shock tube
with Roe's flux to its end time (its transonic rarefaction is where Roe's
entropy fix acts), the benchmark's own tile sizes on smaller meshes of the
same kind, and the full drift-diffusion workload for its 1000 steps with the
first checkpoint above the FP64 bar reported."""
import json
import os

import numpy as np
import pytest

import oracle
import cases
from cases import make_case, normwise, state_err
from paper_2201_01291_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2201_01291_amd import vcx  # noqa: E402
from paper_2201_01291_amd import autotune  # noqa: E402

FP64_TOL = 1e-12
MIXED_TOL = 1e-4


def _setup(case, precision=0):
    print(f"[case] {case.name} prec={precision} tiles={case.tiles} nn={case.mesh.nnodes} "
          f"nc={case.mesh.ncells}", flush=True)
    gm = vcx.Mesh(case.mesh, tile_cells=case.tiles[0], tile_nodes=case.tiles[1])
    s = vcx.Solver(gm, case.vcx_phys(precision), case.E)
    s.upload(case.U)
    return gm, s


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name,nsteps", [("ns3d-sp9", 200), ("ns3d-sp2-smalltile", 200),
                                         ("ns2d-sp2-open", 100)])
def test_multi_species_trajectories_track_the_oracle(name, nsteps, precision):
    """Multi-species runs of up to 200 steps (node-gradient pass, staged
    rows, every node finished in the update pass) against the oracle at
    checkpoints: FP64 to 1e-12, mixed to its stated 1e-4.  (The 2D open case
    stops at 100 steps: beyond, its coarse open-boundary flow becomes
    unstable in the oracle too.)"""
    case = make_case(name)
    gm, s = _setup(case, precision)
    om = oracle.OracleMesh(case.mesh)
    ph = case.oracle_phys()
    U, done = case.U.copy(), 0
    tol = MIXED_TOL if precision else FP64_TOL
    for chk in (10, nsteps // 2, nsteps):
        U, *_ = om.step(ph, U, nsteps=chk - done)
        s.step(chk - done)
        done = chk
        err = state_err(case, s.download(), U)
        print(f"{name} prec={precision} step {chk}: state err {err.max():.2e}", flush=True)
        assert err.max() <= tol, (chk, err)


@pytest.mark.parametrize("name", ["shock1d-roe-vanleer", "sod-hllc"])
def test_shock_tubes_to_t_end(name):
    """The shock tubes of Sec. "One-dimensional shock tube" to t = 0.2: the
    oracle must have taken the entropy-fix branch (Roe) and the GPU must
    match its state and step count."""
    case = make_case(name)
    om = oracle.OracleMesh(case.mesh)
    gm, s = _setup(case)
    oracle.flux_branches()
    Uo, to, _, no = om.step(case.oracle_phys(), case.U, nsteps=100000, t_end=0.2)
    br = oracle.flux_branches()
    if case.scheme["flux"] == "roe":
        assert br["roe_entropy_fix"] > 0
    tg, _ = s.step(100000, t_end=0.2)
    assert s.steps_done() == no and tg == pytest.approx(0.2, abs=1e-14)
    err = state_err(case, s.download(), Uo)
    print(f"{name} to t=0.2 in {no} steps: state err {err}")
    assert err.max() <= FP64_TOL


def _bench_kind_case(key: str, tiles):
    """A mesh and state of the kind a tune-cache key describes, smaller than
    the benchmark's but spanning many tiles of the cached size."""
    parts = key.split("|")
    nd = int(parts[1][2:])
    model = int(parts[2][5:])
    nsp = int(parts[4][3:])
    if nd == 2 and model == 1:
        m = wl.dd_streamer_mesh(90, 60)
        n, E = wl.dd_fields(m, sigma=2e-3)
        return cases.Case(f"dd2d-bench-tiles{tiles}", m, n, E, dict(cases.DD2), tiles=tuple(tiles))
    if nd == 3 and model == 0:
        m = wl.kuhn_tet_mesh(14, 14, 13, jitter=0.1, seed=11)
        U = wl.euler_blob_state(m, nblobs=8, amp=0.1, sigma=0.2)
        return cases.Case(f"euler3d-bench-tiles{tiles}", m, U, None,
                          dict(model="gas", flux="roe", limiter="vanleer", rk=2), tiles=tuple(tiles))
    if nd == 3 and model == 2:
        mix = wl.synthetic_mixture(nsp, seed=3)
        m = wl.kuhn_tet_mesh(9, 8, 8, 0.01, 0.008, 0.008, jitter=0.1, seed=8)
        U = wl.ns_state(m, mix, lattice=4, seed=6)
        return cases.Case(f"ns3d-bench-tiles{tiles}", m, U, None,
                          dict(model="ns", flux="hllc", limiter="vanleer", rk=2, nspecies=nsp,
                               mixture=mix), tiles=tuple(tiles))
    raise KeyError(key)


_CACHE = autotune.load_cache(autotune.DEFAULT_CACHE)


@pytest.mark.parametrize("key", sorted(_CACHE))
def test_benchmark_tilings_match_the_oracle(key):
    """Every tile size the benchmark takes from the shipped tuning cache, on a
    mesh of the same kind: residual and two steps against the oracle (FP64 to
    1e-12, mixed to its stated 1e-4)."""
    tiles = _CACHE[key]["tiles"]
    precision = int(key.split("|")[5][4:])
    case = _bench_kind_case(key, tiles)
    gm, s = _setup(case, precision)
    info = gm.info()
    assert info["max_tile_cells"] <= tiles[0] and info["ntiles"] >= 8
    om = oracle.OracleMesh(case.mesh)
    ph = case.oracle_phys()
    dt = om.timestep(ph, case.U, case.E)
    err = normwise(s.residual(dt), om.residual(ph, case.U, case.E, dt),
                   om.flux_scale(ph, case.U, case.E, dt))
    Uo, *_ = om.step(ph, case.U, case.E, nsteps=2)
    s.step(2)
    serr = state_err(case, s.download(), Uo)
    tol = MIXED_TOL if precision else FP64_TOL
    print(f"{key} tiles {tiles}: residual err {err.max():.2e}, 2-step state err {serr.max():.2e}")
    assert err.max() <= tol and serr.max() <= tol


def _envelope():
    """Oracle-only roundoff envelope per checkpoint (tests/golden)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "dd2d_roundoff_envelope.txt")
    env = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            env[int(k)] = float(v)
    return env


def test_full_drift_diffusion_workload_1000_steps():
    """The 200k-cell drift-diffusion workload for its full 1000 steps in the
    benchmark's tiling, checked every 100 steps against the oracle, with the
    first checkpoint above 1e-12 printed.  The limited Lax-Wendroff face
    value jumps where the edge jump b changes sign, so a rounding difference
    can move the trajectory by more than rounding; the oracle itself does so
    when its input is perturbed by 1e-15 (tests/golden/
    dd2d_roundoff_envelope.txt).  Bar per checkpoint: 1e-12, or ten times
    that oracle-only envelope where the envelope exceeds 1e-13."""
    m = wl.dd_streamer_mesh()
    n, E = wl.dd_fields(m)
    key = next(k for k in _CACHE if "|nd2|model1|" in k and "|prec0|" in k)
    case = cases.Case("dd2d-full-1000", m, n, E, dict(cases.DD2), tiles=tuple(_CACHE[key]["tiles"]))
    gm, s = _setup(case)
    om = oracle.OracleMesh(m)
    ph = case.oracle_phys()
    env = _envelope()
    Uo, t = n.copy(), 0.0
    first_above, worst = None, 0.0
    for chk in range(1, 11):
        Uo, t, _, no = om.step(ph, Uo, E, nsteps=100, t0=t)
        assert no == 100
        tg, _ = s.step(100)
        assert tg == pytest.approx(t, rel=1e-12)
        err = state_err(case, s.download(), Uo).max()
        worst = max(worst, err)
        e = env[100 * chk]
        bar = FP64_TOL if e <= 1e-13 else max(FP64_TOL, 10.0 * e)
        print(f"dd2d full, step {100 * chk}: state err {err:.3e} (oracle roundoff envelope {e:.1e}, "
              f"bar {bar:.1e})", flush=True)
        if err > FP64_TOL and first_above is None:
            first_above = 100 * chk
        assert err <= bar
    print(f"dd2d full 1000 steps: worst {worst:.3e}, first checkpoint above 1e-12: {first_above}")
