"""Batched execution: several independent solves advanced by one launch per
kernel must give, per solve, bit for bit the result of the same solve run
alone (which the parity tests compare with the oracle), with its own time
step, step budget and end time."""
import numpy as np
import pytest

import oracle
from cases import make_case, state_err
from paper_2201_01291_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2201_01291_amd import vcx  # noqa: E402


# Mixed precision (FP32 reconstruction, limiter and flux; FP64 gradients,
# accumulation and update): a batch member must still equal its alone run bit
# for bit, and its state after a few steps stays within this norm-wise bound
# of the FP64 oracle (the stated residual bound of the mixed path).
MIXED_TOL = 1e-4


def _solver(case, mesh=None, U=None, precision=0):
    gm = mesh or vcx.Mesh(case.mesh, tile_cells=case.tiles[0], tile_nodes=case.tiles[1])
    s = vcx.Solver(gm, case.vcx_phys(precision), case.E)
    s.upload(case.U if U is None else U)
    return gm, s


def _alone(case, nsteps, t_end=0.0, U=None, precision=0):
    gm, s = _solver(case, U=U, precision=precision)
    s.step(nsteps, t_end=t_end)
    return s.download(), s.time(), s.steps_done()


def _dd_case(nx, ny, seed):
    import cases
    m = wl.tri_rect_mesh(nx, ny, nx * 1e-3, ny * 1e-3, jitter=0.2, seed=seed, periodic=True)
    n, E = wl.dd_fields(m, sigma=3e-3, seed=seed)
    return cases.Case(f"dd-{nx}x{ny}", m, n, E, dict(cases.DD2))


PREC_GRAPHS = [(0, True), (1, True), (1, False)]


@pytest.mark.parametrize("precision,graphs", PREC_GRAPHS)
def test_batch_drift_diffusion_members_match_alone(precision, graphs):
    """Three meshes of different sizes and step budgets in one batch, in both
    precisions, through graph replays and direct launches."""
    cs = [_dd_case(40, 25, 1), _dd_case(13, 9, 2), _dd_case(61, 47, 3)]
    budgets = [7, 3, 11]
    print(f"[batch] dd members {[c.mesh.nnodes for c in cs]} prec={precision} graphs={graphs}",
          flush=True)
    ref = [_alone(c, k, precision=precision) for c, k in zip(cs, budgets)]
    keep = [_solver(c, precision=precision) for c in cs]
    ss = [s for _, s in keep]
    vcx.solve_batch(ss, budgets, graphs=graphs)
    for s, (U, tt, n), k in zip(ss, ref, budgets):
        assert s.steps_done() == n == k
        assert s.time() == tt
        assert np.array_equal(s.download(), U)
    if precision:
        c, k, s = cs[2], budgets[2], ss[2]
        Uo, *_ = oracle.OracleMesh(c.mesh).step(c.oracle_phys(), c.U, c.E, nsteps=k)
        err = state_err(c, s.download(), Uo)
        print(f"MIXED batch dd state err after {k} steps: {err}")
        assert err.max() <= MIXED_TOL


@pytest.mark.parametrize("precision,graphs", PREC_GRAPHS)
@pytest.mark.parametrize("name", ["sod-hllc", "euler3d-roe", "euler3d-hllc-sp9", "ns2d-sp2-open",
                                  "dd3d-sweby", "euler2d-mach2.5-hllc", "euler3d-mach2-roe"])
def test_batch_single_member_matches_alone_and_oracle(name, precision, graphs):
    case = make_case(name)
    print(f"[batch] single {name} prec={precision} graphs={graphs}", flush=True)
    U, tt, n = _alone(case, 4, precision=precision)
    _, s = _solver(case, precision=precision)
    vcx.solve_batch([s], [4], graphs=graphs)
    assert s.steps_done() == n == 4 and s.time() == tt
    Ub = s.download()
    assert np.array_equal(Ub, U)
    Uo, to, _, no = oracle.OracleMesh(case.mesh).step(case.oracle_phys(), case.U, case.E, nsteps=4)
    err = state_err(case, Ub, Uo)
    if precision:
        print(f"MIXED batch state err {name} after 4 steps: {err}")
    assert err.max() <= (MIXED_TOL if precision else 1e-12)


def test_batch_end_times_and_shared_mesh():
    """Gas members with their own end times, two of them on one mesh object
    with different initial states; one member with a zero budget."""
    c1 = make_case("sod-hllc")
    c2 = make_case("euler2d-roe-sp2")
    c2b = make_case("euler2d-roe-sp2")
    U2b = c2b.U.copy()
    U2b[0] *= 1.1
    U2b[-1] *= 1.2
    # different scheme from sod (Roe vs HLLC) -> separate batches per scheme
    gm2 = vcx.Mesh(c2.mesh)
    ref_a = _alone(c2, 1000, t_end=0.05)
    ref_b = _alone(c2b, 1000, t_end=0.08, U=U2b)
    _, sa = _solver(c2, mesh=gm2)
    _, sb = _solver(c2b, mesh=gm2, U=U2b)
    _, sc = _solver(c2, mesh=gm2)
    vcx.solve_batch([sa, sb, sc], [1000, 1000, 0], [0.05, 0.08, 0.0])
    for s, (U, tt, n) in ((sa, ref_a), (sb, ref_b)):
        assert s.steps_done() == n and s.time() == tt
        assert np.array_equal(s.download(), U)
    assert sc.steps_done() == 0 and np.array_equal(sc.download(), c2.U)
    assert sa.time()[0] == pytest.approx(0.05, abs=1e-15)
    # the Sod tube to t = 0.2 through the batch path against the oracle
    print("[batch] sod to t_end", flush=True)
    _, s1 = _solver(c1)
    vcx.solve_batch([s1], [100000], [0.2])
    Uo, to, _, no = oracle.OracleMesh(c1.mesh).step(c1.oracle_phys(), c1.U, nsteps=100000, t_end=0.2)
    assert s1.steps_done() == no
    assert state_err(c1, s1.download(), Uo).max() <= 1e-12


def test_batch_after_single_steps_continues_the_trajectory():
    """Members may be at different parities of their double buffer."""
    cs = [_dd_case(40, 25, 5), _dd_case(30, 21, 6)]
    ref = [_alone(c, 9) for c in cs]
    keep = [_solver(c) for c in cs]
    ss = [s for _, s in keep]
    ss[0].step(3)
    ss[1].step(4)
    vcx.solve_batch(ss, [6, 5])
    for s, (U, tt, _) in zip(ss, ref):
        assert s.time() == tt
        assert np.array_equal(s.download(), U)
    ss[0].step(2)           # and single steps after a batch
    U11 = _alone(cs[0], 11)[0]
    assert np.array_equal(ss[0].download(), U11)


def test_batch_unstable_member_is_isolated():
    cs = [_dd_case(40, 25, 7), _dd_case(20, 15, 8)]
    ref = _alone(cs[0], 6)
    keep = [_solver(c) for c in cs]
    ss = [s for _, s in keep]
    bad = cs[1].U.copy()
    bad[1, 10] = np.nan
    ss[1].upload(bad)
    with pytest.raises(vcx.VcxError) as e:
        vcx.solve_batch(ss, [6, 6])
    assert e.value.code == vcx.E_UNSTABLE
    assert np.array_equal(ss[0].download(), ref[0]) and ss[0].steps_done() == 6
    assert ss[1].steps_done() == 0
    with pytest.raises(vcx.VcxError):
        ss[1].step(1)       # stays failed until a new state is uploaded
    ss[1].upload(cs[1].U)
    ss[1].step(1)


def test_batch_argument_errors():
    c = _dd_case(13, 9, 2)
    _, s = _solver(c)
    cg = make_case("sod-hllc")
    _, g = _solver(cg)
    for args in (([s, s], [1, 1]), ([s, g], [1, 1]), ([s], [-1])):
        with pytest.raises(vcx.VcxError) as e:
            vcx.solve_batch(*args)
        assert e.value.code == vcx.E_ARG
    with pytest.raises(vcx.VcxError):
        vcx.solve_batch([], [])


def test_batch_members_with_different_tile_sizes_match_alone():
    """Meshes partitioned with different tile sizes (as the autotuner may pick
    per mesh) in one batch: the launch takes the largest block and LDS, and
    each member still gets the bits of its own solve."""
    import cases
    tiles = [(128, 96), (256, 192), (384, 288)]
    cs = [_dd_case(40, 25, 11), _dd_case(33, 21, 12), _dd_case(52, 37, 13)]
    g3 = make_case("euler3d-roe")
    print("[batch] dd members with tiles", tiles, flush=True)
    runs = []
    for c, t in zip(cs, tiles):
        c = cases.Case(c.name, c.mesh, c.U, c.E, c.scheme, tiles=t)
        runs.append((c, _alone(c, 5)))
    keep = [_solver(c) for c, _ in runs]
    ss = [s for _, s in keep]
    vcx.solve_batch(ss, [5] * len(ss))
    for s, (_, (U, tt, n)) in zip(ss, runs):
        assert s.steps_done() == n == 5 and s.time() == tt
        assert np.array_equal(s.download(), U)
    print("[batch] euler3d members with tiles (64, 48) and (128, 96)", flush=True)
    gs = [cases.Case(g3.name, g3.mesh, g3.U, g3.E, g3.scheme, tiles=t) for t in ((64, 48), (128, 96))]
    ref = [_alone(c, 3) for c in gs]
    keep = [_solver(c) for c in gs]
    ss = [s for _, s in keep]
    vcx.solve_batch(ss, [3, 3])
    for s, (U, tt, n) in zip(ss, ref):
        assert s.steps_done() == n == 3 and s.time() == tt
        assert np.array_equal(s.download(), U)
