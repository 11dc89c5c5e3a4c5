"""Serving: continuous batching of independent solves.  Requests of uneven
size and of two schemes arrive while others run; each result must be the
same, bit for bit, as the same solve run alone with vcx_step (whose parity
with the oracle the parity tests establish), and admission must respect the
slot count and the device-memory budget."""
import time

import numpy as np
import pytest

import cases
from paper_2201_01291_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2201_01291_amd import vcx  # noqa: E402

GAS = dict(model="gas", flux="hllc", limiter="vanleer", rk=2)


def _request(kind, side, seed):
    """A serving request as in the request stream: periodic unit square."""
    m = wl.tri_rect_mesh(side, side, 1.0, 1.0, jitter=0.2, seed=seed, periodic=True)
    if kind == "gas":
        U = wl.euler_blob_state(m, nblobs=4, amp=0.3, sigma=0.1, seed=seed)
        return cases.Case(f"gas-{side}", m, U, None, dict(GAS))
    n, E = wl.dd_fields(m, sigma=0.1, bump_sigma=0.1, seed=seed)
    return cases.Case(f"dd-{side}", m, n, E, dict(cases.DD2, fourier=0.25))


def _alone(case, gm, nsteps, t_end=0.0, precision=0):
    s = vcx.Solver(gm, case.vcx_phys(precision), case.E)
    s.upload(case.U)
    s.step(nsteps, t_end=t_end)
    return s.download(), s.time()[0]


def _mix(n, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        side = int(rng.integers(8, 60))
        out.append(_request("gas" if k % 2 == 0 else "dd", side, 100 + k))
    return out


@pytest.mark.parametrize("precision,graphs", [(0, True), (1, True), (1, False)])
def test_requests_in_a_mix_match_alone(precision, graphs):
    """Each served result equals the same solve alone, bit for bit, in the
    FP64 path and in the mixed path the benchmark serves (with graph
    replays and with direct launches); mixed results also stay within the
    stated 1e-4 of the FP64 oracle."""
    import oracle
    reqs = _mix(10)
    meshes = [vcx.Mesh(c.mesh) for c in reqs]
    budgets = [int(b) for b in np.random.default_rng(1).integers(5, 40, size=len(reqs))]
    print(f"[serve] mix prec={precision} graphs={graphs}", [c.name for c in reqs], budgets, flush=True)
    ref = [_alone(c, gm, k, precision=precision) for c, gm, k in zip(reqs, meshes, budgets)]
    sv = vcx.Server(hbm_budget=1 << 34, max_slots=16, chunk_steps=4, graphs=graphs)
    ids = []
    for c, gm, k in zip(reqs[:4], meshes[:4], budgets[:4]):
        ids.append(sv.submit(gm, c.vcx_phys(precision), c.U, c.E, nsteps=k))
    assert sv.wait(ids[0], timeout=60)
    # later arrivals join the running batch
    for c, gm, k in zip(reqs[4:], meshes[4:], budgets[4:]):
        ids.append(sv.submit(gm, c.vcx_phys(precision), c.U, c.E, nsteps=k))
    for rid, (U, t), c, k in zip(ids, ref, reqs, budgets):
        assert sv.wait(rid, timeout=120)
        done, st, Us, ts = sv.poll(rid)
        assert done and st == vcx.OK
        assert ts == t
        assert np.array_equal(Us, U)
        if precision and c.mesh.nnodes <= 1200:
            Uo, *_ = oracle.OracleMesh(c.mesh).step(c.oracle_phys(), c.U, c.E, nsteps=k)
            err = cases.state_err(c, Us, Uo)
            print(f"MIXED served {c.name} after {k} steps vs FP64 oracle: {err}")
            assert err.max() <= 1e-4
    st = sv.stats()
    print("[serve] stats", st, flush=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["peak_running"] >= 2 and st["mean_running"] > 1.0
    assert st["resident_bytes"] == 0 and st["running"] == 0
    assert st["peak_resident_bytes"] >= st["idle_bytes"] > 0
    sv.close()


def test_solver_reuse_on_a_shared_mesh():
    """Requests on one mesh with different states and fields reuse finished
    solvers (and their device memory) and still match the alone results."""
    base = _request("dd", 33, 51)
    gm = vcx.Mesh(base.mesh)
    ins = []
    for k in range(6):
        n, E = wl.dd_fields(base.mesh, sigma=0.1, bump_sigma=0.1, seed=60 + k)
        ins.append(cases.Case(f"dd-shared-{k}", base.mesh, n, E, dict(cases.DD2)))
    ref = [_alone(c, gm, 6 + k) for k, c in enumerate(ins)]
    fp = vcx.footprint(gm, base.vcx_phys())
    sv = vcx.Server(hbm_budget=2 * fp, max_slots=2, chunk_steps=4)
    ids = [sv.submit(gm, c.vcx_phys(), c.U, c.E, nsteps=6 + k) for k, c in enumerate(ins)]
    for rid, (U, t) in zip(ids, ref):
        assert sv.wait(rid, timeout=60)
        done, st, Us, ts = sv.poll(rid)
        assert st == vcx.OK and ts == t and np.array_equal(Us, U)
    s = sv.stats()
    assert s["peak_resident_bytes"] <= 2 * fp and s["running"] == 0
    assert s["resident_bytes"] == 0 and s["idle_bytes"] > 0
    sv.close()


def test_admission_by_memory_budget_and_slots():
    reqs = _mix(6, seed=3)
    meshes = [vcx.Mesh(c.mesh) for c in reqs]
    fp = [vcx.footprint(gm, c.vcx_phys()) for c, gm in zip(reqs, meshes)]
    budget = sorted(fp)[-1] + sorted(fp)[-2]      # at most two of the largest at once
    ref = [_alone(c, gm, 12) for c, gm in zip(reqs, meshes)]
    sv = vcx.Server(hbm_budget=budget, max_slots=3, chunk_steps=5)
    ids = [sv.submit(gm, c.vcx_phys(), c.U, c.E, nsteps=12) for c, gm in zip(reqs, meshes)]
    for rid, (U, t) in zip(ids, ref):
        assert sv.wait(rid, timeout=120)
        done, st, Us, ts = sv.poll(rid)
        assert st == vcx.OK and np.array_equal(Us, U)
    s = sv.stats()
    assert s["peak_resident_bytes"] <= budget and s["peak_running"] <= 3
    sv.close()


def test_oversized_and_unstable_requests_fail_alone():
    good = _request("dd", 30, 7)
    big = _request("gas", 40, 8)
    bad = _request("gas", 20, 9)
    Ubad = bad.U.copy()
    Ubad[3, 11] = 1e-4          # energy below kinetic energy: negative pressure
    gms = [vcx.Mesh(c.mesh) for c in (good, big, bad)]
    ref = _alone(good, gms[0], 9)
    budget = vcx.footprint(gms[0], good.vcx_phys()) + vcx.footprint(gms[2], bad.vcx_phys())
    assert vcx.footprint(gms[1], big.vcx_phys()) > budget
    sv = vcx.Server(hbm_budget=budget, max_slots=4, chunk_steps=4)
    i_big = sv.submit(gms[1], big.vcx_phys(), big.U, nsteps=5)
    i_bad = sv.submit(gms[2], bad.vcx_phys(), Ubad, nsteps=5)
    i_good = sv.submit(gms[0], good.vcx_phys(), good.U, good.E, nsteps=9)
    for rid in (i_big, i_bad, i_good):
        assert sv.wait(rid, timeout=60)
    assert sv.poll(i_big)[1] == vcx.E_OOM
    done, st, Ub, _ = sv.poll(i_bad)
    assert st == vcx.E_UNSTABLE and np.array_equal(Ub, Ubad)   # last good state
    done, st, Ug, _ = sv.poll(i_good)
    assert st == vcx.OK and np.array_equal(Ug, ref[0])
    with pytest.raises(vcx.VcxError):
        sv.poll(i_good)                  # a result is handed over once
    sv.close()


def test_end_times_and_single_slot():
    reqs = [_request("gas", 24, 21), _request("gas", 13, 22)]
    meshes = [vcx.Mesh(c.mesh) for c in reqs]
    ref = [_alone(c, gm, 100000, t_end=te) for c, gm, te in zip(reqs, meshes, (0.02, 0.035))]
    sv = vcx.Server(hbm_budget=1 << 32, max_slots=1, chunk_steps=16)
    ids = [sv.submit(gm, c.vcx_phys(), c.U, nsteps=100000, t_end=te)
           for c, gm, te in zip(reqs, meshes, (0.02, 0.035))]
    for rid, (U, t) in zip(ids, ref):
        assert sv.wait(rid, timeout=120)
        done, st, Us, ts = sv.poll(rid)
        assert st == vcx.OK and ts == t and np.array_equal(Us, U)
    assert sv.stats()["peak_running"] == 1
    sv.close()


def test_shutdown_cancels_queued_requests():
    c = _request("dd", 40, 31)
    gm = vcx.Mesh(c.mesh)
    sv = vcx.Server(hbm_budget=1 << 32, max_slots=1, chunk_steps=8)
    ids = [sv.submit(gm, c.vcx_phys(), c.U, c.E, nsteps=200) for _ in range(4)]
    time.sleep(0.05)
    stats = sv.stats()
    assert stats["submitted"] == 4
    lib = vcx.lib()
    h, sv.h = sv.h, None
    assert lib.vcx_server_destroy(h) == vcx.OK     # finishes the running one, cancels the rest


def test_graph_replay_matches_direct_launches():
    """Batch steps replayed from a captured graph against direct launches,
    over several calls with ordinary single steps in between."""
    reqs = [_request("dd", 35, 41), _request("dd", 17, 42), _request("dd", 50, 43)]
    gms = [vcx.Mesh(c.mesh) for c in reqs]
    A = [vcx.Solver(gm, c.vcx_phys(), c.E) for c, gm in zip(reqs, gms)]
    B = [vcx.Solver(gm, c.vcx_phys(), c.E) for c, gm in zip(reqs, gms)]
    for s, c in zip(A + B, reqs + reqs):
        s.upload(c.U)
    for rep, k in enumerate((7, 10, 3)):
        vcx.solve_batch(A, [k, k + 1, k + 2], graphs=True)
        vcx.solve_batch(B, [k, k + 1, k + 2], graphs=False)
        for a, b in zip(A, B):
            assert np.array_equal(a.download(), b.download()), rep
            assert a.time() == b.time()
        A[0].step(1)
        B[0].step(1)
