"""Tile-size autotuner: cache keys and file (CPU), and a measured choice on
the GPU that the parity bar still holds for."""
import json

import numpy as np
import pytest

from paper_2201_01291_amd import autotune, workloads as wl
from paper_2201_01291_amd import vcx as vcx_mod


class _Mesh:
    ndim, ncells = 2, 200000


def _phys(prec=0):
    return vcx_mod.physics(model=vcx_mod.MODEL_DRIFT_DIFFUSION, limiter=vcx_mod.LIM_MINMOD, rk_stages=1,
                           nspecies=2, precision=prec, z=[-1.0, 1.0], mu=[0.04, 0.04], D=[0.1, 0.1])


def test_key_separates_precision_physics_and_size_bucket():
    k = autotune.tune_key("gfx950", 2, _phys(0), 200000)
    assert k != autotune.tune_key("gfx950", 2, _phys(1), 200000)
    assert k != autotune.tune_key("gfx950", 3, _phys(0), 200000)
    assert k == autotune.tune_key("gfx950", 2, _phys(0), 140000)       # same power of two
    assert k != autotune.tune_key("gfx950", 2, _phys(0), 2 ** 19)
    assert autotune.size_bucket(1) == 0 and autotune.size_bucket(2 ** 20 + 5) == 20


def test_cache_round_trip_and_lookup(tmp_path):
    path = str(tmp_path / "cache.json")
    assert autotune.pick_tiles(_Mesh(), _phys(), None, arch="gfx950", cache=path) == (0, 0, "default")
    key = autotune.tune_key("gfx950", 2, _phys(), _Mesh.ncells)
    autotune.store(path, key, dict(tiles=[192, 144], us_per_step=26.0, table=[]))
    autotune.store(path, "other", dict(tiles=[1, 2]))
    assert autotune.pick_tiles(_Mesh(), _phys(), None, arch="gfx950", cache=path) == (192, 144, "cache")
    assert set(json.load(open(path))) == {key, "other"}


def test_shipped_cache_entries_are_candidates():
    cache = autotune.load_cache(autotune.DEFAULT_CACHE)
    assert cache, "the package ships measured tile choices"
    for key, e in cache.items():
        nd = int(key.split("|")[1][2:])
        assert tuple(e["tiles"]) in autotune.CANDIDATES[nd]
        best = min(r[2] for r in e["table"] if r[2] is not None)
        assert e["us_per_step"] == best


@pytest.mark.gpu
def test_tuned_choice_is_measured_cached_and_parity_green(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from cases import normwise
    m = wl.dd_streamer_mesh(60, 40)
    n, E = wl.dd_fields(m)
    ph = _phys()
    path = str(tmp_path / "cache.json")
    cands = [(128, 96), (256, 192)]
    print("[case] autotune dd 60x40", flush=True)
    tc, tn, src = autotune.pick_tiles(m, ph, n, E, cache=path, tune_if_missing=True, candidates=cands,
                                      steps=10, repeats=2)
    assert src == "tuned" and (tc, tn) in cands
    entry = next(iter(json.load(open(path)).values()))
    assert [r[:2] for r in entry["table"]] == [list(c) for c in cands]
    assert autotune.pick_tiles(m, ph, n, E, cache=path) == (tc, tn, "cache")
    s = vcx_mod.Solver(vcx_mod.Mesh(m, tile_cells=tc, tile_nodes=tn), ph, E)
    s.upload(n)
    om = oracle.OracleMesh(m)
    oph = oracle.Phys(model=oracle.DRIFT_DIFFUSION, limiter=oracle.MINMOD, rk=1, nspecies=2, cfl=0.5,
                      fourier=0.25, z=[-1.0, 1.0], mu=[0.04, 0.04], D=[0.1, 0.1])
    dt = om.timestep(oph, n, E)
    err = normwise(s.residual(dt), om.residual(oph, n, E, dt), om.flux_scale(oph, n, E, dt))
    assert err.max() <= 1e-12
