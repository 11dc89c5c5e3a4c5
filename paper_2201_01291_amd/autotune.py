"""Tile-size autotuner for the tile kernels (measured on the GPU, cached).

The tile size (cells and distinct nodes per tile) fixes a mesh's partition
for its lifetime: the block of every tile kernel is derived from it, the
LDS footprint and so the blocks per CU follow from it, and the sum order of
the deterministic gather depends on it.  So it is chosen once per mesh, at
creation, and never per batch: results stay bitwise reproducible for a
given choice (another choice changes the rounding, not the scheme).

`pick_tiles` returns the cached choice for a key (architecture, mesh
dimension, model, flux, species, precision, RK stages, size bucket) or, if
asked to, times every candidate on the caller's mesh and state and stores
the fastest.  A candidate the library rejects (LDS above the CU's limit)
is skipped.  The cache is a JSON file; `DEFAULT_CACHE` is the one shipped
with the package, written by `python -m paper_2201_01291_amd.autotune` on
an MI355X.
"""
from __future__ import annotations

import json
import math
import os
import time

PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(PKG, "tune_cache.json")

# (max cells, max nodes) per tile
CANDIDATES = {
    2: [(128, 96), (192, 144), (256, 192), (384, 288)],
    3: [(64, 48), (96, 72), (128, 96), (192, 144)],
}


def size_bucket(ncells: int) -> int:
    """Meshes within a factor of two share a choice: floor(log2(cells))."""
    return int(math.floor(math.log2(max(int(ncells), 1))))


def tune_key(arch: str, ndim: int, phys, ncells: int) -> str:
    return (f"{arch}|nd{ndim}|model{phys.model}|flux{phys.flux}|nsp{phys.nspecies}|"
            f"prec{phys.precision}|rk{phys.rk_stages}|cells2^{size_bucket(ncells)}")


def load_cache(path: str) -> dict:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def store(path: str, key: str, entry: dict) -> None:
    cache = load_cache(path)
    cache[key] = entry
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
        fh.write("\n")
    os.replace(tmp, path)


def device_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def time_candidate(mesh, physes, U, E, tiles, steps: int, repeats: int):
    """Seconds per step of vcx_step on mesh with the given tiles, best of
    repeats, for each physics in physes (None where the library rejects the
    tile size); the mesh is built once for all of them.  U is the conserved
    state, or a callable that uploads the state into a solver."""
    import torch
    from . import vcx
    try:
        gm = vcx.Mesh(mesh, tile_cells=tiles[0], tile_nodes=tiles[1])
    except vcx.VcxError:
        return [None] * len(physes)
    out = []
    try:
        for phys in physes:
            try:
                s = vcx.Solver(gm, phys, E)
            except vcx.VcxError:
                out.append(None)
                continue
            try:
                put = U if callable(U) else (lambda sv: sv.upload(U))   # state upload
                put(s)
                s.step(max(2, steps // 5))
                torch.cuda.synchronize()
                best = math.inf
                for _ in range(repeats):
                    put(s)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    s.step(steps)
                    torch.cuda.synchronize()
                    best = min(best, (time.perf_counter() - t0) / steps)
                out.append(best)
            finally:
                s.close()
    finally:
        gm.close()
    return out


def tune_many(mesh, physes, U, E=None, candidates=None, steps: int = 50, repeats: int = 3,
              log=None) -> list:
    """Time every candidate tile size for each physics; per physics the
    fastest and the whole table.  log: optional callable taking a line."""
    cands = candidates or CANDIDATES[mesh.ndim]
    times = []
    for c in cands:
        times.append(time_candidate(mesh, physes, U, E, c, steps, repeats))
        if log:
            log(f"tiles {c}: " + ", ".join("rejected" if t is None else f"{t * 1e6:.1f} us/step"
                                           for t in times[-1]))
    res = []
    for q in range(len(physes)):
        table = [[int(c[0]), int(c[1]), None if t[q] is None else round(t[q] * 1e6, 3)]
                 for c, t in zip(cands, times)]
        ok = [r for r in table if r[2] is not None]
        if not ok:
            raise RuntimeError("no candidate tile size is accepted for this mesh and physics")
        best = min(ok, key=lambda r: r[2])
        res.append(dict(tiles=[best[0], best[1]], us_per_step=best[2], table=table, steps=steps,
                        repeats=repeats, ncells=int(mesh.ncells)))
    return res


def tune(mesh, phys, U, E=None, **kw) -> dict:
    """Time every candidate tile size; the fastest and the whole table."""
    return tune_many(mesh, [phys], U, E, **kw)[0]


def pick_tiles(mesh, phys, U, E=None, cache: str = DEFAULT_CACHE, tune_if_missing: bool = False,
               arch: str | None = None, **kw):
    """(tile_cells, tile_nodes, source): the cached choice ("cache"), a fresh
    measurement stored in the cache ("tuned"), or (0, 0, "default") for the
    library's defaults when nothing is cached and tuning was not asked for."""
    arch = arch or device_arch()
    key = tune_key(arch, mesh.ndim, phys, mesh.ncells)
    entry = load_cache(cache).get(key)
    if entry is not None:
        return int(entry["tiles"][0]), int(entry["tiles"][1]), "cache"
    if not tune_if_missing:
        return 0, 0, "default"
    entry = tune(mesh, phys, U, E, **kw)
    store(cache, key, entry)
    return int(entry["tiles"][0]), int(entry["tiles"][1]), "tuned"


# tile candidates for the size-sweep meshes (HBM-resident working sets,
# long launches)
LARGE_CANDIDATES = {
    2: [(128, 96), (192, 144), (256, 192), (384, 288)],
    3: [(96, 72), (128, 96), (192, 144)],
}


def _main():
    """Tune the benchmark workloads of bench.py (both precisions) into a
    cache file: python -m paper_2201_01291_amd.autotune [cache] [workloads],
    a workload as its name or name@size (the sizes of bench.py's sweep, e.g.
    dd2d@4800x3000), the latter over LARGE_CANDIDATES."""
    import sys
    sys.path.insert(0, os.path.dirname(PKG))
    import bench
    path = sys.argv[1] if len(sys.argv) > 1 else DEFAULT_CACHE
    names = sys.argv[2].split(",") if len(sys.argv) > 2 else ["dd2d", "euler3d", "ns3d"]
    arch = device_arch()
    for item in names:
        name, _, size = item.partition("@")
        scale = tuple(int(v) for v in size.lower().split("x")) if size else None
        print(f"[tune] building {item}", flush=True)
        w = bench.Workload(name, scale)
        m = w.mesh
        physes = [w.vphys(0), w.vphys(1)]
        cands = LARGE_CANDIDATES[m.ndim] if scale else None
        entries = tune_many(m, physes, w.upload, w.E, candidates=cands,
                            steps=10 if name == "ns3d" or scale else 50,
                            log=lambda line: print(f"[tune] {item} {line}", flush=True))
        for ph, entry in zip(physes, entries):
            store(path, tune_key(arch, m.ndim, ph, m.ncells), entry)
            print(f"[tune] {item} precision {ph.precision}: {entry['tiles']} {entry['table']}", flush=True)


if __name__ == "__main__":
    _main()
