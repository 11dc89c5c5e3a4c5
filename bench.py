"""Benchmark of the vertex-centred explicit residual on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ns3d]

Headline workload (default, `ns3d`): 3D multi-species Navier-Stokes transport
on a periodic 1 cm cube, Kuhn split of 110^3 jittered (10%) cubes: 7,986,000
tetrahedra, 1,331,000 nodes, 47,916,000 cell-edges.  Nine synthetic species
with Dirichlet(1) mass fractions and T ~ U(300, 2000) K drawn on a periodic
8^3 lattice and interpolated to the nodes, p = 101325 Pa, u = (100, 50, 25)
m/s; HLLC + van Leer MUSCL + central viscous, heat and species diffusion,
RK2, CFL 0.5, FP64.  The headline `value` is its FP64 throughput; the mixed
path (FP32 reconstruction, limiter and flux, FP64 accumulation) is reported
beside it with its drift from FP64.

Secondary legs (same JSON line): the 3D Euler workload (2M tets, Roe + van
Leer, RK2) and the 2D drift-diffusion workload (200k triangles, LLW +
diffusion, RK1) in both precisions; an HBM-resident size sweep of the 2D
drift-diffusion family (up to 28.8M cells) and of the 3D Euler family (up to
16M tets); the Poisson solve; the serving stream (continuous batching,
mixed precision) beside a measured one-at-a-time FP64 baseline.

One step = CFL time step + K x (nodal gradients + cell-edge fluxes with the
deterministic gather + RK stage update), all on the GPU.  Metric: Mfaces/s =
cell-edge fluxes per residual evaluation x residual evaluations per second /
1e6 (K residual evaluations per RK-K step).

Roofline: the dominant kernel of the headline (the flux tile pass), its
average duration from HIP events recorded around every launch on the
solver's stream; algorithmic bytes (every array once per launch) and
algorithmic flops (per-face count measured with the FP64/FP32 VALU
instruction counters) give the HBM and VALU fractions; the binding one is
`roofline.frac`.  `cpu_baseline` is the FP64 C oracle on a bounded sample of
the headline workload (the same recipe on a smaller cube), one process and
one process per core, timed before the GPU is touched.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
VALU_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}   # dense vector peaks
KERNEL_SOURCES = ("paper_2201_01291_amd/csrc/vcx_kernels.h", "paper_2201_01291_amd/csrc/vcx_device.h",
                  "paper_2201_01291_amd/csrc/vcx_internal.h")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_record(record_file, tag, kernel):
    """Fields of a `<tag>-record:` line for `kernel` in a committed counter
    summary under profiles/, or None when it is missing or the kernel
    sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", record_file)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith(f"{tag}-record:"):
            kv = dict(x.split("=", 1) for x in line.split()[1:])
            if kv.get("kernel") == kernel and kv.get("source") == kernel_source_hash():
                return kv
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ns3d", choices=["ns3d", "euler3d", "dd2d"])
    ap.add_argument("--only", action="store_true", help="the headline workload only (no other legs)")
    ap.add_argument("--secondary", default="euler3d,dd2d", help="secondary workloads")
    ap.add_argument("--tiles", default="", help="CELLS,NODES per tile for the headline workload")
    ap.add_argument("--latency-seconds", type=float, default=2.0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-procs", type=int, default=0, help="oracle processes (0: one per core, <= 16)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the profiled passes")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-pool", type=int, default=16)
    ap.add_argument("--serve-steps", type=int, default=100)
    ap.add_argument("--serve-budget-gb", type=float, default=8.0)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-graphs", type=int, default=0, help="server replays captured graphs")
    ap.add_argument("--serve-only", action="store_true", help="run the serving leg only")
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="arrival rate as a fraction of the measured batched capacity")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with plain 256 MiB device copies (counter calibration)")
    ap.add_argument("--sweep-dd", default="1200x750,2400x1500,4800x3000",
                    help="NXxNY sizes of the drift-diffusion family (h = 50 um); empty: none")
    ap.add_argument("--sweep-euler", default="88x88x86,140x140x136",
                    help="NXxNYxNZ cube counts of the 3D Euler family (h = 1/70); empty: none")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--sweep-only", action="store_true", help="run the size sweep only")
    ap.add_argument("--no-poisson", action="store_true", help="skip the Poisson leg")
    ap.add_argument("--autotune", action="store_true",
                    help="time the candidate tile sizes when the tuning cache has no entry")
    ap.add_argument("--cpu-worker", default="", help=argparse.SUPPRESS)
    return ap.parse_args()


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

class Workload:
    """Mesh, initial state, physics and the per-launch algorithmic figures
    of one benchmark workload."""

    def __init__(self, name, scale=None):
        from paper_2201_01291_amd import vcx, workloads as wl
        self.name = name
        self.E = None
        self.primitive = False
        if name == "dd2d":
            nx, ny = scale or (400, 250)
            m = wl.dd_streamer_mesh(nx, ny)
            self.U0, self.E = wl.dd_fields(m)
            sp = wl.DD_STREAMER_SPECIES
            self.vphys = lambda prec: vcx.physics(
                model=vcx.MODEL_DRIFT_DIFFUSION, limiter=vcx.LIM_MINMOD, rk_stages=1, nspecies=2,
                precision=prec, beta=1.0, cfl=0.5, fourier=0.25, z=[s.z for s in sp],
                mu=[s.mu for s in sp], D=[s.D for s in sp])
            self.cfg = dict(workload=f"dd2d-streamer: periodic {nx}x{ny} jittered (20%) triangles, "
                                     "2 charged species, LLW-minmod + central diffusion, RK1",
                            species=2, residuals_per_step=1)
            N, M = m.nnodes, m.ncells
            # fused gradient + flux pass: reads U, x, E, 1/V, dx_min per node
            # and the cell topology (3 x u16 local vertices + u32 periodic
            # code), writes U
            self.bytes_flux = {p: N * 8 * (2 + 2 + 2 + 1 + 1 + 2) + M * (3 * 2 + 4) for p in (0, 1)}
            self.flops_face_est = 120
            self.flux_kernel = {0: "k_fused<2,2,1,0,double>", 1: "k_fused<2,2,1,0,float>"}
            self.record = "dd2d_streamer_200k"
        elif name == "euler3d":
            nx, ny, nz = scale or (70, 70, 68)
            m = wl.euler3d_mesh(nx, ny, nz)
            self.U0 = wl.euler_blob_state(m)
            self.vphys = lambda prec: vcx.physics(model=vcx.MODEL_GAS, flux=vcx.FLUX_ROE,
                                                  limiter=vcx.LIM_VANLEER, rk_stages=2, precision=prec,
                                                  cfl=0.5)
            self.cfg = dict(workload=f"euler3d: periodic Kuhn {nx}x{ny}x{nz} jittered (10%) tets, "
                                     "8 density/pressure blobs on Mach 0.3, Roe + van Leer, RK2",
                            residuals_per_step=2)
            N, M = m.nnodes, m.ncells
            nr, nd, nv = 6, 3, 5
            # flux pass: reads W, G, x, U^n, 1/V, dx_min per node and the
            # cell topology (4 x u16 local vertices + u32 periodic code),
            # writes W
            self.bytes_flux = {p: N * 8 * (nr + nr * nd + nd + nv + 2 + nr) + M * (4 * 2 + 4) for p in (0, 1)}
            self.flops_face_est = 400
            self.flux_kernel = {0: "k_flux_gas<3,0,1,double,false,false,4>",
                                1: "k_flux_gas<3,0,1,float,false,false,4>"}
            self.record = "euler3d_2m"
        elif name == "ns3d":
            n = scale or 110
            mix = wl.synthetic_mixture(9, seed=3)
            m = wl.ns3d_mesh(n)
            self.U0 = wl.ns_primitive_state(m, mix, lattice=8, seed=4)
            self.primitive = True
            self.vphys = lambda prec: vcx.physics(model=vcx.MODEL_NAVIER_STOKES, flux=vcx.FLUX_HLLC,
                                                  limiter=vcx.LIM_VANLEER, rk_stages=2, nspecies=9,
                                                  precision=prec, cfl=0.5, fourier=0.25, mixture=mix)
            self.mix = mix
            T = self.U0[4]
            self.cfg = dict(workload=f"ns3d: periodic 1 cm cube, Kuhn {n}^3 jittered (10%) tets, 9 "
                                     "synthetic species, Dirichlet(1) Y and T ~ U(300, 2000) K on an 8^3 "
                                     "lattice, p = 101325 Pa, HLLC + van Leer + central viscous/heat/"
                                     "species diffusion, RK2",
                            species=9, residuals_per_step=2,
                            T_range_K=[round(float(T.min()), 1), round(float(T.max()), 1)])
            N, M = m.nnodes, m.ncells
            nrow = 15 + 13 + 21       # conserved + p, primitives, transport/thermo aux
            ng = (15 + 13) * 3        # gradients of the reconstructed rows and primitives
            # rows the flux pass reads: conserved + p, gamma, primitives and
            # mu, lambda (FP64, which forms D_k and h_s,k from them) or every
            # transport/thermo row (mixed); it writes every row of the new state
            rows_read = {0: 15 + 1 + 13 + 2, 1: 15 + 1 + 13 + 20}
            self.bytes_flux = {p: N * 8 * (rows_read[p] + ng + 3 + 14 + 2 + nrow) + M * (4 * 2 + 4)
                               for p in (0, 1)}
            self.flops_face_est = 900
            self.flux_kernel = {0: "k_flux_ns<3,9,double,false>", 1: "k_flux_ns<3,9,float,false>"}
            self.record = "ns3d_8m"
        else:
            raise ValueError(name)
        self.mesh = m
        self.cfg.update(cells=m.ncells, nodes=m.nnodes, faces=m.nfaces)
        self.faces_per_step = m.nfaces * self.cfg["residuals_per_step"]

    def upload(self, s, U=None):
        if U is not None:
            s.upload(U)
        elif self.primitive:
            s.upload_primitive(self.U0)
        else:
            s.upload(self.U0)


def oracle_sample(name):
    """(mesh, conserved state, field, oracle physics, faces per step, what)
    of the bounded CPU sample: the workload's recipe on a smaller mesh."""
    import oracle
    from paper_2201_01291_amd import workloads as wl
    if name == "ns3d":
        n = 30
        mix = wl.synthetic_mixture(9, seed=3)
        m = wl.ns3d_mesh(n)
        ph = oracle.Phys(model=oracle.NAVIER_STOKES, flux=oracle.HLLC, limiter=oracle.VANLEER, rk=2,
                         nspecies=9, cfl=0.5, fourier=0.25, mixture=mix)
        U = oracle.conserved_from_primitive(3, ph, wl.ns_primitive_state(m, mix, lattice=8, seed=4))
        return m, U, None, ph, m.nfaces * 2, f"Kuhn {n}^3 cube ({m.ncells} tets) of the same recipe"
    if name == "euler3d":
        m = wl.euler3d_mesh(35, 35, 34)
        ph = oracle.Phys(model=oracle.GAS, flux=oracle.ROE, limiter=oracle.VANLEER, rk=2, cfl=0.5)
        return m, wl.euler_blob_state(m), None, ph, m.nfaces * 2, f"Kuhn 35x35x34 ({m.ncells} tets)"
    m = wl.dd_streamer_mesh()
    n, E = wl.dd_fields(m)
    sp = wl.DD_STREAMER_SPECIES
    ph = oracle.Phys(model=oracle.DRIFT_DIFFUSION, limiter=oracle.MINMOD, rk=1, nspecies=2, cfl=0.5,
                     fourier=0.25, z=[s.z for s in sp], mu=[s.mu for s in sp], D=[s.D for s in sp])
    return m, n, E, ph, m.nfaces, "the full mesh"


def cpu_worker(spec):
    """Child process: time the oracle on the bounded sample, print JSON."""
    name, seconds = spec.split(":")
    import oracle
    m, U, E, ph, fps, what = oracle_sample(name)
    om = oracle.OracleMesh(m)
    t1 = time.perf_counter()
    U1, *_ = om.step(ph, U, E, nsteps=1)
    one = time.perf_counter() - t1
    nsteps = max(1, int(float(seconds) / max(one, 1e-6)))
    t1 = time.perf_counter()
    om.step(ph, U, E, nsteps=nsteps)
    el = time.perf_counter() - t1
    print(json.dumps(dict(steps=nsteps, seconds=el, mfaces=fps * nsteps / el / 1e6, what=what)))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(a):
    """The oracle on the bounded sample: one process, then one process per
    core (independent copies of the sample, the throughput a perfectly
    scaling parallel oracle would reach).  Runs before the GPU is used."""
    import oracle
    oracle.lib()   # built once here, not by every worker
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    nproc = a.cpu_procs or max(1, min(16, ncores))
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-worker", f"{a.workload}:{a.cpu_seconds}"]
    log(f"cpu baseline: oracle, 1 process on {a.workload}'s sample")
    one = json.loads(subprocess.run(cmd, check=True, capture_output=True, text=True).stdout.strip().splitlines()[-1])
    log(f"cpu baseline: oracle, {nproc} processes")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    procs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True, env=env) for _ in range(nproc)]
    outs = [json.loads(p.communicate()[0].strip().splitlines()[-1]) for p in procs]
    if any(p.returncode for p in procs):
        raise RuntimeError("oracle worker failed")
    agg = sum(o["mfaces"] for o in outs)
    return dict(value=round(one["mfaces"], 3), unit="Mfaces/s", cores=1, kind="oracle",
                sample=(f"{one['steps']} full steps of {one['what']} ({one['seconds']:.1f} s, sequential "
                        f"FP64 C oracle, one process)"),
                all_cores=dict(value=round(agg, 3), unit="Mfaces/s", cores=nproc,
                               sample=f"{nproc} concurrent processes, each the one-process sample"),
                cpu_model=cpu_model(), nproc=ncores)


# ---------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------

def pick_tiles(w, prec, a, override=""):
    from paper_2201_01291_amd import autotune
    if override:
        return tuple(int(v) for v in override.split(",")), "command line"
    tc, tn, src = autotune.pick_tiles(w.mesh, w.vphys(prec), w.upload, w.E, tune_if_missing=a.autotune)
    if src == "default":
        return (0, 0), "library default"
    return (tc, tn), src


def timed_steps(s, k):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(k)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def roofline(w, prec, kern):
    """Roofline entry of the flux pass from its profiled average duration."""
    if "flux" not in kern:
        return None
    us = kern["flux"]["avg_us"]
    dt = "f32" if prec else "f64"
    kname = w.flux_kernel[prec]
    fl = profile_record(f"flops_flux_{w.record}.md", "flops", kname)
    fpf = float(fl["flops_per_face"]) if fl else float(w.flops_face_est)
    flops = fpf * w.mesh.nfaces
    tr = profile_record(f"traffic_flux_{w.record}.md", "traffic", kname)
    nbytes = w.bytes_flux[prec]
    hbm = nbytes / (us * 1e-6) / 1e9
    valu = flops / (us * 1e-6) / 1e12
    ridge = VALU_PEAK_TFLOPS[dt] * 1e12 / (HBM_PEAK_GBS * 1e9)
    alu = flops / nbytes > ridge
    hbm_frac = hbm / HBM_PEAK_GBS
    valu_frac = valu / VALU_PEAK_TFLOPS[dt]
    out = dict(kernel=kname, bound="alu" if alu else "hbm",
               achieved=round(valu, 3) if alu else round(hbm, 1),
               peak=VALU_PEAK_TFLOPS[dt] if alu else HBM_PEAK_GBS,
               unit="TFLOP/s" if alu else "GB/s",
               frac=round(valu_frac if alu else hbm_frac, 4),
               traffic=int(tr["bytes"]) if tr else None,
               avg_us=round(us, 2), alg_bytes_per_launch=int(nbytes),
               alg_flops_per_launch=int(flops), flops_per_face=round(fpf, 1),
               flops_per_face_from="VALU instruction counters" if fl else "estimate",
               hbm=dict(achieved_gbs=round(hbm, 1), peak=HBM_PEAK_GBS, frac=round(hbm_frac, 4)),
               valu=dict(achieved_tflops=round(valu, 3), peak=VALU_PEAK_TFLOPS[dt], dtype=dt,
                         frac=round(valu_frac, 4)))
    return out


def run_workload(w, a, stream, steps, warmup, headline):
    """FP64 and mixed throughput (mixed drift from FP64 after the same
    steps), profiled per-kernel durations, roofline; for the headline also
    the single-step latency and the batch-of-one check."""
    import torch
    from paper_2201_01291_amd import vcx
    res = dict(workload=w.cfg["workload"], cells=w.mesh.ncells, nodes=w.mesh.nnodes,
               faces=w.mesh.nfaces, residuals_per_step=w.cfg["residuals_per_step"])
    meshes, U = {}, {}
    for prec, key in ((0, "fp64"), (1, "mixed")):
        tiles, src = pick_tiles(w, prec, a, a.tiles if headline else "")
        if tiles not in meshes:
            log(f"{w.name}: mesh with tiles {tiles}")
            meshes[tiles] = vcx.Mesh(w.mesh, stream=stream, tile_cells=tiles[0], tile_nodes=tiles[1])
        gm = meshes[tiles]
        s = vcx.Solver(gm, w.vphys(prec), w.E)
        w.upload(s)
        s.step(warmup)
        w.upload(s)
        k = steps
        if not headline:   # about a second of timed work
            k = max(steps, min(5000, int(math.ceil(1.0 / max(timed_steps(s, 2) / 2, 1e-7)))))
            w.upload(s)
        log(f"{w.name}: timing {k} {key} steps")
        el = timed_steps(s, k)
        U[key] = s.download()
        r = dict(value=round(w.faces_per_step * k / el / 1e6, 2), unit="Mfaces/s",
                 ms_per_step=round(el / k * 1e3, 5), steps=k, tiles=list(tiles), tiles_from=src)
        if key == "mixed":
            d = np.abs(U["mixed"] - U["fp64"]).max(axis=1) / np.abs(U["fp64"]).max(axis=1)
            r["drift_vs_fp64_after_steps"] = [float(f"{x:.3e}") for x in d]
        if headline:
            per = el / k
            nl = max(5, min(200, int(a.latency_seconds / max(per, 1e-6))))
            w.upload(s)
            s.step(2)
            ts = []
            for _ in range(nl):
                t1 = time.perf_counter()
                s.step(1)
                ts.append((time.perf_counter() - t1) * 1e3)
            r["latency"] = dict(steps=nl, p50_ms=round(float(np.percentile(ts, 50)), 4),
                                p99_ms=round(float(np.percentile(ts, 99)), 4))
        if headline and key == "fp64":
            w.upload(s)
            vcx.solve_batch([s], [k], graphs=False)
            r["batch_of_one_bitwise_equal"] = bool(np.array_equal(s.download(), U["fp64"]))
        if not a.no_profile:
            w.upload(s)
            s.profile(True)
            s.step(min(k, 50) if not headline else k)
            kern = {}
            for kn in ("gradient", "gradient_shared", "flux", "update"):
                n, ms = s.profile_query(kn)
                if n:
                    kern[kn] = dict(launches=n, avg_us=round(ms / n * 1e3, 3))
            s.profile(False)
            r["kernels"] = kern
            r["roofline"] = roofline(w, prec, kern)
        r["mesh"] = gm.info()
        res[key] = r
        s.close()
    for gm in meshes.values():
        gm.close()
    return res


def size_sweep(a, stream):
    """FP64 throughput and the flux pass's algorithmic HBM / VALU fractions
    at larger sizes of the drift-diffusion and 3D Euler mesh families (fixed
    spacing, larger box), from cache-resident to HBM-resident working sets
    (the device's last-level cache is 256 MB)."""
    from paper_2201_01291_amd import vcx
    out = []
    items = [("dd2d", tuple(int(v) for v in x.lower().split("x"))) for x in a.sweep_dd.split(",") if x]
    items += [("euler3d", tuple(int(v) for v in x.lower().split("x"))) for x in a.sweep_euler.split(",") if x]
    for name, scale in items:
        log(f"sweep: {name} {scale}")
        w = Workload(name, scale)
        tiles, src = pick_tiles(w, 0, a)
        gm = vcx.Mesh(w.mesh, stream=stream, tile_cells=tiles[0], tile_nodes=tiles[1])
        s = vcx.Solver(gm, w.vphys(0), w.E)
        w.upload(s)
        s.step(3)
        w.upload(s)
        k = max(5, min(2000, int(math.ceil(1.0 / max(timed_steps(s, 3) / 3, 1e-7)))))
        w.upload(s)
        el = timed_steps(s, k)
        s.profile(True)
        s.step(min(k, 20))
        kern = {}
        for kn in ("gradient", "gradient_shared", "flux", "update"):
            n, ms = s.profile_query(kn)
            if n:
                kern[kn] = dict(launches=n, avg_us=round(ms / n * 1e3, 2))
        s.profile(False)
        entry = dict(workload=name, cells=w.mesh.ncells, nodes=w.mesh.nnodes, faces=w.mesh.nfaces,
                     steps=k, mfaces=round(w.faces_per_step * k / el / 1e6, 1),
                     ms_per_step=round(el / k * 1e3, 4), tiles=list(tiles), kernels=kern)
        if name == "dd2d" and "gradient" in kern:
            # large drift-diffusion meshes take the separate passes (the
            # node gradient on simplices): the flux pass's own bytes (its
            # gradients read from G), and the whole stage (gradient, any
            # completion, flux) against the stage's minimal bytes (those of
            # the fused pass)
            N, M = w.mesh.nnodes, w.mesh.ncells
            fb = N * 8 * (2 + 2 + 2 + 4 + 2 + 1 + 1 + 2) + M * (3 * 2 + 4)
            us = kern["flux"]["avg_us"]
            st_us = sum(kern[k_]["avg_us"] for k_ in ("gradient", "gradient_shared", "flux") if k_ in kern)
            entry.update(path=("gradient + shared-node completion + flux" if "gradient_shared" in kern
                               else "node gradient + flux"),
                         flux_alg_gbs=round(fb / (us * 1e-6) / 1e9, 1),
                         flux_hbm_frac=round(fb / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                         stage_hbm_frac=round(w.bytes_flux[0] / (st_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4))
        else:
            rf = roofline(w, 0, kern)
            entry.update(path="fused" if name == "dd2d" else "gradient + flux",
                         flux_hbm_frac=rf["hbm"]["frac"], flux_valu_frac=rf["valu"]["frac"],
                         flux_alg_gbs=rf["hbm"]["achieved_gbs"])
        out.append(entry)
        s.close()
        gm.close()
        del w
    return out


def serving_leg(a, stream):
    """Serving workload: requests on 2D meshes of 5e3..2e6 cells (gas: HLLC +
    van Leer, RK2 on the periodic unit square; drift-diffusion as the 2D
    workload), a fixed number of steps each, served by the continuous-
    batching server in mixed precision under a device-memory budget.
    1) capacity: every request submitted at once; 2) open loop: Poisson
    arrivals at a fraction of that capacity, latency from arrival to result;
    3) baseline: the same requests at the same arrival times served one at a
    time, FIFO, on the FP64 single-solve path (vcx_step), measured."""
    from paper_2201_01291_amd import vcx, workloads as wl
    pool, reqs = wl.serving_requests(a.serve_requests, npool=a.serve_pool)
    sp = wl.DD_STREAMER_SPECIES
    log(f"serving: building {len(pool)} x 2 pool meshes")
    meshes = []
    for k, p in enumerate(pool):
        mg = wl.tri_rect_mesh(p["gas_side"], p["gas_side"], 1.0, 1.0, jitter=0.2, seed=1000 + k,
                              periodic=True)
        md = wl.dd_streamer_mesh(p["dd_nx"], p["dd_ny"], seed=2000 + k)
        Ug = wl.euler_blob_state(mg, nblobs=4, amp=0.3, sigma=0.1, seed=k)
        nd_, Ed = wl.dd_fields(md, seed=k)
        meshes.append(dict(gas=(vcx.Mesh(mg, stream=stream), Ug, None, mg.nfaces * 2),
                           dd=(vcx.Mesh(md, stream=stream), nd_, Ed, md.nfaces)))

    def phys(kind, prec):
        if kind == "gas":
            return vcx.physics(model=vcx.MODEL_GAS, flux=vcx.FLUX_HLLC, limiter=vcx.LIM_VANLEER,
                               rk_stages=2, precision=prec, cfl=0.5)
        return vcx.physics(model=vcx.MODEL_DRIFT_DIFFUSION, limiter=vcx.LIM_MINMOD, rk_stages=1,
                           nspecies=2, precision=prec, beta=1.0, cfl=0.5, fourier=0.25,
                           z=[x.z for x in sp], mu=[x.mu for x in sp], D=[x.D for x in sp])

    P = {(k, pr): phys(k, pr) for k in ("gas", "dd") for pr in (vcx.PREC_FP64, vcx.PREC_MIXED)}
    nst = a.serve_steps
    items = []
    for r in reqs:
        gm, U, E, fpr = meshes[r["pool"]][r["kind"]]
        items.append((r["kind"], gm, U * r["scale"], E, fpr * nst))
    total_faces = sum(x[4] for x in items)
    budget = int(a.serve_budget_gb * (1 << 30))

    def serve(todo, arrivals=None):
        sv = vcx.Server(hbm_budget=budget, max_slots=a.serve_slots, chunk_steps=16,
                        graphs=bool(a.serve_graphs))
        ids = []
        t0 = time.perf_counter()
        for k, (kind, gm, U, E, _) in enumerate(todo):
            if arrivals is not None:
                dt = t0 + arrivals[k] - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            ids.append(sv.submit(gm, P[(kind, vcx.PREC_MIXED)], U, E, nsteps=nst))
        done_t = []
        for rid in ids:
            sv.wait(rid)
            done_t.append(time.perf_counter())
        st = sv.stats()
        for rid in ids:
            ok, code, _, _ = sv.poll(rid)
            assert ok and code == vcx.OK, code
        wall = max(done_t) - t0
        sv.close()
        return st, wall

    serve(items[:8])   # warm-up: first launches
    log("serving: capacity run")
    st_c, wall_c = serve(items)
    cap = len(items) / wall_c
    rate = a.serve_load * cap
    gaps = np.array([r["gap"] for r in reqs]) / rate
    arrivals = np.cumsum(gaps) - gaps[0]
    log(f"serving: open loop at {rate:.1f} req/s")
    st_o, wall_o = serve(items, arrivals)

    # baseline: the same arrivals served one at a time (FIFO) on the FP64
    # single-solve path, latency measured from arrival to result
    log("serving: one-at-a-time FP64 baseline, same arrivals")
    lat, svc, step_ms = [], [], []
    t0 = time.perf_counter()
    for arr, (kind, gm, U, E, _) in zip(arrivals, items):
        wait = t0 + arr - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        t1 = time.perf_counter()
        s = vcx.Solver(gm, P[(kind, vcx.PREC_FP64)], E)
        s.upload(U)
        t2 = time.perf_counter()
        s.step(nst)
        t3 = time.perf_counter()
        s.download()
        s.close()
        t4 = time.perf_counter()
        svc.append(t4 - t1)
        step_ms.append((t3 - t2) / nst * 1e3)
        lat.append((t4 - (t0 + arr)) * 1e3)
    wall_b = time.perf_counter() - t0
    svc = np.array(svc)
    base = dict(kind="same arrivals, one request at a time (FIFO), FP64, vcx_step (no batching)",
                throughput_mfaces=round(total_faces / wall_b / 1e6, 1),
                service_capacity_req_s=round(len(items) / svc.sum(), 2),
                latency_p50_ms=round(float(np.percentile(lat, 50)), 2),
                latency_p99_ms=round(float(np.percentile(lat, 99)), 2),
                step_p50_ms=round(float(np.percentile(step_ms, 50)), 4),
                step_p99_ms=round(float(np.percentile(step_ms, 99)), 4))
    cells = np.array([pool[r["pool"]]["cells"] for r in reqs])
    for mm in meshes:
        for v in mm.values():
            v[0].close()
    return dict(
        workload=(f"{len(items)} requests, {nst} steps each, meshes of 5e3..2e6 cells "
                  f"(pool of {len(pool)} sizes per kind), even ids gas HLLC-vanLeer-RK2, odd ids "
                  f"drift-diffusion LLW-minmod-RK1; mixed precision; device budget "
                  f"{a.serve_budget_gb:g} GiB, {a.serve_slots} slots, chunks of 16 steps, "
                  f"{'graph replay' if a.serve_graphs else 'direct launches'}"),
        mean_cells=round(float(cells.mean())),
        capacity_req_s=round(cap, 2),
        capacity_throughput_mfaces=round(total_faces / wall_c / 1e6, 1),
        rate_req_s=round(rate, 2),
        open_loop_throughput_mfaces=round(total_faces / wall_o / 1e6, 1),
        latency_p50_ms=round(st_o["latency_p50_ms"], 2),
        latency_p99_ms=round(st_o["latency_p99_ms"], 2),
        step_p50_ms=round(st_o["step_p50_ms"], 4),
        step_p99_ms=round(st_o["step_p99_ms"], 4),
        mean_running=round(st_o["mean_running"], 2),
        peak_running=int(st_o["peak_running"]),
        peak_resident_gb=round(st_o["peak_resident_bytes"] / (1 << 30), 3),
        baseline=base,
    )


def poisson_leg(a, stream):
    """Poisson solve on the drift-diffusion mesh: space charge e (n_i - n_e)
    / eps0 of the workload's densities with a 20% ion excess in a central
    Gaussian, periodic box (neutralising background), conjugate gradients
    with a two-level (Jacobi plus aggregation) preconditioner to a relative
    residual of 1e-10.  Cold start (zero guess), then steps coupled to the
    field: charge from the solver's state, Poisson solve warm-started from
    the previous potential, E = E_background - grad phi, one drift-diffusion
    step; all of it through the library."""
    import torch
    from paper_2201_01291_amd import vcx, workloads as wl
    m = wl.dd_streamer_mesh()
    n, E0 = wl.dd_fields(m)
    c = m.xyz.mean(axis=1, keepdims=True)
    n[1] *= 1.0 + 0.2 * np.exp(-np.sum((m.xyz - c) ** 2, axis=0) / 4e-6)
    sp = wl.DD_STREAMER_SPECIES
    ph = vcx.physics(model=vcx.MODEL_DRIFT_DIFFUSION, limiter=vcx.LIM_MINMOD, rk_stages=1, nspecies=2,
                     precision=vcx.PREC_FP64, beta=1.0, cfl=0.5, fourier=0.25,
                     z=[s.z for s in sp], mu=[s.mu for s in sp], D=[s.D for s in sp])
    gm = vcx.Mesh(m, stream=stream)
    ps = vcx.Poisson(gm)
    s = vcx.Solver(gm, ph, E0)
    s.upload(n)
    Ebg = np.zeros((2, m.nnodes))
    Ebg[0] = 1e6
    Ebg_d = torch.tensor(Ebg, device="cuda")
    q = torch.empty(m.nnodes, dtype=torch.float64, device="cuda")
    s.charge(out=q)
    tol = 1e-10
    ps.solve(q, tol=tol)               # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi, it_cold, rel = ps.solve(q, tol=tol)
    torch.cuda.synchronize()
    cold = time.perf_counter() - t0
    E = torch.empty((2, m.nnodes), dtype=torch.float64, device="cuda")
    its, times = [], []
    K = 50
    for _ in range(K + 3):
        t1 = time.perf_counter()
        s.charge(out=q)
        phi, it, _ = ps.solve(q, phi0=phi, tol=tol, out=torch.empty_like(phi))
        ps.field(phi, out=E, background=Ebg_d)
        s.set_field(E)
        s.step(1)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        its.append(it)
    times, its = times[3:], its[3:]
    info = ps.info()
    # bytes of one CG iteration, every array once: CSR (rp, col, val), and
    # z, p_old, p_new, q (first half); x, p, r, q, D^-1, r, z, x (second half)
    it_bytes = 4 * (m.nnodes + 1) + 12 * info["nnz"] + 8 * m.nnodes * 12
    ms_it = cold / max(it_cold, 1) * 1e3
    s.close()
    ps.close()
    gm.close()
    return dict(workload="dd2d-streamer mesh (periodic, 100,000 nodes), space charge of the densities "
                         "with a 20% central ion excess, CG with a multilevel preconditioner to relative "
                         "residual 1e-10",
                preconditioner=info, cold_iterations=it_cold, cold_ms=round(cold * 1e3, 3),
                ms_per_iteration=round(ms_it, 4),
                alg_gbs_per_iteration=round(it_bytes / (ms_it * 1e-3) / 1e9, 1),
                coupled_step_ms_p50=round(float(np.percentile(times, 50)) * 1e3, 3),
                coupled_iterations_mean=round(float(np.mean(its)), 2), coupled_steps=K,
                coupled_faces_per_s_M=round(m.nfaces / float(np.percentile(times, 50)) / 1e6, 1))


def main():
    a = parse()
    if a.cpu_worker:
        cpu_worker(a.cpu_worker)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; runs on several GPUs are "
                                   "not supported (the library has no multi-GPU path)", "n_gpus": a.gpus}))
        sys.exit(2)
    cpu = None
    if not (a.no_cpu or a.serve_only or a.sweep_only):
        cpu = cpu_baseline(a)      # before anything touches the GPU
    import torch
    from paper_2201_01291_amd import vcx
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    if a.serve_only:
        print(json.dumps({"serving": serving_leg(a, stream)}))
        return
    if a.sweep_only:
        print(json.dumps({"size_sweep": size_sweep(a, stream)}))
        return
    log(f"building the headline workload {a.workload}")
    w = Workload(a.workload)
    head = run_workload(w, a, stream, a.steps, a.warmup, headline=True)
    cfg = dict(w.cfg)
    del w
    others = {}
    if not a.only:
        for name in [x for x in a.secondary.split(",") if x and x != a.workload]:
            log(f"building the secondary workload {name}")
            ws = Workload(name)
            others[name] = run_workload(ws, a, stream, a.steps, a.warmup, headline=False)
            del ws
    sweep = None if (a.only or a.no_sweep) else size_sweep(a, stream)
    pois = None
    if not (a.only or a.no_poisson):
        log("Poisson leg")
        pois = poisson_leg(a, stream)
    serve = None if (a.only or a.no_serve) else serving_leg(a, stream)

    f64 = head["fp64"]
    cfg["tiles"] = f64["tiles"]
    cfg["tiles_from"] = f64["tiles_from"]
    out = {
        "metric": "Mfaces/s residual throughput",
        "value": f64["value"],
        "unit": "Mfaces/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": f64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": cfg,
        "latency": {"fp64": f64.get("latency"), "mixed": head["mixed"].get("latency")},
        "fp64": f64,
        "mixed": head["mixed"],
        "roofline": f64.get("roofline"),
        "cpu_baseline": cpu,
        "workloads": others,
        "size_sweep": sweep,
        "poisson": pois,
        "serving": serve,
    }
    print(json.dumps(out))
    if a.copy_calibration:
        # a plain copy of known size: reads and writes 256 MiB per launch
        x = torch.rand(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        log(f"copy calibration: {x.numel() * 8} bytes read and written per launch")


if __name__ == "__main__":
    main()
