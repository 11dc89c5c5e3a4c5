"""Benchmark of the vertex-centred explicit residual on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload dd2d]

Workload (default): 2D drift-diffusion of electrons and one positive ion on
a periodic jittered triangular mesh of 200,000 cells (100,000 nodes, 600,000
cell-edges), Gaussian densities peaking at 1e18 m^-3, mobility 0.04 m^2/Vs,
D = 0.1 m^2/s, E from an analytic potential (uniform 1e6 V/m plus a seeded
Gaussian bump), limited Lax-Wendroff (minmod) + central diffusion, RK1, FP64.

One step = CFL time step + nodal gradients + cell-edge fluxes with the
deterministic gather + update, all on the GPU.  Metric: Mfaces/s = cell-edge
fluxes per residual evaluation x residual evaluations per second / 1e6.

The tile size of the mesh is the autotuner's cached choice for the
workload and primary precision (paper_2201_01291_amd/tune_cache.json;
--autotune times the candidates when the cache has no entry, --tiles
overrides it); config.tiles and config.tiles_from say which was used.

Prints ONE JSON line.  Extra fields: algorithmic GB/s of the whole step,
p50/p99 single-step latency of the FP64 path and of the mixed path (FP32
fluxes, FP64 accumulation), the mixed path's drift from FP64 after the timed
run, the roofline of the dominant kernel (HIP-event timing of every launch of
a second, profiled pass over the same number of steps) and the FP64 CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
KERNEL_SOURCES = ("paper_2201_01291_amd/csrc/vcx_kernels.h", "paper_2201_01291_amd/csrc/vcx_device.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(record_file, kernel):
    """HBM bytes per launch of `kernel` from a committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes, scaled by the copy-kernel
    calibration), or None when the record is missing or the kernel sources
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", record_file)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic-record:"):
            kv = dict(x.split("=", 1) for x in line.split()[1:])
            if kv.get("kernel") == kernel and kv.get("source") == kernel_source_hash():
                return int(kv["bytes"])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="dd2d", choices=["dd2d", "euler3d", "ns3d"])
    ap.add_argument("--tiles", default="", help="CELLS,NODES per tile (default: the workload's)")
    ap.add_argument("--latency-steps", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the profiled pass")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-pool", type=int, default=16)
    ap.add_argument("--serve-steps", type=int, default=100)
    ap.add_argument("--serve-budget-gb", type=float, default=8.0)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-graphs", type=int, default=0, help="server replays captured graphs")
    ap.add_argument("--serve-only", action="store_true", help="run the serving leg only")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with plain 256 MiB device copies (counter calibration)")
    ap.add_argument("--sweep", default="",
                    help="comma-separated NXxNY sizes of the drift-diffusion mesh family (h = 50 um) "
                         "timed after the main run, e.g. 1200x750,2400x1500")
    ap.add_argument("--sweep-only", action="store_true", help="run the size sweep only")
    ap.add_argument("--no-poisson", action="store_true", help="skip the Poisson leg")
    ap.add_argument("--autotune", action="store_true",
                    help="time the candidate tile sizes when the tuning cache has no entry")
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="arrival rate as a fraction of the measured batched capacity")
    return ap.parse_args()


def workload(name):
    from paper_2201_01291_amd import vcx, workloads as wl
    if name == "dd2d":
        m = wl.dd_streamer_mesh()
        n, E = wl.dd_fields(m)
        sp = wl.DD_STREAMER_SPECIES

        def phys(prec):
            return vcx.physics(model=vcx.MODEL_DRIFT_DIFFUSION, limiter=vcx.LIM_MINMOD, rk_stages=1,
                               nspecies=2, precision=prec, beta=1.0, cfl=0.5, fourier=0.25,
                               z=[s.z for s in sp], mu=[s.mu for s in sp], D=[s.D for s in sp])

        def ophys():
            import oracle
            return oracle.Phys(model=oracle.DRIFT_DIFFUSION, limiter=oracle.MINMOD, rk=1,
                               nspecies=2, cfl=0.5, fourier=0.25, z=[s.z for s in sp],
                               mu=[s.mu for s in sp], D=[s.D for s in sp])

        cfg = dict(workload="dd2d-streamer: periodic 400x250 jittered (20%) triangles, "
                            "2 charged species, LLW-minmod + central diffusion, RK1",
                   cells=m.ncells, nodes=m.nnodes, faces=m.nfaces, species=2,
                   residuals_per_step=1)
        # algorithmic bytes of the fused gradient + flux pass, every array
        # once: reads U, x, E, 1/V, dx_min per node and the cell topology
        # (3 x u16 local vertices + u32 periodic code), writes U
        N, M = m.nnodes, m.ncells
        ns, nd = 2, 2
        bytes_flux = N * 8 * (ns + nd + nd + 1 + 1 + ns) + M * (3 * 2 + 4)
        bytes_step = bytes_flux
        return m, n, E, phys, ophys, cfg, dict(flux=bytes_flux, step=bytes_step,
                                                traffic_record="traffic_flux_dd2d_streamer_200k.md",
                                                flux_kernel="k_fused<2,2,1,0,double>")
    if name == "euler3d":
        m = wl.euler3d_mesh()
        U = wl.euler_blob_state(m)

        def phys(prec):
            return vcx.physics(model=vcx.MODEL_GAS, flux=vcx.FLUX_ROE, limiter=vcx.LIM_VANLEER,
                               rk_stages=2, precision=prec, cfl=0.5)

        def ophys():
            import oracle
            return oracle.Phys(model=oracle.GAS, flux=oracle.ROE, limiter=oracle.VANLEER, rk=2, cfl=0.5)

        cfg = dict(workload="euler3d: periodic Kuhn 70x70x68 jittered (10%) tets, Roe + van Leer, RK2",
                   cells=m.ncells, nodes=m.nnodes, faces=m.nfaces, residuals_per_step=2)
        N, M = m.nnodes, m.ncells
        nr, nd, nv = 6, 3, 5
        # flux pass: reads W, G, x, U^n, 1/V, dx_min per node and the cell
        # topology (4 x u16 local vertices + u32 periodic code), writes W
        bytes_flux = N * 8 * (nr + nr * nd + nd + nv + 2 + nr) + M * (4 * 2 + 4)
        bytes_step = 2 * (N * 8 * (nr + nd) + M * 16 + N * 8 * nr * nd + bytes_flux
                          + N * 8 * (nv + nr + 1 + nr)) + N * 8 * (nr + nd) + M * 16
        return m, U, None, phys, ophys, cfg, dict(flux=bytes_flux, step=bytes_step,
                                                   traffic_record="traffic_flux_euler3d_2m.md",
                                                   flux_kernel="k_flux_gas<3,0,1,double,false>")
    if name == "ns3d":
        mix = wl.synthetic_mixture(9, seed=3)
        m = wl.ns3d_mesh()
        U = wl.ns_state(m, mix, lattice=8, seed=4)

        def phys(prec):
            return vcx.physics(model=vcx.MODEL_NAVIER_STOKES, flux=vcx.FLUX_HLLC,
                               limiter=vcx.LIM_VANLEER, rk_stages=2, nspecies=9, precision=prec,
                               cfl=0.5, fourier=0.25, mixture=mix)

        def ophys():
            import oracle
            return oracle.Phys(model=oracle.NAVIER_STOKES, flux=oracle.HLLC, limiter=oracle.VANLEER,
                               rk=2, nspecies=9, cfl=0.5, fourier=0.25, mixture=mix)

        cfg = dict(workload="ns3d: periodic 1 cm cube, Kuhn 110^3 jittered (10%) tets, 9 synthetic "
                            "species, HLLC + van Leer + central viscous/heat/species diffusion, RK2",
                   cells=m.ncells, nodes=m.nnodes, faces=m.nfaces, species=9,
                   residuals_per_step=2, primary="mixed", tiles=(64, 48))
        N, M = m.nnodes, m.ncells
        nrow = 15 + 13 + 21       # conserved + p, primitives, transport/thermo aux
        ng = (15 + 13) * 3        # gradients of the reconstructed rows and primitives
        bytes_flux = N * 8 * (nrow + ng + 3 + 14 + 2 + nrow) + M * (4 * 2 + 4)
        bytes_step = 2 * (N * 8 * (28 + 3) + M * 12 + N * 8 * ng + bytes_flux)
        return m, U, None, phys, ophys, cfg, dict(flux=bytes_flux, step=bytes_step,
                                                   traffic_record="traffic_flux_ns3d_8m.md",
                                                   flux_kernel="k_flux_ns<3,9,float>")
    raise ValueError(name)


def serving_leg(a, stream):
    """Serving workload: requests on 2D meshes of 5e3..2e6 cells (gas: HLLC +
    van Leer, RK2 on the periodic unit square; drift-diffusion as the main
    workload), a fixed number of steps each, served by the continuous-batching
    server in mixed precision with graph replay under a device-memory budget.
    1) capacity: every request submitted at once; 2) open loop: Poisson
    arrivals at a fraction of that capacity, latency from arrival to result;
    3) baseline: the same requests one at a time on the FP64 single-solve path
    (vcx_step), FIFO latencies for the same arrival times from the measured
    service times."""
    import threading
    from paper_2201_01291_amd import vcx, workloads as wl
    pool, reqs = wl.serving_requests(a.serve_requests, npool=a.serve_pool)
    sp = wl.DD_STREAMER_SPECIES
    print(f"[bench] serving: building {len(pool)} x 2 pool meshes", file=sys.stderr, flush=True)
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
        # completion times are observed in order; use the server's own latencies
        st = sv.stats()
        for rid in ids:
            ok, code, _, _ = sv.poll(rid)
            assert ok and code == vcx.OK, code
        wall = max(done_t) - t0
        sv.close()
        return st, wall

    serve(items[:8])   # warm-up: first launches and graph captures
    print("[bench] serving: capacity run", file=sys.stderr, flush=True)
    st_c, wall_c = serve(items)
    cap = len(items) / wall_c
    rate = a.serve_load * cap
    gaps = np.array([r["gap"] for r in reqs]) / rate
    arrivals = np.cumsum(gaps) - gaps[0]
    print(f"[bench] serving: open loop at {rate:.1f} req/s", file=sys.stderr, flush=True)
    st_o, wall_o = serve(items, arrivals)

    # baseline: one request at a time, FP64 single-solve path
    print("[bench] serving: sequential FP64 baseline", file=sys.stderr, flush=True)
    svc = []
    for kind, gm, U, E, _ in items:
        t1 = time.perf_counter()
        s = vcx.Solver(gm, P[(kind, vcx.PREC_FP64)], E)
        s.upload(U)
        s.step(nst)
        s.download()
        s.close()
        svc.append(time.perf_counter() - t1)
    svc = np.array(svc)
    fin, lat = 0.0, []
    for arr, sv_t in zip(arrivals, svc):
        fin = max(fin, arr) + sv_t
        lat.append((fin - arr) * 1e3)
    base = dict(kind="one request at a time, FP64, vcx_step (no batching, no graphs)",
                throughput_mfaces=round(total_faces / svc.sum() / 1e6, 1),
                capacity_req_s=round(len(items) / svc.sum(), 2),
                latency_p50_ms=round(float(np.percentile(lat, 50)), 2),
                latency_p99_ms=round(float(np.percentile(lat, 99)), 2),
                step_p50_ms=round(float(np.percentile(svc / nst * 1e3, 50)), 4),
                step_p99_ms=round(float(np.percentile(svc / nst * 1e3, 99)), 4),
                latency_note="FIFO queue over the same arrival times, from measured service times")
    cells = np.array([pool[r["pool"]]["cells"] for r in reqs])
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
    field: Poisson solve warm-started from the previous potential,
    E = E_background - grad phi, one drift-diffusion step."""
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
    e_eps0 = 1.602176634e-19 / 8.8541878128e-12
    zs = torch.tensor([s.z for s in sp], dtype=torch.float64, device="cuda")[:, None]
    Ebg = torch.zeros((2, m.nnodes), dtype=torch.float64, device="cuda")
    Ebg[0] = 1e6
    nd_ = torch.tensor(n, device="cuda")
    q = e_eps0 * (zs * nd_).sum(dim=0)
    tol = 1e-10
    ps.solve(q, tol=tol)               # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi, it_cold, rel = ps.solve(q, tol=tol)
    torch.cuda.synchronize()
    cold = time.perf_counter() - t0
    s = vcx.Solver(gm, ph, E0)
    s.upload(nd_)
    U = torch.empty_like(nd_)
    its, times = [], []
    K = 50
    for _ in range(K + 3):
        t1 = time.perf_counter()
        s.download(out=U)
        q = e_eps0 * (zs * U).sum(dim=0)
        phi, it, _ = ps.solve(q, phi0=phi, tol=tol, out=torch.empty_like(phi))
        E = Ebg + ps.field(phi)
        s.set_field(E)
        s.step(1)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        its.append(it)
    times, its = times[3:], its[3:]
    nnz_est = 7 * m.nnodes
    # bytes of one CG iteration, every array once: CSR (rp, col, val), and
    # z, p_old, p_new, q (first half); x, p, r, q, D^-1, r, z, x (second half)
    it_bytes = 4 * (m.nnodes + 1) + 12 * nnz_est + 8 * m.nnodes * 12
    ms_it = cold / max(it_cold, 1) * 1e3
    return dict(workload="dd2d-streamer mesh (periodic, 100,000 nodes), space charge of the densities "
                         "with a 20% central ion excess, CG with a two-level (Jacobi + aggregation) preconditioner to relative residual 1e-10",
                cold_iterations=it_cold, cold_ms=round(cold * 1e3, 3), ms_per_iteration=round(ms_it, 4),
                alg_gbs_per_iteration=round(it_bytes / (ms_it * 1e-3) / 1e9, 1),
                coupled_step_ms_p50=round(float(np.percentile(times, 50)) * 1e3, 3),
                coupled_iterations_mean=round(float(np.mean(its)), 2), coupled_steps=K,
                coupled_faces_per_s_M=round(m.nfaces / float(np.percentile(times, 50)) / 1e6, 1))


def size_sweep(a, stream):
    """FP64 throughput and the fused pass's algorithmic bandwidth of the
    drift-diffusion workload at larger sizes of the same mesh family (fixed
    spacing, larger box): from cache-resident to HBM-resident working sets."""
    import torch
    from paper_2201_01291_amd import vcx, workloads as wl
    out = []
    sp = wl.DD_STREAMER_SPECIES
    for item in a.sweep.split(","):
        nx, ny = (int(v) for v in item.lower().split("x"))
        print(f"[bench] sweep: dd2d {nx}x{ny}", file=sys.stderr, flush=True)
        m = wl.dd_streamer_mesh(nx, ny)
        n, E = wl.dd_fields(m)
        gm = vcx.Mesh(m, stream=stream)
        ph = vcx.physics(model=vcx.MODEL_DRIFT_DIFFUSION, limiter=vcx.LIM_MINMOD, rk_stages=1,
                         nspecies=2, precision=vcx.PREC_FP64, beta=1.0, cfl=0.5, fourier=0.25,
                         z=[s.z for s in sp], mu=[s.mu for s in sp], D=[s.D for s in sp])
        s = vcx.Solver(gm, ph, E)
        s.upload(n)
        s.step(10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(10)
        torch.cuda.synchronize()
        k = max(10, min(2000, int(2.0 / max(time.perf_counter() - t0, 1e-6) * 10)))
        s.upload(n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(k)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        s.profile(True)
        s.step(min(k, 200))
        nl, ms = s.profile_query("flux")
        s.profile(False)
        N, M = m.nnodes, m.ncells
        alg = N * 8 * (2 + 2 + 2 + 1 + 1 + 2) + M * (3 * 2 + 4)
        us = ms / nl * 1e3
        gbs = alg / (us * 1e-6) / 1e9
        out.append(dict(cells=M, nodes=N, faces=m.nfaces, steps=k,
                        mfaces=round(m.nfaces * k / el / 1e6, 1), ms_per_step=round(el / k * 1e3, 4),
                        fused_avg_us=round(us, 2), fused_alg_bytes=alg, fused_gbs=round(gbs, 1),
                        fused_frac=round(gbs / HBM_PEAK_GBS, 4)))
        s.close()
        gm.close()
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; runs on several GPUs are "
                                   "not supported (the library has no multi-GPU path)", "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    from paper_2201_01291_amd import vcx
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if a.serve_only:
        print(json.dumps({"serving": serving_leg(a, torch.cuda.current_stream().cuda_stream)}))
        return
    if a.sweep_only:
        print(json.dumps({"size_sweep": size_sweep(a, torch.cuda.current_stream().cuda_stream)}))
        return
    print(f"[bench] building workload {a.workload}", file=sys.stderr, flush=True)
    m, U0, E, phys, ophys, cfg, alg = workload(a.workload)
    primary = cfg.pop("primary", "fp64")    # precision of the reported value
    # tile size: the command line, else the autotuner's cached choice for the
    # primary precision (tuned now with --autotune when none is cached), else
    # the workload's default
    if a.tiles:
        tiles, tile_src = tuple(int(v) for v in a.tiles.split(",")), "command line"
    else:
        from paper_2201_01291_amd import autotune
        prim = phys(vcx.PREC_MIXED if primary == "mixed" else vcx.PREC_FP64)
        tc, tn, tile_src = autotune.pick_tiles(m, prim, U0, E, tune_if_missing=a.autotune)
        tiles = (tc, tn) if tile_src != "default" else tuple(cfg.get("tiles", (0, 0)))
        if tile_src == "default":
            tile_src = "workload default"
    cfg["tiles"] = list(tiles)
    cfg["tiles_from"] = tile_src
    stream = torch.cuda.current_stream()
    gm = vcx.Mesh(m, stream=stream.cuda_stream, tile_cells=tiles[0], tile_nodes=tiles[1])
    info = gm.info()
    s64 = vcx.Solver(gm, phys(vcx.PREC_FP64), E)
    s32 = vcx.Solver(gm, phys(vcx.PREC_MIXED), E)

    # ---- throughput, FP64 (the metric)
    s64.upload(U0)
    s64.step(a.warmup)
    s64.upload(U0)
    torch.cuda.synchronize()
    print(f"[bench] timing {a.steps} FP64 steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    s64.step(a.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    faces_per_step = m.nfaces * cfg["residuals_per_step"]
    mfaces = faces_per_step * a.steps / el / 1e6
    U64 = s64.download()

    # ---- the same solve as a batch of one (batched kernels, graph replay)
    s64.upload(U0)
    vcx.solve_batch([s64], [a.warmup])
    s64.upload(U0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vcx.solve_batch([s64], [a.steps])
    torch.cuda.synchronize()
    el_g = time.perf_counter() - t0
    assert np.array_equal(s64.download(), U64), "batch-of-one result differs from vcx_step"
    s64.upload(U0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vcx.solve_batch([s64], [a.steps], graphs=False)
    torch.cuda.synchronize()
    el_e = time.perf_counter() - t0
    assert np.array_equal(s64.download(), U64), "batch-of-one result differs from vcx_step"

    # ---- mixed path over the same steps: throughput and drift from FP64
    s32.upload(U0)
    s32.step(a.warmup)
    s32.upload(U0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s32.step(a.steps)
    torch.cuda.synchronize()
    el32 = time.perf_counter() - t0
    U32 = s32.download()
    drift = (np.abs(U32 - U64).max(axis=1) / np.abs(U64).max(axis=1)).tolist()

    # ---- single-step latency (host call to result, synchronised), p50/p99
    lat = {}
    for name, s in (("fp64", s64), ("mixed", s32)):
        s.upload(U0)
        s.step(5)
        ts = []
        for _ in range(a.latency_steps):
            t1 = time.perf_counter()
            s.step(1)
            ts.append((time.perf_counter() - t1) * 1e3)
        lat[name] = dict(p50_ms=float(np.percentile(ts, 50)), p99_ms=float(np.percentile(ts, 99)))

    # ---- profiled pass: per-kernel HIP-event durations on the solver stream
    kern = {}
    sp = s32 if primary == "mixed" else s64
    if not a.no_profile:
        sp.upload(U0)
        sp.profile(True)
        sp.step(a.steps)
        for k in ("gradient", "flux", "update"):
            n, ms = sp.profile_query(k)   # 2D meshes: "flux" is the fused gradient + flux pass
            if n:
                kern[k] = dict(launches=n, avg_us=ms / n * 1e3)
        sp.profile(False)
    dom = max(kern, key=lambda k: kern[k]["avg_us"]) if kern else None
    roof = None
    if "flux" in kern:
        fl = kern["flux"]
        achieved = alg["flux"] / (fl["avg_us"] * 1e-6) / 1e9
        roof = dict(kernel="flux", bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=measured_traffic(alg["traffic_record"], alg["flux_kernel"]),
                    alg_bytes_per_launch=alg["flux"], avg_us=round(fl["avg_us"], 2),
                    dominant_kernel=dom)

    # ---- CPU oracle on a bounded sample of the same workload
    cpu = None
    if not a.no_cpu:
        import oracle
        om = oracle.OracleMesh(m)
        ph = ophys()
        t1 = time.perf_counter()
        om.step(ph, U0, E, nsteps=1)
        one = time.perf_counter() - t1
        nsteps = max(1, int(a.cpu_seconds / max(one, 1e-6)))
        t1 = time.perf_counter()
        om.step(ph, U0, E, nsteps=nsteps)
        elc = time.perf_counter() - t1
        cpu = dict(value=round(faces_per_step * nsteps / elc / 1e6, 3), unit="Mfaces/s", cores=1,
                   kind="oracle", sample=f"{nsteps} full steps of the same mesh and state "
                                         f"({elc:.1f} s, sequential FP64 C oracle)")

    sweep = size_sweep(a, stream.cuda_stream) if a.sweep else None
    pois = None
    if not a.no_poisson and a.workload == "dd2d":
        print("[bench] Poisson leg", file=sys.stderr, flush=True)
        pois = poisson_leg(a, stream.cuda_stream)
    serve = None
    if not a.no_serve:
        serve = serving_leg(a, stream.cuda_stream)

    el_p = el32 if primary == "mixed" else el
    out = {
        "metric": "Mfaces/s residual throughput",
        "value": round(faces_per_step * a.steps / el_p / 1e6, 2),
        "unit": "Mfaces/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(el_p / a.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 flux, f64 accumulation" if primary == "mixed" else "f64",
        "data": "synthetic",
        "config": cfg,
        "hbm_gbs_algorithmic_step": round(alg["step"] * a.steps / el_p / 1e9, 1),
        "fp64": dict(value=round(mfaces, 2), unit="Mfaces/s", ms_per_step=round(el / a.steps * 1e3, 5)),
        "batch_of_one": dict(graph=round(faces_per_step * a.steps / el_g / 1e6, 2),
                             direct=round(faces_per_step * a.steps / el_e / 1e6, 2),
                             unit="Mfaces/s", bitwise_equal_to_vcx_step=True),
        "mixed": dict(value=round(faces_per_step * a.steps / el32 / 1e6, 2), unit="Mfaces/s",
                      ms_per_step=round(el32 / a.steps * 1e3, 5),
                      drift_vs_fp64_after_steps=drift),
        "latency": lat,
        "kernels": kern,
        "roofline": roof,
        "cpu_baseline": cpu,
        "serving": serve,
        "size_sweep": sweep,
        "poisson": pois,
        "mesh": info,
    }
    print(json.dumps(out))
    if a.copy_calibration:
        # a plain copy of known size: reads and writes 256 MiB per launch
        x = torch.rand(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: {x.numel() * 8} bytes read and written per launch",
              file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
