#!/usr/bin/env python3
"""Benchmark: ms per low-sync GMRES + classical-AMG solve to relative residual 1e-8.

Default workload: 3-D Poisson 7-point, 128^3 (2 097 152 rows, 14 581 760 nnz), b ~ N(0, 1) seed 1,
RS-AMG theta = 0.25, hybrid V-cycle with ILU(0) on the finest level (3 Neumann terms per triangular
solve) and polynomial GS elsewhere, GMRES(30), tol 1e-8, FP64. One step = one whole solve from x0 = 0
with the matrix, hierarchy and right-hand side already resident in HBM; setup is timed separately.

Prints one JSON line (rank 0). Only one GPU is used: --gpus above 1 exits with a message.
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


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3", "c4n", "c4r", "c4rcm"])
    ap.add_argument("--N", type=int, default=None)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--smoother", default="ilu0", choices=["ilu0", "pgs"])
    ap.add_argument("--tri", default="neumann", choices=["neumann", "direct"])
    ap.add_argument("--terms", type=int, default=3)
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--gmres-T", default="neumann", choices=["neumann", "direct"])
    ap.add_argument("--max-coarse", type=int, default=None,
                    help="coarsen to at most this many rows (dense direct solve on the coarsest level); default "
                         "50 for c1, whose configuration fixes it, 1000 otherwise")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-contract", action="store_true",
                    help="skip the contract figures: C2 coarsened to 50 rows, and the FP32 preconditioner against "
                         "all-FP64 at C2 and C3")
    ap.add_argument("--compare", action="store_true",
                    help="also time the direct-triangular, l1-Jacobi and FP32-preconditioner variants")
    ap.add_argument("--serve-requests", type=int, default=0,
                    help="requests of the served stream to replay (2000: the whole stream; default 0, skipped: a "
                         "replay has ended in a host segmentation fault whose cause is not established)")
    ap.add_argument("--serve-inflight", type=int, default=64)
    ap.add_argument("--serve-setup-threads", type=int, default=14)
    ap.add_argument("--serve-only", action="store_true")
    ap.add_argument("--serve-coarsen", default="pmis", choices=["rs", "pmis"],
                    help="setup of the served requests: the device PMIS setup (default) or host RS")
    ap.add_argument("--nonnormality", action="store_true",
                    help="the factor study of Sections 5.3.2 to 5.3.4 instead of the benchmark: orderings of C4 (Table 2) "
                         "and an ILUT fill sweep (Tables 3-5), with GMRES iterations when a GPU is present")
    ap.add_argument("--nn-N", type=int, default=128, help="grid size of the ordering studies")
    ap.add_argument("--orderings", action="store_true",
                    help="only the convection-diffusion orderings: iterations, ms and GMRES-product bandwidth")
    ap.add_argument("--nn-fill-N", type=int, default=64, help="grid size of the fill sweep")
    return ap.parse_args()


HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
PROFILE_EVERY = 3  # time every 3rd run of consecutive dominant-kernel dispatches (one event pair per run;
# odd, so pre- and post-smoothing runs alternate in the sample)

# Measured HBM traffic of the dominant kernel (bytes per launch): rocprofv3 FETCH_SIZE x 2.000 plus
# WRITE_SIZE x 1.000, factors from a 2 GiB copy (profiles/k_neumann_level0_c2_128cubed_traffic.md for FP64,
# profiles/hbm_traffic_c2_128cubed_kernels.md for both; in FP32 the term runs as k_neumann_pairs).
# Valid for the kernel version it was taken on; None when the kernel has changed since.
DOMINANT_TRAFFIC_BYTES = {("c2", 128, "fp64", "ilu0"): 109.79e6, ("c2", 128, "fp32", "ilu0"): 53.37e6}


def copy_ceiling(torch, nbytes=2 << 30, reps=10):
    """Device-to-device copy bandwidth (read + write bytes / time) as a practical HBM ceiling."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def read_ceiling(torch, nbytes=2 << 30, reps=10):
    """Read-only streaming bandwidth (a full reduction of a 2 GiB array) as the ceiling for read-bound kernels."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    a.sum()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        a.sum()
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a
    return nbytes / (ms * 1e-3) / 1e9


def _time_solves(torch, H, bt, xt, kw, steps, warmup):
    for _ in range(warmup):
        xt.zero_()
        H.solve(bt, xt, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(steps):
        xt.zero_()
        stats.append(H.solve(bt, xt, **kw))
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, stats


def served_stream(namg, count, inflight, setup_threads, coarsen="pmis", gen_threads=12, lead=256):
    """Replay the first `count` requests of the served stream (Poisson arrivals at 50/s, n log-uniform in
    [32, 160], variable-k pressure systems) against the continuous-batching server: FP32 AMG + FP64 GMRES(30),
    polynomial GS with 2 Neumann terms, tol 1e-8. Latency runs from each request's scheduled arrival to its
    completion on the server's clock. coarsen "rs": host setup (RS, classical interpolation); "pmis": the
    device setup (PMIS, BAMG direct interpolation).

    The systems are generated while the stream plays, by `gen_threads` threads, at most `lead` requests
    ahead of the last one submitted (memory stays bounded); the clock starts once the first `lead`
    requests exist. Four submitter threads submit request j at its scheduled arrival (or as soon as it
    exists, if generation falls behind: such a request counts as late, and its lateness is part of its
    latency)."""
    import threading
    from concurrent.futures import ThreadPoolExecutor

    from workloads import serve_stream, varcoef3d

    reqs = serve_stream(2000, seed=5)[:count]
    ready = [threading.Event() for _ in range(count)]
    systems = [None] * count
    room = threading.Semaphore(lead)

    def gen(j):
        room.acquire()
        systems[j] = varcoef3d(reqs[j]["N"], 0.5, reqs[j]["seed"])
        ready[j].set()

    gpool = ThreadPoolExecutor(max_workers=gen_threads)
    gfuts = [gpool.submit(gen, j) for j in range(count)]
    ready[min(lead, count) - 1].wait()
    srv = namg.Server(solve=dict(smoother=namg.SMOOTH_PGS, inner_terms=2, restart=30, tol=1e-8),
                      max_inflight=inflight, setup_threads=setup_threads, precision=namg.FP32_PRECOND)
    t0_srv = srv.clock()
    t0 = time.perf_counter()
    tickets = [None] * count
    late = np.zeros(count)
    peak = {"waiting": 0, "inflight": 0, "queue": 0}
    stop = threading.Event()

    def monitor():
        while not stop.wait(0.05):
            c = srv.stats()
            peak["waiting"] = max(peak["waiting"], c["waiting"])
            peak["inflight"] = max(peak["inflight"], c["inflight"])
            peak["queue"] = max(peak["queue"], c["submitted"] - c["completed"] - c["failed"])

    def submitter(k, nsub):
        for j in range(k, count, nsub):
            delay = reqs[j]["arrival_s"] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            ready[j].wait()
            late[j] = max(0.0, (time.perf_counter() - t0) - reqs[j]["arrival_s"])
            A, b = systems[j]
            # polynomial GS throughout: no ILU(0) factors to build
            if coarsen == "pmis":
                tickets[j] = srv.submit(A, b, ilu_levels=0, coarsen=namg.COARSEN_PMIS, seed=j)
            else:
                tickets[j] = srv.submit(A, b, ilu_levels=0)
            systems[j] = None
            room.release()
            if (j + 1) % 250 == 0:
                print(f"[served] submitted {j + 1}/{count} at {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                      flush=True)

    mon = threading.Thread(target=monitor, daemon=True)
    mon.start()
    subs = [threading.Thread(target=submitter, args=(k, 4)) for k in range(4)]
    for t in subs:
        t.start()
    for t in subs:
        t.join()
    for f in gfuts:
        f.result()
    gpool.shutdown()
    results = [srv.wait(t) for t in tickets]
    stop.set()
    mon.join()
    counters = srv.stats()
    srv.close()
    lat = np.array([r["times"]["done"] - (t0_srv + q["arrival_s"]) for r, q in zip(results, reqs)])
    done = np.array([r["times"]["done"] - t0_srv for r in results])
    solve_s = np.array([r["times"]["done"] - r["times"]["admitted"] for r in results])
    setup_s = np.array([r["times"]["setup_done"] - r["times"]["setup_start"] for r in results])
    queue_s = np.array([r["times"]["setup_start"] - r["times"]["submit"] for r in results])
    ok = all(r["status"] == namg.OK and r["relres_true"] <= 1e-8 for r in results)
    span = done.max() - reqs[0]["arrival_s"]
    return {
        "requests": count, "all_converged": bool(ok),
        "p50_s": round(float(np.percentile(lat, 50)), 4), "p99_s": round(float(np.percentile(lat, 99)), 4),
        "max_s": round(float(lat.max()), 4), "solves_per_s": round(count / span, 2),
        "arrival_span_s": round(reqs[-1]["arrival_s"] - reqs[0]["arrival_s"], 3),
        "completion_span_s": round(float(span), 3),
        "late_submissions": int(np.count_nonzero(late > 0.005)), "max_submit_lateness_s": round(float(late.max()), 4),
        "median_queue_s": round(float(np.median(queue_s)), 4), "median_setup_s": round(float(np.median(setup_s)), 4),
        "median_inflight_s": round(float(np.median(solve_s)), 4),
        "mean_iters": round(float(np.mean([r["iters"] for r in results])), 2),
        "alg_GBps_while_serving": round(sum(r["alg_bytes"] for r in results) / span / 1e9, 1),
        "peak_inflight": counters["peak_inflight"], "peak_waiting": peak["waiting"], "peak_outstanding": peak["queue"],
        "ticks": counters["ticks"], "batched_launches": counters["launches"],
        "peak_device_GB": round(counters["peak_device_bytes"] / 1e9, 2),
        "setup_threads": setup_threads, "max_inflight": inflight, "setup": coarsen,
    }


def contract_figures(namg, torch, steps):
    """The figures the targets are stated on, next to the headline: C2 coarsened to <= 50 rows (the
    library default and C1's configuration), and the FP32 preconditioner against all-FP64 at the same
    1e-8 true residual on C2 (ILU(0) hybrid, t = 3) and on C3 (192^3 -div(k grad p), polynomial GS t = 2;
    the configuration that states the 1.5x target). ms per solve, median of `steps` solves after one
    warm-up."""
    from workloads import config_system

    out = {}
    dev = torch.device("cuda:0")

    def run(A, bt, prec, max_coarse, kw, ilu_levels):
        H = namg.Hierarchy(A, device=0, precision=prec, ilu_levels=ilu_levels, max_coarse=max_coarse)
        xt = torch.zeros_like(bt)
        H.solve(bt, xt, **kw)
        times, st = [], None
        for _ in range(steps):
            xt.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = H.solve(bt, xt, **kw)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        info = H.info()
        H.close()
        return {"ms": round(float(np.median(times)), 4), "iters": st["iters"], "relres": st["relres_true"],
                "levels": info["levels"], "status_ok": st["status"] == namg.OK}

    A, b, _ = config_system("c2")
    bt = torch.from_numpy(b).to(dev)
    kw = dict(tol=1e-8, restart=30, smoother=namg.SMOOTH_ILU0, tri_mode=namg.TRI_NEUMANN, inner_terms=3)
    out["c2_fp64_max_coarse_50"] = run(A, bt, namg.FP64, 50, kw, 1)
    f64 = run(A, bt, namg.FP64, 1000, kw, 1)
    f32 = run(A, bt, namg.FP32_PRECOND, 1000, kw, 1)
    out["c2_fp64"], out["c2_fp32_precond"] = f64, f32
    out["c2_fp32_speedup"] = round(f64["ms"] / f32["ms"], 3)
    print("[contract] c2 done", file=sys.stderr, flush=True)
    del bt
    A, b, _ = config_system("c3")
    bt = torch.from_numpy(b).to(dev)
    kw = dict(tol=1e-8, restart=30, smoother=namg.SMOOTH_PGS, tri_mode=namg.TRI_NEUMANN, inner_terms=2)
    f64 = run(A, bt, namg.FP64, 1000, kw, 0)
    f32 = run(A, bt, namg.FP32_PRECOND, 1000, kw, 0)
    out["c3_fp64"], out["c3_fp32_precond"] = f64, f32
    out["c3_fp32_speedup"] = round(f64["ms"] / f32["ms"], 3)
    print("[contract] c3 done", file=sys.stderr, flush=True)
    return out


def orderings_study(namg, torch, N, steps):
    """The convection-diffusion system (Peclet 10, N^3) in natural, random and RCM-of-random order with its
    configuration (ILU(0) Neumann t = 3 on the finest level, FP32 preconditioner, FP64 GMRES(50), tol 1e-8):
    iterations, ms per solve and the achieved bandwidth of the GMRES product w = A z (FP64 A, FP32 z; the
    kernel's own bytes over its live hipEvent time) and of the finest level's Neumann terms, per ordering."""
    from workloads import config_system

    out = {}
    kw = dict(tol=1e-8, restart=50, smoother=namg.SMOOTH_ILU0, tri_mode=namg.TRI_NEUMANN, inner_terms=3)
    for name in ("c4n", "c4r", "c4rcm"):
        A, b, _ = config_system(name, N)
        H = namg.Hierarchy(A, device=0, precision=namg.FP32_PRECOND, ilu_levels=1, max_coarse=1000)
        bt = torch.from_numpy(b).to("cuda:0")
        xt = torch.zeros_like(bt)
        ms, st = _time_solves(torch, H, bt, xt, kw, steps, 1)
        rates = {}
        for key, family in (("gmres_spmv_GBps", namg.KF_GMRES_SPMV), ("level0_neumann_GBps", namg.KF_NEUMANN)):
            H.profile_kernel(family, 0, 1)
            _time_solves(torch, H, bt, xt, kw, 1, 0)
            pr = H.profile_read()
            H.profile_kernel(namg.KF_NONE)
            rates[key] = round(pr["alg_bytes"] / (pr["total_ms"] * 1e-3) / 1e9, 1) if pr["launches"] else None
        out[name] = {"ms": round(ms, 3), "iters": st[-1]["iters"], "relres": st[-1]["relres_true"], **rates}
        H.close()
        print(f"[orderings] {name} done", file=sys.stderr, flush=True)
    return {"metric": "convection-diffusion orderings: iterations, ms and bandwidth",
            "workload": f"c4 {N}^3 Peclet 10, ILU(0) t = 3, FP32 preconditioner, GMRES(50)", **out}


def cpu_baseline(A, b, kw, gpu_iters, max_coarse):
    """The oracle (single-threaded FP64 C++) on the same system and hierarchy configuration: setup
    excluded, full solve timed."""
    import oracle

    t0 = time.perf_counter()
    G = oracle.Hierarchy(A, max_coarse=max_coarse)
    setup_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = G.solve(b, tol=kw["tol"], restart=kw["restart"], smoother=kw["smoother"], tri_mode=kw["tri_mode"],
                t=kw["inner_terms"], gmres_T=kw["gmres_T"])
    solve_s = time.perf_counter() - t0
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            model = next(line.split(":", 1)[1].strip() for line in f if line.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": solve_s * 1e3, "unit": "ms", "cores": 1, "kind": "oracle",
            "host": f"{model}; {os.cpu_count()} logical CPUs visible, the oracle uses 1",
            "sample": f"one full oracle solve of the same system ({r['iters']} iterations, relres "
                      f"{r['relres_true']:.1e}; GPU {gpu_iters}); oracle setup {setup_s:.1f} s excluded"}


def nonnormality_study(namg, torch, N, fill_N):
    """Sections 5.3.2 to 5.3.4 on our workloads, one JSON object. (1) Orderings (Table 2 and its dep table): C4,
    upwind convection-diffusion, in natural, random and RCM-of-random order, ILU(0) on the finest level:
    dep(L), dep(U), ||U_s||_F, ||U_s||_2, the residuals of 5 Jacobi iterations for L y = b and U v = y,
    and the hybrid GMRES(30) solve (ILU(0) Neumann t = 3) when a GPU is present. (2) Fill sweep (Tables
    3 to 5): ILUT(1e-3, lfil) on the finest level of C4 natural at fill_N^3 for lfil = 5, 10, 20, 50:
    ||U_s||_2, ||U_s||_F and Theorem 1's bound, dep(U) before and after Ruiz scaling with Theorem 3's
    bound, and GMRES iterations. (3) Powers of U_s (the figure of Section 5.3.2, a 331-row system there):
    max |(U_s^p)_ij|, ||U_s^p||_2 and nnz(U_s^p) on C4 natural at 7^3 = 343 rows, ILU(0) and ILUT(1e-3, 20),
    for every p up to the power at which U_s^p vanishes."""
    from workloads import config_system

    gpu = torch is not None and torch.cuda.is_available()
    dev = 0 if gpu else -1
    solve_kw = dict(tol=1e-8, restart=30, smoother=namg.SMOOTH_ILU0, tri_mode=namg.TRI_NEUMANN, inner_terms=3)

    def solve(H, b):
        if not gpu:
            return {}
        bt = torch.from_numpy(b).to("cuda:0")
        xt = torch.zeros_like(bt)
        ms, st = _time_solves(torch, H, bt, xt, solve_kw, 2, 1)
        return {"gmres_iters": st[-1]["iters"], "solve_ms": round(ms, 3), "relres": st[-1]["relres_true"]}

    def diag(H, b):
        d = H.ilu_diagnostics(0, power_iters=100)
        rl, ru = H.tri_jacobi_residuals(0, b, 5)
        keep = ("nnz_lower", "nnz_upper", "max_row_upper", "dep_L", "dep_U", "nu", "norm2_Us", "th1_bound",
                "dep_U_ruiz", "ruiz_iters", "th3_bound", "delta", "th4_bound")
        out = {k: (round(d[k], 6) if isinstance(d[k], float) else d[k]) for k in keep}
        out.update(jacobi5_res_L=rl, jacobi5_res_U=ru)
        return out

    orderings = {}
    for name in ("c4n", "c4r", "c4rcm"):
        A, b, _ = config_system(name, N)
        t0 = time.perf_counter()
        H = namg.Hierarchy(A, device=dev, ilu_levels=1)
        row = {"setup_ms": round((time.perf_counter() - t0) * 1e3, 1)}
        row.update(diag(H, b))
        row.update(solve(H, b))
        H.close()
        orderings[name] = row
        print(f"[nonnormality] ordering {name} done", file=sys.stderr, flush=True)
    fill = {}
    A, b, _ = config_system("c4n", fill_N)
    for lfil in (5, 10, 20, 50):
        H = namg.Hierarchy(A, device=dev, ilu_levels=1, ilu_kind=namg.ILUT, ilut_droptol=1e-3, ilut_lfil=lfil)
        row = diag(H, b)
        row.update(solve(H, b))
        H.close()
        fill[str(lfil)] = row
        print(f"[nonnormality] lfil {lfil} done", file=sys.stderr, flush=True)
    powers = {}
    A, b, _ = config_system("c4n", 7)
    for label, kw in (("ilu0", {}), ("ilut_1e-3_20", dict(ilu_kind=namg.ILUT, ilut_droptol=1e-3, ilut_lfil=20))):
        H = namg.Hierarchy(A, device=-1, ilu_levels=1, **kw)
        # U_s^p = 0 by p = n at the latest; powers after the first zero one cost nothing
        seq = H.us_powers(0, A.n, power_iters=300)
        H.close()
        last = int(np.nonzero(seq["nnz"])[0].max()) + 1 if seq["nnz"].any() else 0
        powers[label] = {"vanishes_at_p": last + 1,
                         "max_abs": [float(f"{v:.4g}") for v in seq["max_abs"][:last]],
                         "norm2": [float(f"{v:.4g}") for v in seq["norm2"][:last]],
                         "nnz": [int(v) for v in seq["nnz"][:last]]}
    print("[nonnormality] powers of U_s done", file=sys.stderr, flush=True)
    return {"metric": "non-normality of the ILU factors (Sections 5.3.2 to 5.3.4)", "gpu": gpu,
            "orderings": {"workload": f"c4 convection-diffusion {N}^3, ILU(0) finest level", **orderings},
            "fill_sweep": {"workload": f"c4n {fill_N}^3, ILUT(droptol 1e-3, lfil)", **fill},
            "us_powers": {"workload": f"c4n 7^3 = {A.n} rows, finest-level factors", **powers}}


def main():
    args = _args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solve phase is not sharded across GPUs "
              "(the row-sharded design is described, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2112_14681_amd as namg
    from workloads import config_system

    if args.nonnormality:
        print(json.dumps(nonnormality_study(namg, torch, args.nn_N, args.nn_fill_N)), flush=True)
        return

    if args.orderings:
        print(json.dumps(orderings_study(namg, torch, args.nn_N, args.steps)), flush=True)
        return

    if args.serve_only:
        if args.serve_requests <= 0:
            print("--serve-only replays --serve-requests N requests of the stream (2000: all of it)", file=sys.stderr)
            sys.exit(2)
        print(json.dumps({"metric": "served latency of the pressure-system request stream",
                          "served": served_stream(namg, args.serve_requests, args.serve_inflight,
                                                  args.serve_setup_threads, args.serve_coarsen)}), flush=True)
        return

    A, b, meta = config_system(args.config, args.N)
    prec = namg.FP64 if args.precision == "fp64" else namg.FP32_PRECOND
    t0 = time.perf_counter()
    if args.max_coarse is None:
        args.max_coarse = 50 if args.config == "c1" else 1000
    H = namg.Hierarchy(A, device=0, precision=prec, ilu_levels=1, max_coarse=args.max_coarse)
    setup_ms = (time.perf_counter() - t0) * 1e3
    info = H.info()
    kw = dict(tol=1e-8, restart=args.restart, smoother=namg.SMOOTH_ILU0 if args.smoother == "ilu0" else namg.SMOOTH_PGS,
              tri_mode=namg.TRI_NEUMANN if args.tri == "neumann" else namg.TRI_DIRECT, inner_terms=args.terms,
              gmres_T=namg.T_NEUMANN if args.gmres_T == "neumann" else namg.T_DIRECT)
    dev = torch.device("cuda:0")
    bt = torch.from_numpy(b).to(dev)
    xt = torch.zeros_like(bt)
    # the dominant kernel: the Neumann inner term on the finest level (ILU(0) triangles), timed live during
    # the timed solves: a run of its consecutive dispatches (the four terms of one smoothing sweep) gets
    # one start event on its first dispatch and one stop event after its last, so the events' own cost is
    # spread over the run; every PROFILE_EVERY-th run is timed
    dom_family, dom_level = namg.KF_NEUMANN, 0
    for _ in range(args.warmup):
        xt.zero_()
        H.solve(bt, xt, **kw)
    H.profile_kernel(dom_family, dom_level, PROFILE_EVERY)
    ms, stats = _time_solves(torch, H, bt, xt, kw, args.steps, 0)
    prof = H.profile_read()
    H.profile_kernel(namg.KF_NONE)
    st = stats[-1]
    if st["status"] != namg.OK or st["relres_true"] > 1e-8:
        print(f"solve did not reach 1e-8: {st}", file=sys.stderr)
        sys.exit(1)
    gbs = st["alg_bytes"] / (ms * 1e-3) / 1e9

    out = {
        "metric": "ms per GMRES+AMG solve to rel-res 1e-8 at 128^3; HBM GB/s; served p99",
        "value": round(ms, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == namg.FP64 else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"{meta['name']}: " + {
                "c1": "2-D Poisson 5-point", "c2": "3-D Poisson 7-point", "c3": "3-D -div(k grad p) lognormal k, z 1:100",
                "c4n": "3-D upwind conv-diff natural order", "c4r": "3-D upwind conv-diff random order",
                "c4rcm": "3-D upwind conv-diff RCM order"}[meta["name"]] + f" N={meta['N']}",
            "n": A.n, "nnz": A.nnz, "smoother": args.smoother, "tri_mode": args.tri, "inner_terms": args.terms,
            "restart": args.restart, "gmres_T": args.gmres_T, "precision": args.precision, "tol": 1e-8,
            "max_coarse": args.max_coarse, "levels": info["levels"], "op_complexity": round(info["op_complexity"], 3),
        },
        "iters": st["iters"],
        "relres": st["relres_true"],
        "setup_ms": round(setup_ms, 1),
        "alg_GBps": round(gbs, 1),
    }
    if prof["launches"]:
        # one launch is one pass of a Neumann inner term over a strict half of the finest operator; its
        # algorithmic bytes per pass: ((nnz - n) / 2) (s + 4) + 4 (n + 1) + 4 s n (s = 8 or 4; the strict
        # half's values with int32 indices, its row pointers, and the vectors r, D^-1, g_in, g_out)
        s_val = 8 if prec == namg.FP64 else 4
        pass_bytes = (A.nnz - A.n) / 2 * (s_val + 4) + 4 * (A.n + 1) + 4 * s_val * A.n
        # what the kernel itself moves: at 128^3 the triangle is in the slice-diagonal form (8 or 4 B per entry
        # and 4 B per 64 entries, no per-entry column), so the per-unit figure above, which counts int32
        # columns, exceeds it and `frac` can pass 1; `kernel_GBps` and `traffic_GBps` are the rates of the
        # bytes actually moved
        kernel_bytes = prof["alg_bytes"] / prof["launches"]
        per_launch_ms = prof["total_ms"] / prof["launches"]
        achieved = pass_bytes / (per_launch_ms * 1e-3) / 1e9
        traffic = DOMINANT_TRAFFIC_BYTES.get((meta["name"], meta["N"], args.precision, args.smoother))
        out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBPS, 4),
                           "traffic": traffic,
                           # measured HBM bytes per launch over the same live time: what the memory system moved
                           "traffic_GBps": round(traffic / (per_launch_ms * 1e-3) / 1e9, 1) if traffic else None,
                           "kernel": ("k_neumann<1,double>" if prec == namg.FP64 or os.environ.get("NAMG_DIA_PAIRS") == "0"
                                      else "k_neumann_pairs (FP32, two rows per lane)") + " on level 0 "
                                     f"({'ILU(0)' if args.smoother == 'ilu0' else 'poly-GS'} Neumann term)",
                           "launches_timed": prof["launches"],
                           "timing": f"hipEvents around every {PROFILE_EVERY}th run of consecutive dispatches",
                           "avg_us": round(per_launch_ms * 1e3, 3),
                           "alg_MB_per_launch": round(pass_bytes / 1e6, 3),
                           "kernel_MB_per_launch": round(kernel_bytes / 1e6, 3),
                           "kernel_GBps": round(kernel_bytes / (per_launch_ms * 1e-3) / 1e9, 1)}
    out["copy_ceiling_GBps"] = round(copy_ceiling(torch), 1)
    out["read_ceiling_GBps"] = round(read_ceiling(torch), 1)

    if args.compare:
        # the Table 7 family on this workload: ILUT(1e-2, 5) on the finest level with Jacobi (Neumann) or
        # direct triangular solves next to ILU(0), plus the Table 6 comparator, aggressive coarsening on
        # the first two levels, the other precision and one more Neumann term (t + 1)
        cmp = {}
        ilut = dict(ilu_kind=namg.ILUT, ilut_droptol=1e-2, ilut_lfil=5)
        H_ilut = None
        for name, extra, prec2, setup2 in (("direct_tri", dict(tri_mode=namg.TRI_DIRECT), prec, None),
                                           ("l1_jacobi", dict(smoother=namg.SMOOTH_L1JAC), prec, None),
                                           ("ilut_jacobi", dict(smoother=namg.SMOOTH_ILU0), prec, ilut),
                                           ("ilut_direct", dict(smoother=namg.SMOOTH_ILU0, tri_mode=namg.TRI_DIRECT),
                                            prec, ilut),
                                           ("aggressive2", {}, prec, dict(agg_levels=2)),
                                           ("pmis_device_setup", {}, prec, dict(coarsen=namg.COARSEN_PMIS)),
                                           ("fp32_precond", {}, namg.FP32_PRECOND, None), ("fp64", {}, namg.FP64, None),
                                           ("inner_terms_4", dict(inner_terms=4), prec, None)):
            if setup2 is ilut:
                if H_ilut is None:
                    t0 = time.perf_counter()
                    H_ilut = namg.Hierarchy(A, device=0, precision=prec, ilu_levels=1, max_coarse=args.max_coarse,
                                            **setup2)
                    ilut_setup_ms = (time.perf_counter() - t0) * 1e3
                H2 = H_ilut
            elif setup2 is not None:
                t0 = time.perf_counter()
                H2 = namg.Hierarchy(A, device=0, precision=prec, ilu_levels=1, max_coarse=args.max_coarse, **setup2)
                other_setup_ms = (time.perf_counter() - t0) * 1e3
            else:
                H2 = H if prec2 == prec else namg.Hierarchy(A, device=0, precision=prec2, ilu_levels=1,
                                                            max_coarse=args.max_coarse)
            kw2 = dict(kw, **extra)
            ms2, st2 = _time_solves(torch, H2, bt, xt, kw2, max(1, args.steps // 2), 1)
            cmp[name] = {"ms": round(ms2, 3), "iters": st2[-1]["iters"], "relres": st2[-1]["relres_true"]}
            if setup2 is ilut:
                cmp[name].update(setup=dict(droptol=setup2["ilut_droptol"], lfil=setup2["ilut_lfil"]),
                                 setup_ms=round(ilut_setup_ms, 1))
            elif setup2 is not None:
                info2 = H2.info()
                cmp[name].update(setup=setup2, setup_ms=round(other_setup_ms, 1), levels=info2["levels"],
                                 op_complexity=round(info2["op_complexity"], 3))
                H2.close()
        if H_ilut is not None:
            H_ilut.close()
        out["compare"] = cmp

    if not args.no_contract and args.config == "c2" and args.N is None:
        H.close()
        out["contract"] = contract_figures(namg, torch, max(3, min(args.steps, 7)))
    if args.serve_requests > 0:
        H.close()
        out["served"] = served_stream(namg, args.serve_requests, args.serve_inflight, args.serve_setup_threads,
                                      args.serve_coarsen)
    else:
        out["served"] = {"skipped": "off by default: one replay of the 2000-request stream ended in a host "
                                    "segmentation fault in its first seconds (no GPU fault), cause not established; "
                                    "--serve-requests 2000 runs it"}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, b, kw, st["iters"], args.max_coarse)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
