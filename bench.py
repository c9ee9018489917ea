#!/usr/bin/env python3
"""Factor + GMRES solves per second on one MI355X.

Workload (default): 2-D variable-coefficient diffusion on a 256 x 256 grid
(n = 65,536, 5-point, kappa = exp(g) with g a seeded Gaussian field of unit
variance and correlation length 8 cells), RCB cluster tree with leaf clusters
of 64 (depth 10), epsilon = 1e-4, 8 seeded right-hand sides uniform in [-1, 1],
right-preconditioned GMRES(30) to a true relative residual of 1e-10.

One step = lrx_factor_dev (symbolic plan on the host + numeric factorization
from values resident in HBM) + lrx_gmres_dev on the 8 right-hand sides
resident in HBM.  value = right-hand sides solved per second over the timed
steps, in the precision given by --precision (default mixed: FP32 compression
arithmetic and FP32 stored factor for the solve, FP64 pivots, Schur updates
and GMRES); the other precision is measured the same way and reported in
detail, with the distance between the two solutions.  The line also carries
the roofline entry of the dominant kernel class (event-timed inside the timed
region) and the CPU-oracle baseline measured on a bounded sample of the same
recipe.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 (vector and matrix)
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 (vector and dense matrix)
BF16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix
# HBM bytes per launch of the dominant kernel class, from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE over every dispatch of that kernel in this bench (each counter scaled by
# what it reads for a plain device copy of known size: FETCH_SIZE x 2.00, WRITE_SIZE
# x 1.00); kept per (workload, precision, kernel class) and reported as the
# roofline's traffic.
TRAFFIC_BYTES = {
    ("varcoef2d_256", "mixed", "compress"): 1.388e6,          # FP32 QR path (compress_gram = 0)
    ("varcoef2d_256", "mixed", "compress_gram"): 2.200e6,     # FETCH 707.9 KiB, WRITE 732.4 KiB
    ("varcoef2d_256", "fp64", "compress"): 1.393e6,           # FETCH 454.8 KiB, WRITE 451.0 KiB
}
TOL = 1e-10
RESTART = 30


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="varcoef2d_256")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"],
                    help="precision of the reported value; the other one is measured too and "
                         "reported in detail")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune-file", default=os.path.join(ROOT, "paper_1510_07363_amd", "tune_mi355x.json"),
                    help="launch shapes measured by paper_1510_07363_amd.autotune (read before timing)")
    ap.add_argument("--no-bf16-trial", action="store_true",
                    help="skip the BF16-projection trial run (LRX_MIXED_BF16)")
    ap.add_argument("--batch-group", type=int, default=32,
                    help="systems per lrx_factor_batch call in the batch256 workload")
    ap.add_argument("--cpu-sample-side", type=int, default=128,
                    help="grid side of the oracle's bounded sample (same recipe)")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests of the serving stream replayed (the recipe has 2,000)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="arrivals per second")
    ap.add_argument("--serve-n-max", type=int, default=65536,
                    help="largest system of a factor request (the recipe has 262,144)")
    ap.add_argument("--serve-cycle", type=int, default=8,
                    help="Arnoldi steps per serving round (one FGMRES restart cycle; unconverged "
                         "right-hand sides continue in the next round); 0: rounds solve to convergence")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only copy this many bytes device to device and exit (a plain copy of known "
                         "size, the reference for the HBM traffic counters)")
    return ap.parse_args()


def blas_info():
    """BLAS vendor and thread count of the oracle's NumPy."""
    vendor = "unknown"
    try:
        cfg = np.show_config(mode="dicts")
        bl = cfg.get("Build Dependencies", {}).get("blas", {})
        vendor = f"{bl.get('name', '?')} {bl.get('version', '')}".strip()
    except Exception:
        pass
    threads = None
    try:
        from threadpoolctl import threadpool_info
        for d in threadpool_info():
            if d.get("user_api") == "blas":
                threads = d.get("num_threads")
                vendor = f"{d.get('internal_api', vendor)} {d.get('version', '')}".strip()
                break
    except Exception:
        pass
    return vendor, threads


def cpu_baseline(workload, side, repeats=3):
    """Oracle (plain FP64 NumPy/SciPy) on the same recipe at a smaller grid,
    median of `repeats` runs; the rate is scaled to the full size by the unknown
    count (the method's cost is linear in n for a fixed leaf size)."""
    import oracle
    from paper_1510_07363_amd import workloads
    full = workloads.make_config(workload)
    p = workloads.make_config(workload, size=side)
    A = p.scipy()
    runs = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        F = oracle.factor(p.row_ptr, p.col_idx, p.val, p.perm, p.leaf_ptr, p.depth, p.epsilon,
                          check=False)
        t1 = time.perf_counter()
        its = []
        for k in range(p.rhs.shape[1]):
            out = oracle.fgmres(A, lambda v: oracle.solve(F, v), p.rhs[:, k], tol=TOL,
                                restart=RESTART, maxit=500)
            its.append(out["iters"])
        t2 = time.perf_counter()
        runs.append((t2 - t0, t1 - t0, t2 - t1, its))
    runs.sort(key=lambda r: r[0])
    t_all, t_fac, t_gm, its = runs[len(runs) // 2]
    scale = full.n / p.n
    t_full = t_all * scale
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count()
    vendor, blas_threads = blas_info()
    return {"value": p.rhs.shape[1] / t_full, "unit": "solves/s", "cores": threads,
            "kind": "oracle",
            "blas": vendor, "blas_threads": blas_threads,
            "sample": (f"{workload} recipe on a {side}x{side} grid (n={p.n}, depth {p.depth}), median of "
                       f"{repeats} runs (totals {[round(r[0], 2) for r in runs]} s): factor {t_fac:.1f}s + "
                       f"FGMRES(30) of {p.rhs.shape[1]} RHS {t_gm:.1f}s (iters {its}); rate scaled by n ratio "
                       f"{scale:.1f} to n={full.n}")}


def roofline(timing, dom, precision="fp64"):
    """Roofline entry of kernel class dom from its event-timed launches: HBM
    bound for the sweeps and the SpMV (algorithmic bytes per launch), ALU bound
    otherwise (algorithmic flops per launch, against the FP32 vector peak for the
    compression in mixed precision, whose reduced QRs and Jacobi run in FP32,
    else the FP64 peak)."""
    d = timing[dom]
    avg_ms = d["total_ms"] / max(d["launches"], 1)
    if dom in ("solve_fwd", "solve_bwd", "spmv"):
        per_launch = d["bytes"] / max(d["launches"], 1)
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None}
    else:
        per_launch = d["flops"] / max(d["launches"], 1)
        achieved = per_launch / (avg_ms * 1e-3) / 1e12
        # the compression's arithmetic runs on the vector ALUs (FP32 in mixed
        # precision; the Gram-path class compress_gram computes in FP64); the
        # Schur and projection products on the matrix cores (FP64 MFMA, or FP32
        # MFMA in mixed precision: same published peaks) (the pivot inverses of
        # factor_node stay FP64 in every mode)
        mixed = precision in ("mixed", "mixed_bf16") and dom in ("compress", "schur", "project")
        peak = FP32_PEAK_TFLOPS if mixed else FP64_PEAK_TFLOPS
        if dom == "project" and precision == "mixed_bf16":
            peak = BF16_MFMA_PEAK_TFLOPS
        bound = "mfma" if dom in ("schur", "project") else "alu"
        roof = {"bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None}
    roof["kernel"] = dom
    roof["avg_launch_ms"] = avg_ms
    roof["launches"] = d["launches"]
    roof["algorithmic_bytes_per_launch"] = d["bytes"] / max(d["launches"], 1)
    return roof


def timed_steps(args, lorax, torch, step, precision="fp64"):
    """Warm-up, one untimed probe step (finds the dominant kernel class), then
    exactly args.steps timed steps bracketed by stream synchronisation."""
    t_start = time.perf_counter()

    def progress(what):
        print(f"[bench] {what} done at {time.perf_counter() - t_start:.1f} s ({precision})", file=sys.stderr,
              flush=True)

    for i in range(args.warmup):
        step()
        progress(f"warm-up step {i + 1}")
    lorax.timing_enable(None)
    lorax.timing_read(reset=True)
    step()
    progress("probe step")
    probe = lorax.timing_read(reset=True)
    dom = max(probe, key=lambda k: probe[k]["total_ms"])
    lorax.timing_enable([dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    progress(f"{args.steps} timed steps")
    timing = lorax.timing_read(reset=True)
    lorax.timing_enable([])
    return t1 - t0, probe, roofline(timing, dom, precision)


def measure_batch(args, probs, lorax, torch, precision, sptr):
    """Batched form: one step = for each group of args.batch_group systems,
    lrx_factor_batch of the group (values resident in HBM) + lrx_gmres_batch_dev
    of all their right-hand sides, then the group's factors are freed (groups
    bound the HBM held at once)."""
    nrhs = probs[0].rhs.shape[1]
    eps = probs[0].epsilon
    systems = [(p.row_ptr, p.col_idx, None, p.perm, p.leaf_ptr, p.depth) for p in probs]
    vals = [torch.from_numpy(p.val).to("cuda:0") for p in probs]
    bs = [torch.from_numpy(np.ascontiguousarray(p.rhs.T)).to("cuda:0") for p in probs]
    xs = [torch.zeros_like(b) for b in bs]
    vptr = [v.data_ptr() for v in vals]
    bptr = [b.data_ptr() for b in bs]
    xptr = [x.data_ptr() for x in xs]
    torch.cuda.synchronize()
    state = {}

    G = max(1, args.batch_group)

    def step():
        its_all, stats_all = [], []
        for g0 in range(0, len(systems), G):
            sl = slice(g0, g0 + G)
            Fs = lorax.factor_batch(systems[sl], eps, stream=sptr, precision=precision, val_dev=vptr[sl])
            its, rr, st = lorax.gmres_batch_dev(Fs, nrhs, bptr[sl], xptr[sl], tol=TOL, restart=RESTART, maxit=500)
            if st != lorax.LRX_OK or float(np.max(rr)) > TOL:
                raise RuntimeError(f"batched GMRES did not reach {TOL}: status {st}, max relres {np.max(rr)}")
            its_all.append(its)
            stats_all += [F.stats() for F in Fs]
            print(f"[batch] group {g0 // G + 1}/{(len(systems) + G - 1) // G} done ({precision}, "
                  f"factor {Fs[0].stats()['t_factor_ms']:.0f} ms)", file=sys.stderr, flush=True)
            for F in Fs:
                F.free()
        state["its"], state["stats"] = np.concatenate(its_all), stats_all

    T, probe, roof = timed_steps(args, lorax, torch, step, precision)
    res = 0.0
    for p, x in zip(probs, xs):
        X = x.cpu().numpy().T
        r = np.linalg.norm(p.scipy() @ X - p.rhs, axis=0) / np.linalg.norm(p.rhs, axis=0)
        res = max(res, float(r.max()))
    if res > TOL:
        raise RuntimeError(f"true residual {res:.3e} above {TOL}")
    sts = state["stats"]
    its = state["its"]
    return {
        "ms_per_step": 1e3 * T / args.steps,
        "value": len(probs) * nrhs * args.steps / T,
        "roofline": roof,
        "detail": {"gmres_iters_min": int(its.min()), "gmres_iters_max": int(its.max()),
                   "gmres_iters_mean": float(its.mean()), "true_relres_max": res,
                   "batch_group": G,
                   "t_factor_batch_ms_first_group": sts[0]["t_factor_ms"],
                   "t_plan_ms_sum": float(sum(s["t_plan_ms"] for s in sts)),
                   "t_factor_sync_ms": sts[0]["t_sync_ms"],
                   "factor_bytes": int(sum(s["factor_bytes"] for s in sts)),
                   "solve_bytes": int(sum(s["solve_bytes"] for s in sts)),
                   "max_rank": int(max(s["max_rank"] for s in sts)),
                   "kernel_ms_per_step_probe": {k: round(v["total_ms"], 3) for k, v in probe.items()},
                   "kernel_launches_per_step_probe": {k: v["launches"] for k, v in probe.items()}},
    }


def cpu_baseline_batch(probs, budget_s=20.0):
    """Oracle on the smallest systems of the batch (at least one 2-D and one 3-D,
    then more while the running time stays within budget_s); the rate is scaled
    to the whole batch by the unknown count (the cost is linear in n)."""
    import oracle
    order = sorted(range(len(probs)), key=lambda i: probs[i].n)
    picks, seen_dim = [], set()
    for i in order:
        d = probs[i].coords.shape[1]
        if d not in seen_dim:
            picks.append(i)
            seen_dim.add(d)
    t_all, n_done, solves, done = 0.0, 0, 0, []
    queue = picks + [i for i in order if i not in picks]
    for i in queue:
        if done and t_all >= budget_s:
            break
        p = probs[i]
        A = p.scipy()
        t0 = time.perf_counter()
        F = oracle.factor(p.row_ptr, p.col_idx, p.val, p.perm, p.leaf_ptr, p.depth, p.epsilon, check=False)
        for k in range(p.rhs.shape[1]):
            oracle.fgmres(A, lambda v: oracle.solve(F, v), p.rhs[:, k], tol=TOL, restart=RESTART, maxit=500)
        t_all += time.perf_counter() - t0
        n_done += p.n
        solves += p.rhs.shape[1]
        done.append(i)
    n_total = sum(p.n for p in probs)
    scale = n_total / n_done
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count()
    total_solves = len(probs) * probs[0].rhs.shape[1]
    return {"value": total_solves / (t_all * scale), "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": (f"{len(done)} smallest systems of the batch (n = {[probs[i].n for i in done]}), "
                       f"factor + FGMRES(30) of {solves} RHS in {t_all:.1f}s; time scaled by the "
                       f"unknown ratio {scale:.0f} to the {len(probs)} systems (n = {n_total})")}


def measure(args, p, lorax, torch, precision, sptr, val_d, b_d, x_d):
    """Warm-up, one untimed probe step (finds the dominant kernel class), then
    exactly args.steps timed steps bracketed by stream synchronisation."""
    nrhs = p.rhs.shape[1]
    state = {}

    state["t_gmres"] = []

    def step():
        F = lorax.Factor(p.row_ptr, p.col_idx, None, p.perm, p.leaf_ptr, p.depth, p.epsilon,
                         stream=sptr, val_dev=val_d.data_ptr(), precision=precision)
        tg = time.perf_counter()
        its, rr, st = F.gmres_dev(b_d.data_ptr(), x_d.data_ptr(), nrhs, tol=TOL,
                                  restart=RESTART, maxit=500)
        torch.cuda.current_stream().synchronize()
        state["t_gmres"].append(time.perf_counter() - tg)
        if st != lorax.LRX_OK or float(np.max(rr)) > TOL:
            raise RuntimeError(f"GMRES did not reach {TOL}: status {st}, relres {rr}")
        state["its"], state["rr"], state["stats"] = its, rr, F.stats()
        F.free()

    T, probe, roof = timed_steps(args, lorax, torch, step, precision)
    t_gmres = state["t_gmres"][-args.steps:]
    roof["traffic"] = TRAFFIC_BYTES.get((args.workload, precision, roof["kernel"]))
    if roof["traffic"]:
        roof["traffic_over_algorithmic"] = roof["traffic"] / max(roof["algorithmic_bytes_per_launch"], 1.0)
    # independent check of the last solution
    A = p.scipy()
    X = x_d.cpu().numpy().T
    res = np.linalg.norm(A @ X - p.rhs, axis=0) / np.linalg.norm(p.rhs, axis=0)
    if float(res.max()) > TOL:
        raise RuntimeError(f"true residual {res.max():.3e} above {TOL}")
    st = state["stats"]
    return {
        "ms_per_step": 1e3 * T / args.steps,
        "value": nrhs * args.steps / T,
        "roofline": roof,
        "X": X,
        "detail": {"steady_state_solves_per_s": nrhs * len(t_gmres) / sum(t_gmres),
                   "t_gmres_ms": 1e3 * float(np.median(t_gmres)),
                   "gmres_iters": [int(i) for i in state["its"]],
                   "true_relres_max": float(res.max()),
                   "t_factor_ms": st["t_factor_ms"], "t_plan_ms": st["t_plan_ms"],
                   "t_factor_sync_ms": st["t_sync_ms"], "t_solve_prog_ms": st["t_solve_prog_ms"],
                   "t_host_compress_ms": st["t_host_compress_ms"], "t_host_node_ms": st["t_host_node_ms"],
                   "sweep_stages": st["sweep_stages"], "sweep_launches": st["sweep_launches"],
                   "factor_bytes": st["factor_bytes"], "solve_bytes": st["solve_bytes"],
                   "mean_rank": st["mean_rank"], "max_rank": st["max_rank"],
                   "kernel_ms_per_step_probe": {k: round(v["total_ms"], 3) for k, v in probe.items()},
                   "kernel_launches_per_step_probe": {k: v["launches"] for k, v in probe.items()}},
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU implementation: --gpus must be 1"}))
        sys.exit(2)
    import torch
    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes}), flush=True)
        return
    from paper_1510_07363_amd import lorax, workloads

    torch.cuda.set_device(0)
    if args.workload == "batch256":
        return main_batch(args, torch, lorax, workloads)
    if args.workload == "serve":
        return main_serve(args, torch, lorax, workloads)
    p = workloads.make_config(args.workload)
    nrhs = p.rhs.shape[1]
    # a non-blocking stream of the default priority: the library captures the
    # GMRES preconditioner into a HIP graph there (never on the null stream)
    stream = torch.cuda.Stream()
    sptr = stream.cuda_stream
    val_d = torch.from_numpy(p.val).to("cuda:0")
    b_d = torch.from_numpy(np.ascontiguousarray(p.rhs.T)).to("cuda:0")      # column-major n x nrhs
    x_d = torch.zeros_like(b_d)
    torch.cuda.synchronize()

    from paper_1510_07363_amd import autotune
    other = "fp64" if args.precision == "mixed" else "mixed"
    runs, tuned = {}, {}
    order = [other, args.precision]
    if not args.no_bf16_trial:
        order = ["mixed_bf16"] + order
    for prec in order:                              # the reported precision is timed last
        tuned[prec] = autotune.load(args.tune_file, "fp64" if prec == "fp64" else "mixed", lorax)
        with torch.cuda.stream(stream):
            runs[prec] = measure(args, p, lorax, torch, prec, sptr, val_d, b_d, x_d)
    main_run, other_run = runs[args.precision], runs[other]
    # error of the reported solutions against the other precision's (both at 1e-10 residual)
    diff = np.linalg.norm(main_run["X"] - other_run["X"], axis=0) / np.linalg.norm(other_run["X"], axis=0)

    line = {
        "metric": "factor+GMRES solves/s at 1e-10 resid",
        "value": main_run["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": p.n, "nnz": p.nnz, "depth": p.depth,
                   "leaf": p.meta["leaf"], "epsilon": p.epsilon, "nrhs": nrhs, "gmres": f"FGMRES({RESTART})",
                   "tol": TOL, "precision": args.precision, "compress": "svd"},
        "roofline": main_run["roofline"],
        "detail": dict(main_run["detail"], **{
            other: {"value": other_run["value"], "ms_per_step": other_run["ms_per_step"],
                    "roofline": other_run["roofline"], **other_run["detail"]},
            f"rel_diff_vs_{other}_solution_max": float(diff.max()),
            "tune": tuned.get(args.precision) or lorax.tune_get()}),
    }
    if "mixed_bf16" in runs:
        rb = runs["mixed_bf16"]
        ref = runs["fp64"]["X"]
        db = np.linalg.norm(rb["X"] - ref, axis=0) / np.linalg.norm(ref, axis=0)
        line["detail"]["mixed_bf16_trial"] = {
            "value": rb["value"], "ms_per_step": rb["ms_per_step"],
            "gmres_iters": rb["detail"]["gmres_iters"], "true_relres_max": rb["detail"]["true_relres_max"],
            "rel_diff_vs_fp64_solution_max": float(db.max()),
            "note": "projection B V on BF16 operands (FP32 accumulation); compression bound not claimed"}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_sample_side)
    print(json.dumps(line), flush=True)


def main_serve(args, torch, lorax, workloads):
    """Wall-clock replay of the serving request stream (make_serve_stream):
    factor requests run on a worker thread and stream of their own while solve
    rounds run on the main thread's stream."""
    from paper_1510_07363_amd.serve import LoraxBackend, Server, SystemSpec
    reqs = workloads.make_serve_stream(count=args.serve_requests, rate=args.serve_rate,
                                       n_max=args.serve_n_max)
    specs, bs = {}, []
    for r in reqs:
        if r["kind"] == "factor":
            specs[r["key"]] = SystemSpec(r["key"], *workloads.build_serve_system(r))
    for r in reqs:
        if r["kind"] == "solve":
            rng = np.random.default_rng(r["rhs_seed"])
            bs.append(rng.uniform(-1, 1, (specs[r["key"]].n, r["nrhs"])))
        else:
            bs.append(None)
    print(f"[serve] {len(reqs)} requests, {len(specs)} systems built", file=sys.stderr, flush=True)
    srv = Server(LoraxBackend(precision=args.precision), 200 << 30, tol=TOL, restart=RESTART,
                 factor_backend=LoraxBackend(precision=args.precision), max_factor_batch=8,
                 cycle=args.serve_cycle or None)
    for sp in specs.values():
        srv.register(sp)
    # warm-up (untimed): module load and first launches on a small system
    wkey = min(specs, key=lambda k: specs[k].n)
    srv.submit(wkey, np.ones(specs[wkey].n))
    srv.run_until_idle()
    srv.evict(wkey)
    for k in srv.latencies:
        srv.latencies[k].clear()
    srv.batches.clear()
    srv.start()
    futs = []
    t0 = time.perf_counter()
    t_print = t0
    i, last = 0, 0
    while i < len(reqs) or not srv.idle():
        now = time.perf_counter() - t0
        while i < len(reqs) and reqs[i]["t"] <= now:
            r = reqs[i]
            if r["kind"] == "factor":
                futs.append(("factor", r, srv.submit_factor(r["key"], arrival=t0 + r["t"])))
            else:
                futs.append(("solve", r, srv.submit(r["key"], bs[i], arrival=t0 + r["t"])))
            i += 1
        if srv.step() == 0:
            time.sleep(0.0005)
        ndone = sum(f.done() for _, _, f in futs)
        tnow = time.perf_counter()
        if ndone > last and (tnow - t_print > 5.0 or ndone == len(reqs)):
            last, t_print = ndone, tnow
            print(f"[serve] {ndone}/{len(reqs)} requests done at {tnow - t0:.1f} s "
                  f"({srv.n_factored} factored)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    srv.stop()
    worst, n_rhs, failed = 0.0, 0, 0
    for kind, r, f in futs:
        if f.exception() is not None:
            failed += 1
            continue
        if kind == "solve":
            x, its, rr = f.result()
            worst = max(worst, float(np.max(rr)))
            n_rhs += r["nrhs"]
    if worst > TOL or failed:
        raise RuntimeError(f"served relres {worst:.3e}, {failed} failed requests")
    lat_all = np.array(srv.latencies["solve"] + srv.latencies["factor"])
    line = {
        "metric": "served solves/s at 1e-10 resid",
        "value": n_rhs / T,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": 1e3 * T,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "serve", "requests": len(reqs), "rate_req_s": args.serve_rate,
                   "cycle": args.serve_cycle,
                   "n_range": [16384, args.serve_n_max], "factor_requests": len(specs), "rhs_total": n_rhs,
                   "hbm_budget_gib": 200, "gmres": f"FGMRES({RESTART})", "tol": TOL, "precision": args.precision},
        "detail": {"latency_solve": srv.latency_stats("solve"), "latency_factor": srv.latency_stats("factor"),
                   "latency_all_p50_ms": float(np.percentile(lat_all, 50) * 1e3),
                   "latency_all_p99_ms": float(np.percentile(lat_all, 99) * 1e3),
                   "requests_per_s": len(reqs) / T, "solve_rounds": srv.n_rounds,
                   "round": f"FGMRES({args.serve_cycle}) cycle" if args.serve_cycle else "solve to convergence",
                   "mean_systems_per_round": float(np.mean(srv.batches)) if srv.batches else 0.0,
                   "factored": srv.n_factored, "evicted": srv.n_evicted,
                   "resident_bytes_end": srv.resident_bytes()},
    }
    srv.close()
    print(json.dumps(line), flush=True)


def main_batch(args, torch, lorax, workloads):
    probs = workloads.make_batch()
    print(f"[batch] {len(probs)} systems generated, n = {sum(p.n for p in probs)}", file=sys.stderr, flush=True)
    from paper_1510_07363_amd import autotune
    stream = torch.cuda.Stream()                 # non-blocking: GMRES replays its preconditioner as a graph
    tuned = autotune.load(args.tune_file, "fp64" if args.precision == "fp64" else "mixed", lorax)
    with torch.cuda.stream(stream):
        main_run = measure_batch(args, probs, lorax, torch, args.precision, stream.cuda_stream)
    main_run["detail"]["tune"] = tuned or lorax.tune_get()
    nrhs = probs[0].rhs.shape[1]
    line = {
        "metric": "factor+GMRES solves/s at 1e-10 resid",
        "value": main_run["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "batch256", "systems": len(probs), "n_total": int(sum(p.n for p in probs)),
                   "n_min": int(min(p.n for p in probs)), "n_max": int(max(p.n for p in probs)),
                   "depth_min": int(min(p.depth for p in probs)), "depth_max": int(max(p.depth for p in probs)),
                   "leaf": 64, "epsilon": probs[0].epsilon, "nrhs": nrhs, "gmres": f"FGMRES({RESTART})",
                   "tol": TOL, "precision": args.precision, "compress": "svd"},
        "roofline": main_run["roofline"],
        "detail": main_run["detail"],
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_batch(probs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
