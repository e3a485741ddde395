#!/usr/bin/env python3
"""Throughput of the batched AM iteration on one MI355X.

Workload (one "step"): the spiked-covariance matrix A (n = 1000, p = 10000,
three spikes with thetas 60/40/25 on disjoint 50-element supports), 1024
random unit starting points, and a solve of each of the 8 formulations of
Table 1 from all 1024 starts with maxit = 200 and the stop test disabled, so
every start does exactly 200 iterations (fixed work).  s = 50 for the
constraints, gamma = 0.1 max_i ||a_i||_2 for the penalties.  A and the
starts are resident in HBM before timing starts.

Metric: AM iterations x starts per second over the timed steps.  Also
reported: the roofline position of the dominant kernel (the FP32 MFMA
product V = A^T Y, timed with HIP events on the solve's stream around its
launches in every 8th iteration of the timed steps: an event pair costs the
stream a few microseconds, so events around every launch would slow the
step), the whole step against the FP32 MFMA bound of its algorithmic work
(running starts and iterate nonzeros counted on the device), and the FP64
CPU oracle's throughput on a bounded sample of the same workload.

The default run adds, under "secondary", short runs of the other
configurations (about two minutes in all): the BF16 + polish precision study
at 5000 x 50000, the 16 GB instance at 20000 x 200000, and a 2000-request
serving stream at 40 requests/s, batched against one request at a time
(--no-secondary skips them; --workload selects one of them alone, in full).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the A^T Y product on the spiked-all8 workload, from
# rocprofv3 FETCH_SIZE / WRITE_SIZE counter passes scaled by the same
# counters on a 1 GiB copy (fetch x 2.0, write x 1.0); valid only for the
# GEMM source they were taken on.
TRAFFIC_ATY = {"gemm_kernel_sha256":
               "5f5e9c75553825e3076bdeeafe9b0b6daac79865826051a58bc420f182d9c765",
               "read_bytes": 3.919e4 * 1024 * 2.0, "write_bytes": 4.257e4 * 1024 * 1.0,
               "profile": "profiles/traffic_spiked-1000x10000-F1-r1024_fetch_write.md"}


def gemm_kernel_digest():
    """sha256 of the GEMM kernel's source (its tile configuration and the
    kernel body, not the host-side planner in the same file)."""
    import hashlib

    src = os.path.join(ROOT, "paper_1212_4137_amd", "csrc", "gemm_f32.hip")
    with open(src) as f:
        text = f.read()
    a = text.index("template <int BM, int BN, int WM, int WN>\nstruct GemmCfg")
    b = text.index("// Compiled tile shapes.")
    return hashlib.sha256(text[a:b].encode()).hexdigest()


def traffic_aty():
    """Measured traffic of the A^T Y product, or None once the GEMM kernel
    differs from the one the counters were taken on."""
    if gemm_kernel_digest() != TRAFFIC_ATY["gemm_kernel_sha256"]:
        return None
    return {"bytes_per_launch": TRAFFIC_ATY["read_bytes"] + TRAFFIC_ATY["write_bytes"],
            "read_bytes": TRAFFIC_ATY["read_bytes"], "write_bytes": TRAFFIC_ATY["write_bytes"],
            "algorithmic_bytes": None, "source": TRAFFIC_ATY["profile"]}


def cpu_baseline(A_np, X0_np, params, maxit_sample=100):
    """FP64 oracle on a bounded sample of the same workload: every
    formulation, the first 2 x threads starts, maxit_sample iterations each
    (stop test disabled).  Returns iterations x starts per second."""
    import oracle

    threads = max(1, min(len(os.sched_getaffinity(0)), 16))
    starts = 2 * threads
    X = np.asarray(X0_np[:starts], dtype=np.float64)
    work = 0
    t0 = time.perf_counter()
    for fid in range(1, 9):
        res = oracle.am_multi(A_np, fid, params[fid], X, -1.0, maxit_sample,
                              nthreads=threads, want_x=False)
        work += int(res["iters"].sum())
    dt = time.perf_counter() - t0
    return {"value": work / dt, "unit": "iter*start/s", "cores": threads,
            "kind": "oracle",
            "sample": f"all 8 formulations x first {starts} starts x {maxit_sample} "
                      f"iterations ({work} iteration-starts, {dt:.1f} s, FP64 C, "
                      f"{threads} threads over starts)"}


def _roofline_aty(kt, r, n, p, peak, unit_flops_name="TFLOP/s"):
    """Roofline point of the dominant kernel, V = A^T Y: 2 r n p flops per
    launch over the average launch time measured with HIP events."""
    launches = kt["aty_launches"]
    avg_ms = kt["aty_ms"] / launches
    achieved = 2.0 * r * n * p / (avg_ms * 1e-3) / 1e12
    return {"kernel": "gemm_nt (V = A^T Y), the dominant kernel", "bound": "mfma",
            "achieved": round(achieved, 2), "peak": peak, "unit": unit_flops_name,
            "frac": round(achieved / peak, 4), "traffic": None,
            "avg_launch_ms": round(avg_ms, 5), "launches": int(launches)}


def _timed_steps(step, steps, warmup):
    import torch

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [step(True) for _ in range(steps)]
    torch.cuda.synchronize()
    return time.perf_counter() - t0, outs


def _sum_kt(outs):
    kt = {}
    for o in outs:
        for k, v in o["kt"].items():
            kt[k] = kt.get(k, 0) + v
    return kt


def bench_all8(args, spca, torch, timed_events=True):
    dev = torch.device("cuda:0")
    cfg = workloads.SPIKED_ALL8
    n, p, r, maxit = cfg["n"], cfg["p"], cfg["r"], cfg["maxit"]
    sp = workloads.spiked_matrix(cfg["seed"], n, p, cfg["thetas"], cfg["spike_nnz"])
    A_np = sp.A
    X0_np = workloads.random_unit_starts(cfg["seed"] + 1000, r, p)
    params = {fid: workloads.s_or_gamma_for(fid, A_np, cfg["s"]) for fid in range(1, 9)}
    fids = [int(f) for f in args.fids.split(",")]

    A = torch.from_numpy(np.ascontiguousarray(A_np.T)).to(dev).t()  # column-major
    X0 = torch.from_numpy(X0_np).to(dev)
    # the 8 solves of a step are independent: with --streams K they run on K
    # streams at once (a context and a host thread each), so that one solve's
    # memory-bound kernels overlap another's matrix-core products; the
    # formulations are dealt to the streams by their measured cost
    ns = max(1, min(args.streams, len(fids)))
    ctxs = [spca.Context(0) for _ in range(ns)]
    streams = ([torch.cuda.current_stream()] if ns == 1 else
               [torch.cuda.Stream() for _ in range(ns)])
    cost = {1: 50, 2: 50, 3: 63, 4: 62, 5: 82, 6: 82, 7: 45, 8: 82}
    lanes = [[] for _ in range(ns)]
    load = [0] * ns
    for fid in sorted(fids, key=lambda f: (-cost[f], f)):
        w = load.index(min(load))
        lanes[w].append(fid)
        load[w] += cost[fid]
    modes = {}

    def step(timing):
        results = {}

        def run_lane(w):
            for fid in lanes[w]:
                results[fid] = spca.am_solve(
                    A, fid, params[fid], X0, tol=-1.0, maxit=maxit, ctx=ctxs[w],
                    stream=streams[w], kernel_times=timing,
                    flags=args.flags | (spca.FLAG_TIME_SAMPLED if timing else 0))

        if ns == 1:
            run_lane(0)
        else:
            import threading

            threads = [threading.Thread(target=run_lane, args=(w,)) for w in range(ns)]
            for t in threads:
                t.start()
            for t in threads:
                t.join()
            if len(results) != len(fids):
                raise RuntimeError("a solve of the step failed")
        work = 0.0
        kt = {}
        nnz = {}
        for fid in fids:
            res = results[fid]
            work += res["iters_x_starts"]
            nnz[fid] = float(np.mean(res["nnz_per_start"]))
            if timing:
                for k, v in res["kernel_times"].items():
                    kt[k] = kt.get(k, 0) + v
                t = res["kernel_times"]
                modes[fid] = (t["iters_dense"], t["iters_list"], t["iters_union"])
        return {"work": work, "kt": kt, "nnz": nnz}

    ctx, stream = ctxs[0], streams[0]

    if args.autotune:
        # a8: one tuned solve per formulation fills the tuning table before
        # the timed steps (which then plan from it)
        for fid in fids:
            spca.am_solve(A, fid, params[fid], X0, tol=-1.0, maxit=2, ctx=ctx,
                          stream=stream, flags=args.flags | spca.FLAG_AUTOTUNE)
    if not timed_events:
        # throughput only: no kernel events on any iteration
        dt, outs = _timed_steps(lambda timing: step(False), args.steps, args.warmup)
        return {"metric": "AM iters x starts/sec",
                "value": sum(o["work"] for o in outs) / dt, "unit": "iter*start/s",
                "ms_per_step": dt / args.steps * 1e3,
                "config": {"concurrent_solves": ns, "solves_per_stream": lanes}}
    dt, outs = _timed_steps(step, args.steps, args.warmup)
    work = sum(o["work"] for o in outs)
    kt_all = _sum_kt(outs)
    roofline = _roofline_aty(kt_all, r, n, p, PEAK_FP32_MFMA_TFLOPS)
    # the whole iteration against its algorithmic bound: per running start
    # and iteration 2 n p flops for A^T Y, and 2 n flops per nonzero of the
    # iterate for A x, with the running starts and the nonzeros counted on
    # the device at every iteration; beside it the dense-equivalent count
    # (both products dense, 4 n p per start and iteration)
    alg_flops = (2.0 * n * p * kt_all["active_starts_sum"] +
                 2.0 * n * kt_all["ax_nnz_sum"]) / args.steps
    dense_flops = 4.0 * n * p * kt_all["active_starts_sum"] / args.steps
    t_step = dt / args.steps
    path = {"bound": "mfma", "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
            "algorithmic_flop_per_step": alg_flops,
            "t_bound_ms": alg_flops / (PEAK_FP32_MFMA_TFLOPS * 1e12) * 1e3,
            "achieved": round(alg_flops / t_step / 1e12, 2),
            "frac": round(alg_flops / (PEAK_FP32_MFMA_TFLOPS * 1e12) / t_step, 4),
            "dense_equivalent_flop_per_step": dense_flops,
            "dense_equivalent_frac": round(dense_flops / (PEAK_FP32_MFMA_TFLOPS * 1e12) / t_step, 4),
            "note": "whole AM step (all 8 formulations) against the FP32 MFMA bound of its "
                    "algorithmic work; 'roofline' above is the A^T Y kernel alone"}
    tr = traffic_aty()
    if tr is not None:
        tr["algorithmic_bytes"] = 4.0 * (n * p + r * n + r * p)
    roofline["traffic"] = tr["bytes_per_launch"] if tr else None
    roofline["traffic_unit"] = "bytes per launch (HBM, FETCH_SIZE + WRITE_SIZE, calibrated)"
    roofline["traffic_detail"] = tr
    other = {"x_update_avg_ms": round(kt_all["x_update_ms"] / kt_all["x_update_launches"], 5),
             "ax_dense_avg_ms": round(kt_all["ax_dense_ms"] / kt_all["ax_dense_launches"], 5),
             "mean_nnz_per_start": outs[-1]["nnz"],
             "ax_modes_dense_list_union": modes,
             "gemm_plans": {"aty": spca.gemm_plan(r, p, n, 16),
                            "ax_dense": spca.gemm_plan(r, n, p, 16)},
             "tuning_table": spca.tune_table_export()}
    rec = {
        "metric": "AM iters x starts/sec",
        "value": work / dt,
        "unit": "iter*start/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "n": n, "p": p, "starts": r,
                   "formulations": fids, "maxit": maxit, "tol": "disabled (fixed work)",
                   "s": cfg["s"], "gamma": "0.1*max_i ||a_i||_2",
                   "spikes": list(cfg["thetas"]), "spike_nnz": cfg["spike_nnz"],
                   "concurrent_solves": ns, "solves_per_stream": lanes},
        "roofline": roofline,
        "path_roofline": path,
        "kernels": other,
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(A_np, X0_np, params)
    return rec


def bench_large(args, spca, torch):
    """One-GPU large instance: 20000 x 200000 FP32 (16 GB) generated in HBM
    by the counter-based generator, F1 with s = 200, 64 starts; a step is one
    solve with the stop test disabled (fixed work of maxit iterations)."""
    from workloads import counter

    cfg = workloads.SPIKED_LARGE
    n, p, r = cfg["n"], cfg["p"], cfg["r"]
    maxit = args.maxit or 30
    f = counter.spike_factors(cfg["seed"], n, p, cfg["thetas"], cfg["spike_nnz"])
    A = spca.generate_spiked(cfg["seed"], n, p, cfg["thetas"], f.U, f.V)
    X0 = torch.from_numpy(workloads.random_unit_starts(cfg["seed"] + 1000, r, p)).cuda()
    ctx = spca.Context(0)
    stream = torch.cuda.current_stream()
    res_last = {}
    tuned = not args.no_autotune
    if tuned:
        # a8: the configuration asks for autotuned tiles: one short tuned
        # solve fills the table for both products before the timed steps
        spca.am_solve(A, cfg["fid"], float(cfg["s"]), X0, tol=-1.0, maxit=2, ctx=ctx,
                      stream=stream, flags=args.flags | spca.FLAG_AUTOTUNE)
    plans = {"aty": spca.gemm_plan(r, p, n, 16), "ax_dense": spca.gemm_plan(r, n, p, 16)}

    def step(timing):
        res = spca.am_solve(A, cfg["fid"], float(cfg["s"]), X0, tol=-1.0, maxit=maxit,
                            ctx=ctx, stream=stream, kernel_times=timing,
                            flags=args.flags | (spca.FLAG_TIME_SAMPLED if timing else 0))
        res_last.update(res)
        return {"work": res["iters_x_starts"], "kt": res["kernel_times"] if timing else {}}

    dt, outs = _timed_steps(step, args.steps, args.warmup)
    kt = _sum_kt(outs)
    sup = set(res_last["support"].tolist())
    recovered = [len(sup & set(s.tolist())) for s in f.supports]
    return {
        "metric": "AM iters x starts/sec",
        "value": sum(o["work"] for o in outs) / dt,
        "unit": "iter*start/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (counter-based spiked model generated in HBM)",
        "config": {"workload": cfg["name"], "n": n, "p": p, "starts": r, "formulation": 1,
                   "s": cfg["s"], "maxit": maxit, "tol": "disabled (fixed work)",
                   "spikes": list(cfg["thetas"]), "spike_nnz": cfg["spike_nnz"],
                   "A_bytes": 4 * n * p},
        "roofline": _roofline_aty(kt, r, n, p, PEAK_FP32_MFMA_TFLOPS),
        "kernels": {"x_update_avg_ms": round(kt["x_update_ms"] / kt["x_update_launches"], 5),
                    "ax_dense_avg_ms": round(kt["ax_dense_ms"] / max(1, kt["ax_dense_launches"]), 5),
                    "ax_modes_dense_list_union": (kt["iters_dense"], kt["iters_list"],
                                                  kt["iters_union"])},
        "result": {"objective": res_last["objective"], "nnz": int(res_last["nnz"]),
                   "support_overlap_with_spikes": recovered},
        "autotuned": tuned, "gemm_plans_shape_splits": plans,
    }


def bench_precision(args, spca, torch):
    """BF16 storage + FP32 polish against the FP32 path on the 5000 x 50000
    spiked workload (F8 and F1, 256 starts, stop test on): solves/s of each
    path and the relative gap of their final FP64 objectives."""
    cfg = workloads.SPIKED_BF16
    n, p, r = cfg["n"], cfg["p"], cfg["r"]
    sp = workloads.spiked_matrix(cfg["seed"], n, p, cfg["thetas"], cfg["spike_nnz"])
    A = torch.from_numpy(np.ascontiguousarray(sp.A.T)).cuda().t()
    X0 = torch.from_numpy(workloads.random_unit_starts(cfg["seed"] + 1000, r, p)).cuda()
    params = {fid: workloads.s_or_gamma_for(fid, sp.A, cfg["s"]) for fid in cfg["fids"]}
    del sp
    ctx = spca.Context(0)
    stream = torch.cuda.current_stream()
    out = {}
    for prec in ("fp32", "bf16"):
        last = {}

        def step(timing, prec=prec, last=last):
            for fid in cfg["fids"]:
                last[fid] = spca.am_solve(A, fid, params[fid], X0, tol=1e-7,
                                          maxit=cfg["maxit"], precision=prec,
                                          polish_maxit=cfg["maxit"], ctx=ctx,
                                          stream=stream, flags=args.flags)
            return {"work": len(cfg["fids"]), "kt": {}}

        dt, outs = _timed_steps(step, args.steps, args.warmup)
        out[prec] = {"solves_per_s": args.steps * len(cfg["fids"]) / dt,
                     "ms_per_step": dt / args.steps * 1e3,
                     "per_fid": {fid: {"objective": v["objective"],
                                       "objective_pre_polish": v["objective_pre_polish"],
                                       "iters": int(v["iters"]), "nnz": int(v["nnz"]),
                                       "polish_iters": int(v["polish_iters"])}
                                 for fid, v in last.items()}}
    # signed relative gaps: positive when the BF16 path's objective is the
    # higher one (the objective is maximised)
    f32 = {fid: out["fp32"]["per_fid"][fid]["objective"] for fid in cfg["fids"]}
    gaps = {fid: (out["bf16"]["per_fid"][fid]["objective"] - f32[fid]) / abs(f32[fid])
            for fid in cfg["fids"]}
    pre = {fid: (out["bf16"]["per_fid"][fid]["objective_pre_polish"] - f32[fid]) / abs(f32[fid])
           for fid in cfg["fids"]}
    ref_gaps = None
    ref_path = os.path.join(ROOT, "tests", "golden", "spiked_5000x50000_F1F8_reference.json")
    if os.path.exists(ref_path):
        # the FP64 oracle's best over the same 256 starts, stored
        with open(ref_path) as fh:
            ref = json.load(fh)["formulations"]
        ref_gaps = {fid: {prec: (out[prec]["per_fid"][fid]["objective"] - ref[str(fid)]["f_best"])
                          / abs(ref[str(fid)]["f_best"]) for prec in ("fp32", "bf16")}
                    for fid in cfg["fids"] if str(fid) in ref}
    return {
        "metric": "solves/s, BF16 storage + FP32 polish",
        "value": out["bf16"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": out["bf16"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16 (FP32 accumulate, FP32 polish)",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "n": n, "p": p, "starts": r,
                   "formulations": list(cfg["fids"]), "s": cfg["s"], "tol": 1e-7,
                   "maxit": cfg["maxit"]},
        "fp32_solves_per_s": out["fp32"]["solves_per_s"],
        "speedup_vs_fp32": out["bf16"]["solves_per_s"] / out["fp32"]["solves_per_s"],
        "signed_rel_gap_to_fp32_post_polish": gaps,
        "signed_rel_gap_to_fp32_pre_polish": pre,
        "post_polish_not_below_fp32": all(g >= -1e-5 for g in gaps.values()),
        "signed_rel_gap_to_fp64_oracle_best": ref_gaps,
        "paths": out,
    }


def serve_requests(count, seed, precision):
    """The serving stream: n ~ U[200, 5000], p ~ U[1000, 50000], formulation
    uniform over the 8, s ~ U[5, 200] (at most p) or gamma = 0.1 max_i
    ||a_i||_2, r in {16, 64, 256}; A is the 3-spike model (thetas 60/40/25,
    50 nonzeros per spike) generated on the device from the request's seed.
    precision: "fp32", "bf16" or "mixed" (drawn per request)."""
    from workloads import counter

    rng = np.random.default_rng(seed)
    prng = np.random.default_rng(seed + 1)  # precision draws: the shapes stay the same
    specs = []
    for i in range(count):
        n = int(rng.integers(200, 5001))
        p = int(rng.integers(1000, 50001))
        fid = int(rng.integers(1, 9))
        r = int(rng.choice([16, 64, 256]))
        s = int(rng.integers(5, 201))
        coin = prng.random()
        prec = precision if precision != "mixed" else ("bf16" if coin < 0.5 else "fp32")
        thetas = (60.0, 40.0, 25.0)
        f = counter.spike_factors(seed + i, n, p, thetas, 50)
        spec = dict(n=n, p=p, seed=seed + i, thetas=thetas, U=f.U, V=f.V,
                    start_seed=seed + 100000 + i, formulation=fid, r=r, maxit=200,
                    tol=1e-6, precision=prec, polish_maxit=200, flags=1)
        if fid <= 4:
            spec["s_or_gamma"] = float(min(s, p))
        else:
            spec["gamma_rel"] = 0.1
        specs.append(spec)
    return specs


def run_stream(spca, specs, qps, workers, arena, seed, group_limit=None):
    """Submits the requests at Poisson arrival times (all at once when qps is
    infinite) and collects them.  group_limit: requests per group of small
    requests (None: the server's default, 0: every request alone)."""
    rng = np.random.default_rng(seed + 7)
    gaps = rng.exponential(1.0 / qps, len(specs)) if np.isfinite(qps) else np.zeros(len(specs))
    done = {}
    with spca.Server(arena, workers=workers, group_limit=group_limit) as srv:
        t0 = time.monotonic()
        due = t0 + np.cumsum(gaps)
        ids = {}
        for i, spec in enumerate(specs):
            while True:
                wait = due[i] - time.monotonic()
                if wait <= 0:
                    break
                for c in srv.poll(wait_ms=max(1, int(wait * 1000))):
                    done[ids[c["id"]]] = c
            ids[srv.submit(spec)] = i
        while len(done) < len(specs):
            for c in srv.poll(wait_ms=1000):
                done[ids[c["id"]]] = c
        stats = srv.stats()
    comps = [done[i] for i in range(len(specs))]
    bad = [c for c in comps if c["rc"] != 0]
    if bad:
        raise RuntimeError(f"{len(bad)} requests failed, first: {bad[0]['error']}")
    lat = np.array([c["t_done"] - c["t_submit"] for c in comps])
    solve = np.array([c["t_done"] - c["t_solve"] for c in comps])
    first = min(c["t_submit"] for c in comps)
    last = max(c["t_done"] for c in comps)
    return {"offered_qps": qps if np.isfinite(qps) else "all at t=0",
            "solves_per_s": len(comps) / (last - first),
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "solve_only_p50_ms": float(np.percentile(solve, 50) * 1e3),
            "solve_only_p99_ms": float(np.percentile(solve, 99) * 1e3),
            "wall_s": last - first, "peak_running": stats["peak_running"],
            "peak_in_use_GB": stats["peak_in_use_bytes"] / 1e9}, comps


def bench_serve(args, spca, torch):
    """Serving: Poisson streams of requests of mixed shape, formulation and
    precision.  First the saturation rate C of the baseline (one request at
    a time, FP32, every request queued at t = 0) and of the batched paths;
    then latency at offered loads of 0.5, 1 and 2 x C, continuous batching
    with per-request precision against the baseline."""
    count = args.requests
    seed = workloads.SEED_BASE + 5
    arena = int(args.arena_gb * (1 << 30))
    runs = {}
    comps = {}
    warm = serve_requests(4, seed + 999, "mixed")
    run_stream(spca, warm, float("inf"), args.workers, arena, seed)

    def go(name, prec, workers, qps, group_limit=None):
        specs = serve_requests(count, seed, prec)
        runs[name], comps[name] = run_stream(spca, specs, qps, workers, arena, seed,
                                             group_limit)
        print(json.dumps({name: runs[name]}), file=sys.stderr, flush=True)

    # the baseline: one request at a time, each its own solve (no groups)
    go("saturated/one_at_a_time_fp32", "fp32", 1, float("inf"), 0)
    C = runs["saturated/one_at_a_time_fp32"]["solves_per_s"]
    go("saturated/batched_fp32", "fp32", args.workers, float("inf"))
    go("saturated/batched_mixed", "mixed", args.workers, float("inf"))
    go("saturated/batched_mixed_no_groups", "mixed", args.workers, float("inf"), 0)
    loads = [float(x) for x in args.loads.split(",")]
    for mult in loads:
        go(f"{mult}xC/batched_mixed", "mixed", args.workers, mult * C)
        go(f"{mult}xC/one_at_a_time_fp32", "fp32", 1, mult * C, 0)
    # accuracy, request by request: the served precision mix against the
    # FP32 one-at-a-time result of the same request
    base = comps["saturated/one_at_a_time_fp32"]
    mixed = comps["saturated/batched_mixed"]
    specs = serve_requests(count, seed, "mixed")
    bf = [i for i, sp in enumerate(specs) if sp["precision"] == "bf16"]
    signed = np.array([(mixed[i]["objective"] - base[i]["objective"]) /
                       max(abs(base[i]["objective"]), 1e-300) for i in bf])
    gaps = np.abs(signed)
    # requests outside the groups are the same solves in both runs; grouped
    # ones differ from their ungrouped solve only in the order of the sums
    small = [i for i, sp in enumerate(serve_requests(count, seed, "fp32"))
             if sp["p"] <= spca.GROUP_MAX_P and sp["n"] * sp["p"] * sp["r"] <= 5.4e8]
    same32 = all(comps["saturated/batched_fp32"][i]["objective"] == base[i]["objective"]
                 for i in range(count) if i not in set(small))
    grouped_gap = [abs(comps["saturated/batched_fp32"][i]["objective"] - base[i]["objective"])
                   / max(abs(base[i]["objective"]), 1e-300) for i in small]
    ref = f"{loads[len(loads) // 2]}xC"
    m = runs[f"{ref}/batched_mixed"]
    return {
        "metric": "solves/s with p50/p99 latency (continuous batching)",
        "value": runs["saturated/batched_mixed"]["solves_per_s"], "unit": "solves/s",
        "n_gpus": 1, "steps": count, "warmup": 4,
        "ms_per_step": runs["saturated/batched_mixed"]["wall_s"] / count * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "mixed f32 / bf16+f32 polish",
        "data": "synthetic (per-request spiked model generated in HBM)",
        "config": {"workload": f"serve-poisson-{count}req", "requests": count,
                   "workers": args.workers, "arena_GB": args.arena_gb,
                   "n": "U[200,5000]", "p": "U[1000,50000]", "formulation": "U{1..8}",
                   "s": "U[5,200]", "gamma": "0.1*max_i ||a_i||_2", "r": [16, 64, 256],
                   "precision": "50% fp32, 50% bf16+polish", "tol": 1e-6, "maxit": 200,
                   "baseline_saturation_C_per_s": C, "loads_x_C": loads},
        "p50_ms": m["p50_ms"], "p99_ms": m["p99_ms"], "latency_at": ref,
        "baseline_p50_ms": runs[f"{ref}/one_at_a_time_fp32"]["p50_ms"],
        "baseline_p99_ms": runs[f"{ref}/one_at_a_time_fp32"]["p99_ms"],
        "speedup_vs_one_at_a_time_fp32": runs["saturated/batched_mixed"]["solves_per_s"] / C,
        "batched_fp32_solves_per_s": runs["saturated/batched_fp32"]["solves_per_s"],
        "fp32_batched_equals_one_at_a_time_ungrouped": same32,
        "grouped_requests": len(small),
        "grouped_vs_alone_max_rel_gap": float(max(grouped_gap)) if grouped_gap else None,
        "batched_mixed_no_groups_solves_per_s":
            runs["saturated/batched_mixed_no_groups"]["solves_per_s"],
        "bf16_requests_objective_rel_gap_vs_fp32": {
            "count": len(bf), "median": float(np.median(gaps)),
            "p90": float(np.percentile(gaps, 90)), "max": float(gaps.max()),
            "frac_le_1e-5": float(np.mean(gaps <= 1e-5)),
            "frac_le_1e-3": float(np.mean(gaps <= 1e-3)),
            "frac_bf16_better": float(np.mean(signed > 1e-5)),
            "frac_bf16_worse": float(np.mean(signed < -1e-5)),
            "mean_signed": float(np.mean(signed))},
        "runs": runs,
    }


def bench_otf(args, spca, torch):
    """Section 4.3 on the spiked 1000 x 10000 model: 1024 starting points
    (F1 and F5, tol 1e-6, maxit 200) solved all at once (1024 slots), in 16
    sequential batches of 64, and with on-the-fly replacement through 64
    slots.  A step is one solve of all 1024 starts in each of the three
    ways; reported per way: ms per solve and iterations x starts/s."""
    cfg = workloads.SPIKED_ALL8
    n, p, l = cfg["n"], cfg["p"], cfg["r"]
    slots = args.slots
    sp = workloads.spiked_matrix(cfg["seed"], n, p, cfg["thetas"], cfg["spike_nnz"])
    A = torch.from_numpy(np.ascontiguousarray(sp.A.T)).cuda().t()
    X0 = torch.from_numpy(workloads.random_unit_starts(cfg["seed"] + 1000, l, p)).cuda()
    ctx = spca.Context(0)
    stream = torch.cuda.current_stream()
    fids = (1, 5)
    params = {fid: workloads.s_or_gamma_for(fid, sp.A, cfg["s"]) for fid in fids}
    ways = {}

    def all_at_once(fid):
        return [spca.am_solve(A, fid, params[fid], X0, tol=1e-6, maxit=200, ctx=ctx,
                              stream=stream, flags=args.flags)]

    def batches(fid):
        return [spca.am_solve(A, fid, params[fid], X0[b:b + slots].contiguous(), tol=1e-6,
                              maxit=200, ctx=ctx, stream=stream, flags=args.flags)
                for b in range(0, l, slots)]

    def otf(fid):
        return [spca.am_solve(A, fid, params[fid], X0, tol=1e-6, maxit=200, ctx=ctx,
                              stream=stream, flags=args.flags, slots=slots)]

    for name, fn in ((f"all_at_once_{l}", all_at_once), (f"batches_of_{slots}", batches),
                     (f"otf_{slots}_slots", otf)):
        for fid in fids:
            def step(timing, fn=fn, fid=fid):
                res = fn(fid)
                return {"work": sum(r["iters_x_starts"] for r in res), "kt": {},
                        "best": max(r["objective"] for r in res)}
            dt, outs = _timed_steps(step, args.steps, args.warmup)
            ways[f"{name}/F{fid}"] = {"ms_per_solve": dt / args.steps * 1e3,
                                      "iter_x_starts_per_s": sum(o["work"] for o in outs) / dt,
                                      "best_objective": outs[-1]["best"]}
    key = f"otf_{slots}_slots/F1"
    return {
        "metric": "ms per solve of 1024 starting points",
        "value": ways[key]["ms_per_solve"], "unit": "ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ways[key]["ms_per_solve"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"spiked-1000x10000-F1F5-l1024-otf{slots}", "n": n, "p": p,
                   "starting_points": l, "slots": slots, "formulations": list(fids),
                   "tol": 1e-6, "maxit": 200},
        "ways": ways,
    }


def bench_hunt(args, spca, torch):
    """Section 4.1, explained-variance hunt, on a faces-shaped stand-in: a
    400 x 10304 Gaussian matrix with rows normalised and columns centred;
    1000 random starts, maxit 200, tol 1e-6; for s = 1, 2, 4, ..., 4096 all
    8 formulations, the constraints with parameter s and the penalties with
    the sparsity-targeted warm-up (10 iterations) to s nonzeros, the L1
    constraint with lambda frozen after 10 iterations.  A step is the whole
    sweep; reported: solves/s, iterations x starts/s and the best explained
    variance per formulation and s."""
    rng = np.random.default_rng(workloads.SEED_BASE + 7)
    n, p, l = 400, 10304, 1000
    A_np = rng.standard_normal((n, p))
    A_np /= np.linalg.norm(A_np, axis=1, keepdims=True)
    A_np -= A_np.mean(axis=0, keepdims=True)
    A = torch.from_numpy(np.ascontiguousarray(A_np.astype(np.float32).T)).cuda().t()
    X0 = torch.from_numpy(workloads.random_unit_starts(workloads.SEED_BASE + 8, l, p)).cuda()
    ctx = spca.Context(0)
    stream = torch.cuda.current_stream()
    svals = [2 ** k for k in range(13)]
    best = {}

    def step(timing):
        work = 0.0
        for fid in range(1, 9):
            for sv in svals:
                if fid <= 2:
                    res = spca.am_solve(A, fid, float(sv), X0, tol=1e-6, maxit=200, ctx=ctx,
                                        stream=stream, flags=args.flags)
                elif fid <= 4:
                    res = spca.am_solve(A, fid, float(sv), X0, tol=1e-6, maxit=200, ctx=ctx,
                                        stream=stream, flags=args.flags, warmup_iters=10)
                else:
                    res = spca.am_solve(A, fid, 0.0, X0, tol=1e-6, maxit=200, ctx=ctx,
                                        stream=stream, flags=args.flags, warmup_iters=10,
                                        target_nnz=sv)
                work += res["iters_x_starts"]
                best[f"F{fid}/s={sv}"] = (round(res["explained_variance"], 6), int(res["nnz"]))
        return {"work": work, "kt": {}}

    dt, outs = _timed_steps(step, args.steps, args.warmup)
    solves = 8 * len(svals)
    return {
        "metric": "solves/s (explained-variance hunt sweep)",
        "value": solves * args.steps / dt, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (faces-shaped stand-in: Gaussian rows normalised, columns centred)",
        "config": {"workload": "hunt-400x10304-l1000-s1to4096", "n": n, "p": p,
                   "starting_points": l, "s": svals, "formulations": list(range(1, 9)),
                   "warmup_iters": 10, "tol": 1e-6, "maxit": 200},
        "iter_x_starts_per_s": sum(o["work"] for o in outs) / dt,
        "best_explained_variance_and_nnz": best,
    }


def bench_components(args, spca, torch):
    """The first 5 sparse components (deflation) on the spiked 1000 x 10000
    model, F1 with s = 50, 1024 starts, tol 1e-6, maxit 200."""
    cfg = workloads.SPIKED_ALL8
    n, p, r = cfg["n"], cfg["p"], cfg["r"]
    sp = workloads.spiked_matrix(cfg["seed"], n, p, cfg["thetas"], cfg["spike_nnz"])
    A = torch.from_numpy(np.ascontiguousarray(sp.A.T)).cuda().t()
    X0 = torch.from_numpy(workloads.random_unit_starts(cfg["seed"] + 1000, r, p)).cuda()
    ctx = spca.Context(0)
    out = {}

    def step(timing):
        comps = spca.am_components(A, 1, float(cfg["s"]), X0, 5, tol=1e-6, maxit=200,
                                   ctx=ctx, flags=args.flags)
        out["comps"] = comps
        return {"work": 5, "kt": {}}

    dt, outs = _timed_steps(step, args.steps, args.warmup)
    comps = out["comps"]
    planted = [set(s_.tolist()) for s_ in sp.supports]
    return {
        "metric": "components/s (deflation)", "value": 5 * args.steps / dt,
        "unit": "components/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "spiked-1000x10000-F1-s50-r1024-5components", "n": n, "p": p,
                   "starts": r, "components": 5, "tol": 1e-6, "maxit": 200},
        "components": [{"objective": c["objective"], "nnz": int(c["nnz"]),
                        "overlap_with_planted": [len(set(c["support"].tolist()) & s_)
                                                 for s_ in planted]} for c in comps],
    }


def bench_sparse(args, spca, torch):
    """Sparse A shaped like the paper's NYTimes bag of words (300000 documents
    x 102660 words, about 70M nonzero counts, Zipf word frequencies,
    generated on the host from a seed), F1 with s = 5 from 20 random starts,
    maxit 20, tol 1e-6 (the paper's setting for that corpus).  A step is one
    solve."""
    from workloads import sparse as sparse_w

    mat = sparse_w.bag_of_words(workloads.SEED_BASE + 9, 300000, 102660, 103_000_000)
    D = spca.sparse_to_device(mat)
    r = args.starts or 20
    X0 = torch.from_numpy(workloads.random_unit_starts(workloads.SEED_BASE + 10, r,
                                                       mat.p)).cuda()
    ctx = spca.Context(0)
    last = {}
    flags = args.flags | {"auto": 0, "on": spca.FLAG_SPARSE_PANELS,
                          "off": spca.FLAG_SPARSE_NO_PANELS}[args.panels]

    def step(timing):
        res = spca.am_solve_sparse(D, 1, 5.0, X0, tol=1e-6, maxit=20, ctx=ctx, flags=flags)
        last.update(res)
        return {"work": res["iters_x_starts"], "kt": {}}

    dt, outs = _timed_steps(step, args.steps, args.warmup)
    counts = np.diff(mat.col_ptr)
    # every formulation once with the same starts (20 iterations, tol 1e-6):
    # s = 5 for the constraints; for the penalties gamma comes from the
    # sparsity-targeted warm-up (5 iterations, 5 nonzeros), not from a guess
    per_fid = {}
    for fid in range(1, 9):
        kw = {} if fid <= 4 else {"warmup_iters": 5, "target_nnz": 5}
        par = 5.0 if fid <= 4 else 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = spca.am_solve_sparse(D, fid, par, X0, tol=1e-6, maxit=20, ctx=ctx, flags=flags,
                                   **kw)
        torch.cuda.synchronize()
        per_fid[str(fid)] = {"ms": (time.perf_counter() - t0) * 1e3,
                             "objective": res["objective"],
                             "explained_variance": res["explained_variance"],
                             "nnz": int(len(res["support"])), "iters": int(res["iters"])}
    # the first five components by deflation (the paper lists several per
    # corpus), F1, s = 5, the same starts
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    comps = spca.am_components_sparse(D, 1, 5.0, X0, 5, tol=1e-6, maxit=20, ctx=ctx,
                                      flags=flags)
    torch.cuda.synchronize()
    comp_ms = (time.perf_counter() - t0) * 1e3
    components = {"ms_for_5": comp_ms,
                  "supports": [c["support"].tolist() for c in comps],
                  "objectives": [c["objective"] for c in comps]}
    # A^T Y per launch with every start running (stop test off, 8 iterations),
    # HIP events on the solve's stream
    kt = spca.am_solve_sparse(D, 1, 5.0, X0, tol=-1.0, maxit=8, ctx=ctx, flags=flags,
                              kernel_times=True)["kernel_times"]
    aty_ms = kt["aty_ms"] / kt["aty_launches"]
    aty_bytes = mat.nnz * 8 + (mat.n + mat.p) * r * 4
    return {
        "metric": "solves/s (sparse A)", "value": args.steps / dt, "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (Zipf bag-of-words stand-in for the NYTimes corpus)",
        "config": {"workload": "bagofwords-300000x102660-F1-s5", "n": mat.n, "p": mat.p,
                   "nnz": mat.nnz, "largest_column": int(counts.max()), "starts": r,
                   "tol": 1e-6, "maxit": 20},
        "iter_x_starts_per_s": sum(o["work"] for o in outs) / dt,
        "result": {"objective": last["objective"], "support": last["support"].tolist(),
                   "iters": int(last["iters"])},
        "all_formulations": per_fid,
        "components": components,
        "roofline": {"kernel": "sp_seg_kernel (V = A^T Y, columns)", "bound": "hbm",
                     "achieved": aty_bytes / (aty_ms * 1e-3) / 1e9, "peak": 8000.0,
                     "unit": "GB/s", "frac": aty_bytes / (aty_ms * 1e-3) / 8e12,
                     "traffic": None, "avg_launch_ms": aty_ms,
                     "launches": kt["aty_launches"],
                     "algorithmic_bytes": aty_bytes,
                     "note": "8 B per nonzero (row index, value) + Y + V; the kernel is "
                             "bound by random row reads of Y, not HBM"},
    }


def bench_secondary(args, spca, torch, main_rec):
    """The other configurations, short, beside the headline line: the
    headline step with its solves on 4 streams at once (throughput only),
    the BF16 + polish precision study (5000 x 50000, 2 steps), the 16 GB
    instance (2 steps of 30 iterations) and a 2000-request serving stream at
    a fixed offered load, batched with mixed precision and the
    one-request-at-a-time FP32 baseline.  A failing part records its error
    instead of ending the run."""
    import copy
    import gc

    out = {}

    def part(name, fn):
        t0 = time.monotonic()
        try:
            out[name] = fn()
        except Exception as e:  # recorded, the headline line still prints
            out[name] = {"error": f"{type(e).__name__}: {e}"}
        out[name]["wall_s"] = round(time.monotonic() - t0, 1)
        gc.collect()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        print(json.dumps({name: out[name]})[:400], file=sys.stderr, flush=True)

    a = copy.copy(args)
    a.steps, a.warmup, a.maxit = 2, 1, 0

    def precision():
        r = bench_precision(a, spca, torch)
        return {k: r[k] for k in ("metric", "value", "unit", "ms_per_step", "fp32_solves_per_s",
                                  "speedup_vs_fp32", "signed_rel_gap_to_fp32_post_polish",
                                  "signed_rel_gap_to_fp32_pre_polish", "post_polish_not_below_fp32",
                                  "signed_rel_gap_to_fp64_oracle_best", "config")}

    def large():
        r = bench_large(a, spca, torch)
        spca.tune_table_clear()  # its entries are for this instance's products only
        return {k: r[k] for k in ("metric", "value", "unit", "ms_per_step", "roofline", "config",
                                  "autotuned", "gemm_plans_shape_splits")}

    def serve():
        count, qps = args.serve_requests, args.serve_qps
        seed = workloads.SEED_BASE + 5
        arena = int(args.arena_gb * (1 << 30))
        run_stream(spca, serve_requests(4, seed + 999, "mixed"), float("inf"), args.workers,
                   arena, seed)
        batched, _ = run_stream(spca, serve_requests(count, seed, "mixed"), qps, args.workers,
                                arena, seed)
        base, _ = run_stream(spca, serve_requests(count, seed, "fp32"), qps, 1, arena, seed, 0)
        return {"metric": "solves/s with p50/p99 latency at a fixed offered load",
                "requests": count, "offered_qps": qps,
                "batched_mixed": batched, "one_at_a_time_fp32": base,
                "speedup_solves_per_s": batched["solves_per_s"] / base["solves_per_s"],
                "config": {"workload": f"serve-poisson-{count}req-{qps:g}qps",
                           "n": "U[200,5000]", "p": "U[1000,50000]", "formulation": "U{1..8}",
                           "r": [16, 64, 256], "precision": "50% fp32, 50% bf16+polish (batched); "
                           "fp32 (baseline)", "workers": args.workers, "tol": 1e-6, "maxit": 200}}

    def concurrent():
        # the headline step with its 8 solves on 4 streams at once, no
        # kernel events (events of overlapping kernels measure time shared
        # with the other streams, so the kernel roofline stays with the
        # sequential line above)
        b = copy.copy(args)
        b.streams, b.steps, b.warmup, b.no_cpu_baseline = 4, 3, 1, True
        r = bench_all8(b, spca, torch, timed_events=False)
        t_bound = main_rec["path_roofline"]["t_bound_ms"]  # the same work
        return {"metric": r["metric"], "value": r["value"], "unit": r["unit"],
                "ms_per_step": r["ms_per_step"],
                "path_roofline_frac": round(t_bound / r["ms_per_step"], 4),
                "concurrent_solves": 4, "solves_per_stream": r["config"]["solves_per_stream"]}

    part("headline_concurrent", concurrent)
    part("precision", precision)
    part("large", large)
    part("serve", serve)
    return out


WORKLOADS = {"spiked-all8": bench_all8, "otf": bench_otf, "hunt": bench_hunt,
             "sparse": bench_sparse,
             "components": bench_components, "large": bench_large, "precision": bench_precision,
             "serve": bench_serve}


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="spiked-all8", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fids", default="1,2,3,4,5,6,7,8",
                    help="formulations in a step of spiked-all8 (default: all 8)")
    ap.add_argument("--maxit", type=int, default=0, help="iterations per solve (large)")
    ap.add_argument("--slots", type=int, default=64, help="otf: slots")
    ap.add_argument("--starts", type=int, default=0, help="sparse: starting points")
    ap.add_argument("--panels", default="auto", choices=("auto", "on", "off"),
                    help="sparse: row panels of the columns for A^T Y")
    ap.add_argument("--requests", type=int, default=200, help="serve: requests")
    ap.add_argument("--loads", default="0.5,1,2",
                    help="serve: offered loads as multiples of the baseline saturation rate")
    ap.add_argument("--workers", type=int, default=4, help="serve: concurrent solves")
    ap.add_argument("--arena-gb", type=float, default=64.0, help="serve: HBM arena")
    ap.add_argument("--autotune", action="store_true",
                    help="spiked-all8: time every tile shape and split first")
    ap.add_argument("--no-autotune", action="store_true",
                    help="large: plan the tiles from the model instead of tuning them first")
    ap.add_argument("--no-union", action="store_true",
                    help="keep the planner off the union-of-supports product")
    ap.add_argument("--graph", action="store_true",
                    help="replay the iterations from a captured HIP graph")
    ap.add_argument("--streams", type=int, default=1,
                    help="spiked-all8: run the step's solves on this many streams at once")
    ap.add_argument("--no-secondary", action="store_true",
                    help="spiked-all8: skip the short runs of the other configurations")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="secondary serving stream: requests")
    ap.add_argument("--serve-qps", type=float, default=40.0,
                    help="secondary serving stream: offered load (requests/s)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: "
              "the batched AM path runs on a single MI355X", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1212_4137_amd as spca

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    args.flags = (spca.FLAG_GRAPH if args.graph else 0) | (spca.FLAG_NO_UNION if args.no_union else 0)
    rec = WORKLOADS[args.workload](args, spca, torch)
    if args.workload == "spiked-all8" and not args.no_secondary and args.fids == "1,2,3,4,5,6,7,8":
        rec["secondary"] = bench_secondary(args, spca, torch, rec)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
