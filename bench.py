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
product V = A^T Y, timed with HIP events on the solve's stream) and the
FP64 CPU oracle's throughput on a bounded sample of the same workload.

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


def cpu_baseline(A_np, X0_np, params, maxit_sample=25):
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


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fids", default="1,2,3,4,5,6,7,8",
                    help="formulations in a step (default: all 8)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: "
              "the batched AM path runs on a single MI355X", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1212_4137_amd as spca

    assert torch.cuda.is_available(), "bench.py needs a GPU"
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
    ctx = spca.Context(0)
    stream = torch.cuda.current_stream()

    modes = {}

    def step(timing):
        work = 0.0
        kt = {}
        nnz = {}
        for fid in fids:
            res = spca.am_solve(A, fid, params[fid], X0, tol=-1.0, maxit=maxit,
                                ctx=ctx, stream=stream, kernel_times=timing)
            work += res["iters_x_starts"]
            nnz[fid] = float(np.mean(res["nnz_per_start"]))
            if timing:
                for k, v in res["kernel_times"].items():
                    kt[k] = kt.get(k, 0) + v
                t = res["kernel_times"]
                modes[fid] = (t["iters_dense"], t["iters_list"], t["iters_union"])
        return work, kt, nnz

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    work = 0.0
    kt_all = {}
    nnz = {}
    for _ in range(args.steps):
        w, kt, nnz = step(True)
        work += w
        for k, v in kt.items():
            kt_all[k] = kt_all.get(k, 0) + v
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    # dominant kernel: V = A^T Y, 2 r n p flops per launch (dense product)
    launches = kt_all["aty_launches"]
    avg_ms = kt_all["aty_ms"] / launches
    flops = 2.0 * r * n * p
    achieved = flops / (avg_ms * 1e-3) / 1e12
    roofline = {"kernel": "gemm_nt_f32 (V = A^T Y)", "bound": "mfma",
                "achieved": round(achieved, 2), "peak": PEAK_FP32_MFMA_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_MFMA_TFLOPS, 4),
                "traffic": None, "avg_launch_ms": round(avg_ms, 5),
                "launches": int(launches)}
    other = {"x_update_avg_ms": round(kt_all["x_update_ms"] / kt_all["x_update_launches"], 5),
             "ax_dense_avg_ms": round(kt_all["ax_dense_ms"] / kt_all["ax_dense_launches"], 5),
             "mean_nnz_per_start": nnz,
             "ax_modes_dense_list_union": modes}

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
                   "spikes": list(cfg["thetas"]), "spike_nnz": cfg["spike_nnz"]},
        "roofline": roofline,
        "kernels": other,
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(A_np, X0_np, params)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
