"""Writes tests/golden/spiked_5000x50000_F1F8_reference.json: the FP64
oracle's multi-start AM (Algorithm 2 from each start, the best start by the
objective of Table 1) on the 5000 x 50000 spiked workload of the precision
study, from its 256 seeded starts, for F1 (s = 100) and F8 (gamma =
0.1 max_i ||a_i||_2), tol 1e-7, maxit 200.  The reference the BF16 + FP32
polish results are compared with.

Calls only ``oracle`` and the seeded input generators in ``workloads``; it
takes tens of minutes of CPU.  Run from the repository root:
    python -m tests.golden.make_precision_reference [threads]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "spiked_5000x50000_F1F8_reference.json")


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else max(1, len(os.sched_getaffinity(0)) - 2)
    cfg = workloads.SPIKED_BF16
    sp = workloads.spiked_matrix(cfg["seed"], cfg["n"], cfg["p"], cfg["thetas"], cfg["spike_nnz"])
    X0 = workloads.random_unit_starts(cfg["seed"] + 1000, cfg["r"], cfg["p"])
    rec = {"citation": "Algorithm 2 (stop test of Section 2.2) from every start, best start by "
                       "f of Table 1 (Section 4); FP64 oracle on the FP32 matrix",
           "workload": cfg["name"], "tol": 1e-7, "maxit": cfg["maxit"], "starts": cfg["r"],
           "formulations": {}}
    for fid in cfg["fids"]:
        par = workloads.s_or_gamma_for(fid, sp.A, cfg["s"])
        t0 = time.time()
        res = oracle.am_multi(sp.A, fid, par, X0, 1e-7, cfg["maxit"], nthreads=threads,
                              want_x=False)
        srt = np.sort(res["f"])[::-1]
        rec["formulations"][str(fid)] = {
            "s_or_gamma": par, "best": int(res["best"]), "f_best": float(res["f"][res["best"]]),
            "top2_gap": float((srt[0] - srt[1]) / abs(srt[0])),
            "f": res["f"].tolist(), "iters": res["iters"].tolist(),
            "status": res["status"].tolist(), "seconds": time.time() - t0}
        print(f"F{fid}: best {res['best']} f {res['f'][res['best']]:.12g} "
              f"({time.time() - t0:.0f} s)", flush=True)
        with open(OUT, "w") as fh:
            json.dump(rec, fh)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
