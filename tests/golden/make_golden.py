"""Writes the stored expected values under tests/golden/ from the FP64 oracle.

Calls only ``oracle`` and the seeded input generators in ``workloads``.
Run from the repository root:  python -m tests.golden.make_golden
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def small_single_start():
    cfg = workloads.SMALL_SINGLE_START
    A = workloads.gaussian_matrix(cfg["seed"], cfg["n"], cfg["p"])
    x0 = oracle.unit_vector_start(A)
    out = oracle.am_single(A, cfg["fid"], cfg["s"], x0, cfg["tol"], cfg["maxit"])
    support = np.flatnonzero(out["x"]).tolist()
    rec = {
        "citation": "Algorithm 2 with the L0-constraint x-update T_s (Table 3, S3) "
                    "and the ratio stop test of Section 2.2; FP64 oracle",
        "workload": cfg["name"],
        "seed": cfg["seed"], "n": cfg["n"], "p": cfg["p"], "s": cfg["s"],
        "tol": cfg["tol"], "maxit": cfg["maxit"],
        "start_column": int(np.flatnonzero(x0)[0]),
        "f": out["f"], "explained_variance": out["ev"], "iters": out["iters"],
        "status": out["status"], "support": support,
        "x_support_values": [float(out["x"][i]) for i in support],
    }
    with open(os.path.join(HERE, "gauss_100x500_F1_s10.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    return rec


if __name__ == "__main__":
    r = small_single_start()
    print(r["f"], r["iters"], r["support"])
