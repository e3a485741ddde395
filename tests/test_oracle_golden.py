"""Regression of the oracle against its stored small-workload result.

The fixture was written by tests/golden/make_golden.py, which calls only the
oracle; the pins in test_oracle_operators.py and test_oracle_am.py are what
tie the oracle to the paper.  This test guards against silent drift.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gauss_100x500_F1_s10.json")


def test_small_single_start_matches_stored_result():
    with open(GOLDEN) as fh:
        g = json.load(fh)
    cfg = workloads.SMALL_SINGLE_START
    A = workloads.gaussian_matrix(cfg["seed"], cfg["n"], cfg["p"])
    x0 = oracle.unit_vector_start(A)
    assert int(np.flatnonzero(x0)[0]) == g["start_column"]
    out = oracle.am_single(A, cfg["fid"], cfg["s"], x0, cfg["tol"], cfg["maxit"])
    assert out["f"] == pytest.approx(g["f"], rel=1e-13)
    assert out["ev"] == pytest.approx(g["explained_variance"], rel=1e-13)
    assert out["iters"] == g["iters"] and out["status"] == g["status"]
    assert np.flatnonzero(out["x"]).tolist() == g["support"]
    # F1 value is sigma_max of the support's columns at a fixed point of T_s
    S = g["support"]
    sig = np.linalg.svd(A[:, S].astype(np.float64), compute_uv=False)[0]
    assert g["f"] == pytest.approx(sig, rel=1e-7)
