"""Pins of the oracle's deflation for further components (projection
deflation of the data matrix, A_t = A_{t-1} (I - x_t x_t^T)):

* with s = p (no sparsity) AM is the power method, and the loadings of
  successive components are the right singular vectors: the objectives are
  sigma_1, sigma_2, sigma_3 of A from a dense SVD;
* the deflated matrix annihilates the loading it was deflated by, and keeps
  A x for every x orthogonal to it;
* deflating by nothing is the plain solve."""
import numpy as np
import pytest

import oracle
import workloads


def test_components_of_the_power_method_are_singular_values():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((40, 25))
    sig = np.linalg.svd(A, compute_uv=False)
    X0 = workloads.random_unit_starts(8, 3, 25)
    for fid in (1, 3):
        comps = oracle.am_components(A, fid, 25.0, X0, 3, 1e-14, 5000)
        for t in range(3):
            assert abs(comps[t]["f"] - sig[t]) <= 1e-9 * sig[0], (fid, t)


def test_deflation_annihilates_and_keeps_orthogonal_directions():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((30, 50))
    x = np.zeros(50)
    x[[3, 7, 20]] = rng.standard_normal(3)
    x /= np.linalg.norm(x)
    D = oracle.deflate(A, x)
    assert np.max(np.abs(D @ x)) <= 1e-13
    z = rng.standard_normal(50)
    z -= x * (x @ z)
    np.testing.assert_allclose(D @ z, A @ z, rtol=0, atol=1e-12)
    np.testing.assert_allclose(D, A - np.outer(A @ x, x), rtol=0, atol=1e-13)


def test_sparse_second_component_on_disjoint_spikes():
    # two planted components on disjoint supports: the second loading is
    # found on the second support after deflating the first
    sp = workloads.spiked_matrix(13, 200, 600, thetas=(150.0, 100.0), spike_nnz=10)
    X0 = workloads.random_unit_starts(14, 16, 600)
    comps = oracle.am_components(sp.A, 1, 10, X0, 2, 1e-10, 500)
    s1 = set(np.flatnonzero(comps[0]["x"]))
    s2 = set(np.flatnonzero(comps[1]["x"]))
    assert s1 == set(sp.supports[0]) and s2 == set(sp.supports[1])
    assert comps[1]["f"] < comps[0]["f"]


def test_one_component_is_the_plain_solve():
    sp = workloads.spiked_matrix(15, 60, 200, thetas=(30.0,), spike_nnz=8)
    X0 = workloads.random_unit_starts(16, 4, 200)
    a = oracle.am_multi(sp.A, 7, 0.5, X0, 1e-9, 300)
    (c,) = oracle.am_components(sp.A, 7, 0.5, X0, 1, 1e-9, 300)
    assert c["f"] == a["f"][a["best"]] and np.array_equal(c["x"], a["X"][a["best"]])
