"""The oracle's sparse (compressed sparse columns) AM is the dense AM on the
same matrix, bit for bit: the products only skip terms that are zero; and
the sparse generator's two layouts describe the same matrix."""
import numpy as np
import pytest

import oracle
import workloads
from workloads import sparse


@pytest.fixture(scope="module")
def mat():
    return sparse.bag_of_words(31, 150, 400, 6000)


def test_layouts_agree(mat):
    A = mat.dense()
    rows = np.repeat(np.arange(mat.n), np.diff(mat.row_ptr))
    B = np.zeros_like(A)
    B[rows, mat.col_idx] = mat.row_val
    assert np.array_equal(A, B)
    assert mat.nnz == np.count_nonzero(A)
    for c in range(0, mat.p, 37):
        seg = mat.row_idx[mat.col_ptr[c]:mat.col_ptr[c + 1]]
        assert np.all(np.diff(seg) > 0)
    # Zipf: the first words are the most frequent
    counts = np.diff(mat.col_ptr)
    assert counts[:10].mean() > 5 * counts[-100:].mean()


@pytest.mark.parametrize("fid", range(1, 9))
def test_sparse_oracle_equals_dense_oracle(mat, fid):
    A = mat.dense()
    X0 = workloads.random_unit_starts(32, 6, mat.p)
    par = {1: 10, 2: 10, 3: 4.0, 4: 4.0}.get(fid, None)
    if par is None:
        par = workloads.s_or_gamma_for(fid, A, 10, "scaled")
    d = oracle.am_multi(A, fid, par, X0, 1e-9, 300)
    s = oracle.am_multi_csc(mat.col_ptr, mat.row_idx, mat.col_val, mat.n, mat.p, fid, par,
                            X0, 1e-9, 300, nthreads=3)
    assert np.array_equal(d["X"], s["X"])
    assert np.array_equal(d["f"], s["f"]) and np.array_equal(d["ev"], s["ev"])
    assert d["best"] == s["best"] and np.array_equal(d["iters"], s["iters"])
