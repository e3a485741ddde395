"""Sparse A (bag-of-words stand-in for the paper's text corpora) through
spca_am_solve_sparse: parity with the oracle's sparse AM (itself bitwise the
dense oracle), agreement with the dense GPU path on the same matrix, long
rows (chunked x-update), graph replay and the warm-up."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import compare_solve, rel_err, to_device_colmajor, to_device_rows
from workloads import sparse

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def spca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1212_4137_amd as m

    m.load()
    return m


def _param(fid, mat):
    if fid <= 2:
        return 10.0
    if fid <= 4:
        return 4.0
    return workloads.s_or_gamma_for(fid, mat.dense(), 10, "scaled")


@pytest.mark.parametrize("fid", range(1, 9))
def test_sparse_matches_oracle(spca, fid):
    print(f"sparse case fid={fid}", flush=True)
    mat = sparse.bag_of_words(41, 1500, 3000, 60000)
    X0n = workloads.random_unit_starts(42, 32, mat.p)
    par = _param(fid, mat)
    D = spca.sparse_to_device(mat)
    got = spca.am_solve_sparse(D, fid, par, to_device_rows(X0n), tol=1e-8, maxit=300)
    ref = oracle.am_multi_csc(mat.col_ptr, mat.row_idx, mat.col_val.astype(np.float64), mat.n,
                              mat.p, fid, par, X0n.astype(np.float64), 1e-8, 300, nthreads=8)
    compare_solve(got, ref, f"sparse F{fid}")
    dense = spca.am_solve(to_device_colmajor(mat.dense().astype(np.float32)), fid, par,
                          to_device_rows(X0n), tol=1e-8, maxit=300)
    assert rel_err(got["objective"], dense["objective"]) <= 1e-5


@pytest.mark.parametrize("fid", [1, 3, 7])
def test_sparse_long_rows_and_graph(spca, fid):
    mat = sparse.bag_of_words(43, 800, 20000, 50000)
    X0n = workloads.random_unit_starts(44, 12, mat.p)
    X0 = to_device_rows(X0n)
    par = _param(fid, mat)
    D = spca.sparse_to_device(mat)
    got = spca.am_solve_sparse(D, fid, par, X0, tol=1e-8, maxit=300, return_X=True)
    ref = oracle.am_multi_csc(mat.col_ptr, mat.row_idx, mat.col_val.astype(np.float64), mat.n,
                              mat.p, fid, par, X0n.astype(np.float64), 1e-8, 300, nthreads=6)
    compare_solve(got, ref, f"sparse long rows F{fid}")
    g = spca.am_solve_sparse(D, fid, par, X0, tol=1e-8, maxit=300, return_X=True,
                             flags=spca.FLAG_GRAPH)
    assert g["objective"] == got["objective"] and torch.equal(g["X_final"], got["X_final"])


def test_sparse_warmup_and_checks(spca):
    mat = sparse.bag_of_words(45, 600, 2000, 30000)
    X0n = workloads.random_unit_starts(46, 16, mat.p)
    D = spca.sparse_to_device(mat)
    got = spca.am_solve_sparse(D, 7, 0.0, to_device_rows(X0n), tol=-1.0, maxit=30,
                               warmup_iters=6, target_nnz=12)
    ref = oracle.am_multi_warm(mat.dense(), 7, 0.0, X0n.astype(np.float64), -1.0, 30, 6, 12,
                               nthreads=8)
    ok = np.array([rel_err(a, b) <= 1e-5 for a, b in zip(got["f_per_start"], ref["f"])])
    assert ok.mean() >= 0.9
    with pytest.raises(spca.SpcaError):
        spca.am_solve_sparse(D, 1, 5000.0, to_device_rows(X0n))
