"""Sparse A (bag-of-words stand-in for the paper's text corpora) through
spca_am_solve_sparse: parity with the oracle's sparse AM (itself bitwise the
dense oracle), agreement with the dense GPU path on the same matrix, long
rows (chunked x-update), graph replay and the warm-up."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import compare_solve, gpu_stepper, rel_err, to_device_colmajor, to_device_rows
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
    X0d = to_device_rows(X0n)
    got = spca.am_solve_sparse(D, fid, par, X0d, tol=1e-8, maxit=300, return_X=True)
    ref = oracle.am_multi_csc(mat.col_ptr, mat.row_idx, mat.col_val.astype(np.float64), mat.n,
                              mat.p, fid, par, X0n.astype(np.float64), 1e-8, 300, nthreads=8)
    compare_solve(got, ref, f"sparse F{fid}", mat.dense(), fid, par, X0=X0n,
                  stepper=gpu_stepper(spca.am_solve_sparse, D, fid, par, X0d, tol=1e-8))
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
    compare_solve(got, ref, f"sparse long rows F{fid}", mat.dense(), fid, par, X0=X0n,
                  stepper=gpu_stepper(spca.am_solve_sparse, D, fid, par, X0, tol=1e-8))
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


def _from_columns(n, cols):
    """SparseMatrix from per-column (rows, values), rows ascending."""
    p = len(cols)
    col_ptr = np.zeros(p + 1, dtype=np.int64)
    col_ptr[1:] = np.cumsum([len(rw) for rw, _ in cols])
    row_idx = np.concatenate([rw for rw, _ in cols]).astype(np.int32)
    col_val = np.concatenate([v for _, v in cols]).astype(np.float32)
    col = np.repeat(np.arange(p), np.diff(col_ptr))
    order = np.lexsort((col, row_idx))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(row_idx, minlength=n), out=row_ptr[1:])
    return sparse.SparseMatrix(n, p, col_ptr, row_idx, col_val, row_ptr,
                               col[order].astype(np.int32), col_val[order])


def _chunk_boundary_matrix():
    """Columns laid out so that nonzero chunks of 2048 end exactly at column
    ends followed by empty columns, one column spans several chunks, and the
    first and last columns and rows are empty."""
    rng = np.random.default_rng(0x5BA5E)
    n = 5000

    def col(k, lo=5, hi=4990):
        rows = np.sort(rng.choice(np.arange(lo, hi), size=k, replace=False))
        return rows, rng.integers(1, 6, size=k).astype(np.float32)

    empty = (np.zeros(0, np.int64), np.zeros(0, np.float32))
    cols = [empty, col(2048), empty, empty, col(2148), col(1948), empty, col(4980, 5, 4985)]
    cols += [col(int(k)) for k in rng.integers(1, 41, size=300)]
    cols += [empty, empty, empty]
    mat = _from_columns(n, cols)
    assert mat.col_ptr[2] == 2048 and mat.col_ptr[6] == 3 * 2048
    return mat


@pytest.mark.parametrize("r", [4, 12, 20, 33, 40, 70])
@pytest.mark.parametrize("panels", [False, True])
def test_sparse_chunk_boundaries(spca, r, panels):
    """Every start-block width of the balanced products (4 .. 32 starts per
    block; two or three blocks above 32) over chunk-aligned column ends,
    empty columns and rows, and a column crossing several chunks; with and
    without the row-panel copy of the columns."""
    print(f"sparse chunk boundaries r={r} panels={panels}", flush=True)
    mat = _chunk_boundary_matrix()
    X0n = workloads.random_unit_starts(48 + r, r, mat.p)
    D = spca.sparse_to_device(mat)
    flags = spca.FLAG_SPARSE_PANELS if panels else spca.FLAG_SPARSE_NO_PANELS
    dense = mat.dense()
    for fid, par in ((1, 10.0), (6, workloads.s_or_gamma_for(6, dense, 10, "scaled"))):
        X0d = to_device_rows(X0n)
        got = spca.am_solve_sparse(D, fid, par, X0d, tol=1e-8, maxit=200,
                                   flags=flags, return_X=True)
        ref = oracle.am_multi_csc(mat.col_ptr, mat.row_idx, mat.col_val.astype(np.float64),
                                  mat.n, mat.p, fid, par, X0n.astype(np.float64), 1e-8, 200,
                                  nthreads=8)
        compare_solve(got, ref, f"sparse boundaries F{fid} r={r} panels={panels}", dense,
                      fid, par, X0=X0n,
                      stepper=gpu_stepper(spca.am_solve_sparse, D, fid, par, X0d, tol=1e-8,
                                          flags=flags))


def test_sparse_heavy_column(spca):
    """Zipf words steep enough that the top column holds most documents and
    crosses many nonzero chunks; parity with the oracle and with the dense
    GPU path."""
    mat = sparse.bag_of_words(47, 30000, 400, 600000, zipf=1.3)
    assert np.diff(mat.col_ptr).max() > 8 * 2048
    X0n = workloads.random_unit_starts(49, 20, mat.p)
    D = spca.sparse_to_device(mat)
    dense_np = mat.dense()
    ref = oracle.am_multi_csc(mat.col_ptr, mat.row_idx, mat.col_val.astype(np.float64), mat.n,
                              mat.p, 1, 5.0, X0n.astype(np.float64), 1e-8, 300, nthreads=8)
    dense = spca.am_solve(to_device_colmajor(dense_np.astype(np.float32)), 1, 5.0,
                          to_device_rows(X0n), tol=1e-8, maxit=300)
    for flags in (spca.FLAG_SPARSE_NO_PANELS, spca.FLAG_SPARSE_PANELS,
                  spca.FLAG_SPARSE_PANELS | spca.FLAG_GRAPH):
        X0d = to_device_rows(X0n)
        got = spca.am_solve_sparse(D, 1, 5.0, X0d, tol=1e-8, maxit=300,
                                   flags=flags, return_X=True)
        compare_solve(got, ref, f"sparse heavy column flags={flags}", dense_np, 1, 5.0,
                      X0=X0n, stepper=gpu_stepper(spca.am_solve_sparse, D, 1, 5.0, X0d,
                                                  tol=1e-8, flags=flags))
        assert rel_err(got["objective"], dense["objective"]) <= 1e-5
        if flags & spca.FLAG_GRAPH:
            assert torch.equal(got["X_final"], eager["X_final"])
        eager = got


def test_sparse_rejects_malformed(spca):
    """Malformed arrays (sized consistently with their pointer arrays) are
    rejected by the solve's checks before any product runs."""
    mat = _chunk_boundary_matrix()
    X0 = to_device_rows(workloads.random_unit_starts(50, 4, mat.p))
    base = spca.sparse_to_device(mat)
    spca.am_solve_sparse(base, 1, 10.0, X0, maxit=5)

    def bad(**repl):
        D = dict(base)
        for k, v in repl.items():
            D[k] = torch.from_numpy(v).cuda()
        with pytest.raises(spca.SpcaError):
            spca.am_solve_sparse(D, 1, 10.0, X0, maxit=5)

    ri = mat.row_idx.copy()
    ri[3000] = mat.n
    bad(row_idx=ri)
    ci = mat.col_idx.copy()
    ci[10] = -1
    bad(col_idx=ci)
    ri = mat.row_idx.copy()
    ri[[100, 101]] = ri[[101, 100]]
    bad(row_idx=ri)
    cp = mat.col_ptr.copy()
    cp[[5, 6]] = cp[[6, 5]]
    bad(col_ptr=cp)
    rp = mat.row_ptr.copy()
    rp[-1] -= 1
    bad(row_ptr=rp)


@pytest.mark.parametrize("fid", [1, 3, 7])
@pytest.mark.parametrize("panels", [False, True])
def test_sparse_components_match_oracle(spca, fid, panels):
    """Further components on a sparse A (implicit projection deflation, FP64
    scores from the columns): per component the objective and the support
    agree with the oracle, which deflates the dense copy explicitly, and
    with the dense GPU component loop."""
    print(f"sparse components fid={fid} panels={panels}", flush=True)
    mat = sparse.bag_of_words(53, 900, 1600, 45000)
    A = mat.dense()
    X0n = workloads.random_unit_starts(54, 16, mat.p)
    par = {1: 8.0, 3: 4.0}.get(fid) or workloads.s_or_gamma_for(fid, A, 8, "scaled")
    flags = spca.FLAG_SPARSE_PANELS if panels else spca.FLAG_SPARSE_NO_PANELS
    got = spca.am_components_sparse(spca.sparse_to_device(mat), fid, par, to_device_rows(X0n),
                                    3, tol=1e-9, maxit=400, flags=flags)
    ref = oracle.am_components(A, fid, par, X0n.astype(np.float64), 3, 1e-9, 400, nthreads=8)
    dense = spca.am_components(to_device_colmajor(A.astype(np.float32)), fid, par,
                               to_device_rows(X0n), 3, tol=1e-9, maxit=400)
    for c in range(3):
        print(c, got[c]["objective"], ref[c]["f"], len(got[c]["support"]), flush=True)
        assert rel_err(got[c]["objective"], ref[c]["f"]) <= 1e-5, (fid, c)
        assert np.array_equal(got[c]["support"], np.flatnonzero(ref[c]["x"])), (fid, c)
        assert rel_err(got[c]["objective"], dense[c]["objective"]) <= 1e-5, (fid, c)
        assert abs(np.linalg.norm(got[c]["x"]) - 1.0) < 1e-12
