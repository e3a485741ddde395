"""Kernel-level parity on the GPU: the MFMA GEMM against an FP64 host
product, and the x-update operators against the FP64 oracle operators on the
same FP32 inputs (Table 3, rows S3-S6)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def spca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1212_4137_amd as m

    m.load()
    return m


def _padded(rows, cols, rng, scale=1.0):
    """Row-major FP32 (rows x cols) on the GPU with a leading dimension that is
    a multiple of 4, plus its FP64 host copy."""
    ld = (cols + 3) // 4 * 4
    h = (rng.standard_normal((rows, cols)) * scale).astype(np.float32)
    buf = torch.zeros((rows, ld), dtype=torch.float32)
    buf[:, :cols] = torch.from_numpy(h)
    return buf.cuda()[:, :cols], h.astype(np.float64)


GEMM_SHAPES = [(1, 1, 1), (3, 130, 37), (32, 128, 32), (33, 129, 33), (64, 257, 1001),
               (100, 1000, 513), (129, 200, 64), (300, 77, 1500), (1024, 300, 96),
               (40, 1500, 300), (7, 5, 4099)]


@pytest.mark.parametrize("M,N,K", GEMM_SHAPES)
def test_gemm_nt_matches_fp64(spca, M, N, K):
    print(f"gemm case M={M} N={N} K={K}", flush=True)
    rng = np.random.default_rng(M * 131 + N * 7 + K)
    P, P64 = _padded(M, K, rng)
    Q, Q64 = _padded(N, K, rng)
    C = spca.gemm_nt(P, Q)
    torch.cuda.synchronize()
    ref = P64 @ Q64.T
    bound = (np.abs(P64) @ np.abs(Q64).T) * (K * 2.0 ** -24) * 1.01 + 1e-30
    err = np.abs(C.cpu().numpy().astype(np.float64) - ref)
    assert np.all(err <= bound), float(np.max(err / bound))


@pytest.mark.parametrize("shape", range(12))
@pytest.mark.parametrize("M,N,K,splits", [(130, 333, 1001, 1), (37, 161, 517, 4),
                                          (256, 100, 4100, 16)])
def test_gemm_every_shape_and_split(spca, shape, M, N, K, splits):
    print(f"gemm shape={shape} M={M} N={N} K={K} splits={splits}", flush=True)
    rng = np.random.default_rng(shape * 17 + M + N + K + splits)
    P, P64 = _padded(M, K, rng)
    Q, Q64 = _padded(N, K, rng)
    parts = spca.gemm_nt_shape(P, Q, shape, splits)
    torch.cuda.synchronize()
    C = parts.cpu().numpy().astype(np.float64).sum(axis=0)
    ref = P64 @ Q64.T
    bound = (np.abs(P64) @ np.abs(Q64).T) * ((K + splits) * 2.0 ** -24) * 1.01 + 1e-30
    assert np.all(np.abs(C - ref) <= bound)


def _oracle_rows(fid, V64, par):
    X, phi, nnz = [], [], []
    for v in V64:
        w, ph = oracle.x_operator(fid, v, par)
        nrm = np.linalg.norm(w)
        X.append(w / nrm if nrm > 0 else w)
        phi.append(ph)
        nnz.append(int(np.count_nonzero(w)))
    return np.array(X), np.array(phi), np.array(nnz)


def _check_xupdate(spca, fid, V_h, par, exact_support=True):
    V = torch.from_numpy(V_h).cuda()
    X, phi, nnz = spca.x_update(fid, V, par)
    torch.cuda.synchronize()
    X = X.cpu().numpy().astype(np.float64)
    phi = phi.cpu().numpy()
    nnz = nnz.cpu().numpy()
    Xr, phir, nnzr = _oracle_rows(fid, V_h.astype(np.float64), par)
    np.testing.assert_allclose(phi, phir, rtol=1e-11, atol=1e-300)
    if exact_support:
        np.testing.assert_array_equal(nnz, nnzr)
        np.testing.assert_array_equal(X != 0, Xr != 0)
    np.testing.assert_allclose(X, Xr, rtol=0, atol=2e-7)
    return X, phi, nnz


# p = 10000 is the row length of the 1000 x 10000 throughput workload (rows
# of 40 floats per thread in the one-workgroup kernel)
@pytest.mark.parametrize("p", [37, 1500, 10000, 20000, 60001, 200000])
@pytest.mark.parametrize("fid", [1, 3, 5, 7])
def test_x_update_random(spca, fid, p):
    print(f"x_update case fid={fid} p={p}", flush=True)
    rng = np.random.default_rng(fid * 1000 + p)
    V_h = (rng.standard_normal((6, p)) * 3).astype(np.float32)
    par = {1: min(10 if p < 50000 else 200, p), 3: 7.3, 5: 4.0, 7: 1.5}[fid]
    if p >= 50000 and fid >= 5:  # keep the penalised supports a few hundred wide
        par = {5: 16.0, 7: 3.0}[fid] * 9 / 4
    _check_xupdate(spca, fid, V_h, par)
    # L1-variance twins share the operator
    _check_xupdate(spca, fid + 1, V_h, par)


def test_x_update_T_s_ties_and_edges(spca):
    p = 300
    V_h = np.zeros((6, p), np.float32)
    V_h[0, [5, 17, 40, 41, 250]] = [2.0, -2.0, 2.0, 1.0, -2.0]  # ties at |2|
    V_h[1, :] = 1.0                                                # all equal
    V_h[2, [3]] = -4.0                                             # fewer nonzeros than s
    # row 3: all zero
    V_h[4, :] = np.arange(p, dtype=np.float32)
    V_h[5, :] = -np.arange(p, dtype=np.float32)[::-1]
    X, phi, nnz = _check_xupdate(spca, 1, V_h, 3)
    assert np.flatnonzero(X[0]).tolist() == [5, 17, 40]     # lowest indices win
    assert np.flatnonzero(X[1]).tolist() == [0, 1, 2]
    assert np.flatnonzero(X[2]).tolist() == [3] and nnz[3] == 0 and phi[3] == 0
    # s = 1 and s = p
    _check_xupdate(spca, 1, V_h, 1)
    _check_xupdate(spca, 2, V_h, p)


@pytest.mark.parametrize("p", [5000, 10000])
def test_x_update_T_s_ties_across_rows(spca, p):
    """p = 5000 and 10000: the one-workgroup kernel holds elements 1024
    apart in one thread, so ties at the s-th key that span several such
    groups, and a cut through an all-equal row, must still keep the lowest
    indices."""
    V_h = np.zeros((4, p), np.float32)
    V_h[0, [4999, 7, 1027, 2100, 1030, 3071, 4096]] = [2.0, -2.0, 2.0, -2.0, 2.0, 2.0, -2.0]
    V_h[0, 500] = 3.0
    V_h[1, :] = 1.0
    rng = np.random.default_rng(11)
    V_h[2] = rng.integers(-3, 4, size=p).astype(np.float32)  # many ties
    V_h[3] = (rng.standard_normal(p) * 3).astype(np.float32)
    X, phi, nnz = _check_xupdate(spca, 1, V_h, 4)
    assert np.flatnonzero(X[0]).tolist() == [7, 500, 1027, 1030]
    X, _, _ = _check_xupdate(spca, 2, V_h, 1500)
    assert np.flatnonzero(X[1]).tolist() == list(range(1500))
    if p == 10000:
        # ties in the last row groups and the ragged tail of the row
        V_h[2] = 0.0
        V_h[2, [9999, 8191, 8192, 9216, 10, 9500]] = [3.0, -3.0, 3.0, 3.0, -3.0, 3.0]
        V_h[2, 9001] = 4.0
        X, _, _ = _check_xupdate(spca, 1, V_h, 5)
        assert np.flatnonzero(X[2]).tolist() == [10, 8191, 8192, 9001, 9216]
        for fid, par in ((3, 30.0), (5, 4.0), (7, 1.5), (6, 9.0), (8, 2.0)):
            _check_xupdate(spca, fid, V_h, par, exact_support=fid != 3)


@pytest.mark.parametrize("p", [12287, 12288])
def test_x_update_widest_register_rows(spca, p):
    """The widest rows the one-workgroup kernel holds in registers (48 per
    thread, twelve row groups, three packed scan words): ties spread over
    every group, a ragged tail, and all four operators."""
    rng = np.random.default_rng(p)
    V_h = (rng.standard_normal((6, p)) * 2).astype(np.float32)
    V_h[0] = 0.0
    V_h[0, np.arange(7, p, 1000)] = 2.0          # 13 ties, one per 1000
    V_h[0, [3, p - 1]] = 5.0
    V_h[1] = rng.integers(-2, 3, size=p).astype(np.float32)
    X, _, _ = _check_xupdate(spca, 1, V_h, 6)
    assert np.flatnonzero(X[0]).tolist() == [3, 7, 1007, 2007, 3007, p - 1]
    _check_xupdate(spca, 2, V_h, 300)
    _check_xupdate(spca, 3, V_h, 40.0, exact_support=False)
    _check_xupdate(spca, 5, V_h, 4.0)
    _check_xupdate(spca, 7, V_h, 1.5)


def test_x_update_gamma_boundaries(spca):
    rng = np.random.default_rng(5)
    V_h = (rng.standard_normal((4, 513)) * 2).astype(np.float32)
    g = float(np.float64(V_h[0, 7]) ** 2)  # v_7^2 == gamma exactly: dropped
    X, _, _ = _check_xupdate(spca, 5, V_h, g)
    assert X[0, 7] == 0
    _check_xupdate(spca, 5, V_h, 0.0)
    big = float(np.max(np.abs(V_h).astype(np.float64)) ** 2)
    X, phi, nnz = _check_xupdate(spca, 6, V_h, big)
    assert np.all(nnz == 0) and np.all(X == 0) and np.all(phi == 0)
    gs = float(abs(np.float64(V_h[1, 9])))
    X, _, _ = _check_xupdate(spca, 7, V_h, gs)
    assert X[1, 9] == 0
    _check_xupdate(spca, 8, V_h, 0.0)
    X, phi, nnz = _check_xupdate(spca, 7, V_h, float(np.max(np.abs(V_h))))
    assert np.all(nnz == 0)


@pytest.mark.parametrize("p", [2049, 20000])
@pytest.mark.parametrize("s", [1.0, 1.7, 12.0, 99.5, 5000.0, 3000.0])
def test_x_update_lambda_s_regimes(spca, s, p):
    # p = 20000: the chunked kernels (candidates, and the interval search
    # when the root lies below the candidates: s = 3000 needs M > 2048)
    rng = np.random.default_rng(int(s * 10) + p)
    V_h = (rng.standard_normal((5, p)) * 10).astype(np.float32)
    V_h[4, 100:] = 0.0
    X, phi, nnz = _check_xupdate(spca, 3, V_h, s, exact_support=False)
    if s >= 5000 and p < 5000:  # inactive constraint: x = v / ||v||
        Vn = V_h.astype(np.float64)
        np.testing.assert_allclose(X, Vn / np.linalg.norm(Vn, axis=1, keepdims=True),
                                   atol=2e-7)
    if s == 1.0:
        assert np.all(nnz == 1)


def test_x_update_chunked_ties_across_chunks(spca):
    # p = 12800 (aligned, beyond the register-resident rows): the chunked
    # kernels, with ties at the s-th key spread over several 4096-wide chunks
    p = 12800
    rng = np.random.default_rng(77)
    V_h = (rng.standard_normal((6, p)) * 0.5).astype(np.float32)
    tie_cols = [5, 4100, 4101, 8200, 12000, 12799]
    V_h[0, tie_cols] = [3.0, -3.0, 3.0, 3.0, -3.0, 3.0]
    V_h[0, [10, 9000]] = [4.0, -5.0]          # two above the tie value
    V_h[1, :] = -2.0                          # every key equal
    V_h[2, :] = 0.0
    V_h[2, [7, 11111]] = [1.0, -1.0]          # fewer nonzeros than s
    V_h[3, :] = 0.0                           # zero row
    V_h[4, :] = np.float32(1e-30)             # tiny but nonzero
    X, phi, nnz = _check_xupdate(spca, 1, V_h, 5)
    assert np.flatnonzero(X[0]).tolist() == [5, 10, 4100, 4101, 9000]
    assert np.flatnonzero(X[1]).tolist() == [0, 1, 2, 3, 4]
    assert np.flatnonzero(X[2]).tolist() == [7, 11111]
    assert nnz[3] == 0 and phi[3] == 0 and np.all(X[3] == 0)
    assert np.flatnonzero(X[4]).tolist() == [0, 1, 2, 3, 4]
    for s in (1, 4096, 4097, p):
        _check_xupdate(spca, 2, V_h, s)


@pytest.mark.parametrize("fid", [1, 2, 5, 6, 7, 8, 3])
def test_solve_long_rows_match_oracle(spca, fid):
    # p = 20000 > 12288: the chunked x-update inside the solve (the L1
    # constraint keeps the one-workgroup kernel)
    import workloads
    from gpu_helpers import compare_solve, gpu_stepper, to_device_colmajor, to_device_rows

    print(f"long-row solve fid={fid}", flush=True)
    sp = workloads.spiked_matrix(41, 150, 20000, thetas=(80.0, 40.0), spike_nnz=30)
    X0 = workloads.random_unit_starts(42, 6, 20000)
    par = workloads.s_or_gamma_for(fid, sp.A, 30, "scaled" if fid in (6, 8) else "literal")
    Ad, X0d = to_device_colmajor(sp.A), to_device_rows(X0)
    got = spca.am_solve(Ad, fid, par, X0d, tol=1e-8, maxit=300, return_X=True)
    ref = oracle.am_multi(sp.A.astype(np.float64), fid, par, X0.astype(np.float64),
                          1e-8, 300, nthreads=6)
    compare_solve(got, ref, f"long rows F{fid}", sp.A, fid, par, X0=X0,
                  stepper=gpu_stepper(spca.am_solve, Ad, fid, par, X0d, tol=1e-8))
