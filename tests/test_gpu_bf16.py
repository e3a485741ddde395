"""BF16-storage path (A, X, Y operands in BF16, FP32 accumulation) with FP32
polish on the final support and FP64 objective: kernel parity of the BF16
product and solve parity against the FP64 oracle at the tolerances of the
precision study: the BF16-phase best within 1e-3 of the oracle's best, and
after the FP32 polish an FP64 stationary point no worse than the oracle's
best by more than 1e-5 (a better stationary point is allowed), except at a
documented near-tie of the oracle's own top stationary points."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import fixed_point_certificate, rel_err, to_device_colmajor, to_device_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def spca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1212_4137_amd as m

    m.load()
    return m


def _bf16_round(x):
    """FP32 -> nearest-even BF16 value, returned as float64 (host reference)."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (37, 161, 517), (130, 333, 1001),
                                   (256, 100, 4100), (1024, 300, 64)])
def test_gemm_bf16_matches_fp64(spca, M, N, K):
    print(f"bf16 gemm M={M} N={N} K={K}", flush=True)
    rng = np.random.default_rng(M + 3 * N + 7 * K)
    ldk = (K + 7) // 8 * 8
    P = torch.zeros((M, ldk), dtype=torch.bfloat16)
    Q = torch.zeros((N, ldk), dtype=torch.bfloat16)
    P[:, :K] = torch.from_numpy(rng.standard_normal((M, K)).astype(np.float32)).to(torch.bfloat16)
    Q[:, :K] = torch.from_numpy(rng.standard_normal((N, K)).astype(np.float32)).to(torch.bfloat16)
    P64 = P[:, :K].float().numpy().astype(np.float64)
    Q64 = Q[:, :K].float().numpy().astype(np.float64)
    C = spca.gemm_nt_bf16(P.cuda()[:, :K], Q.cuda()[:, :K])
    torch.cuda.synchronize()
    ref = P64 @ Q64.T
    bound = (np.abs(P64) @ np.abs(Q64).T) * (K * 2.0 ** -24) * 1.01 + 1e-30
    assert np.all(np.abs(C.cpu().numpy().astype(np.float64) - ref) <= bound)


@pytest.mark.parametrize("shape", range(12))
@pytest.mark.parametrize("M,N,K,splits", [(130, 333, 1001, 1), (300, 290, 4100, 4)])
def test_gemm_bf16_every_shape_and_split(spca, shape, M, N, K, splits):
    print(f"bf16 gemm shape={shape} M={M} N={N} K={K} splits={splits}", flush=True)
    rng = np.random.default_rng(shape * 13 + M + 3 * N + 7 * K + splits)
    ldk = (K + 7) // 8 * 8
    P = torch.zeros((M, ldk), dtype=torch.bfloat16)
    Q = torch.zeros((N, ldk), dtype=torch.bfloat16)
    P[:, :K] = torch.from_numpy(rng.standard_normal((M, K)).astype(np.float32)).to(torch.bfloat16)
    Q[:, :K] = torch.from_numpy(rng.standard_normal((N, K)).astype(np.float32)).to(torch.bfloat16)
    P64 = P[:, :K].float().numpy().astype(np.float64)
    Q64 = Q[:, :K].float().numpy().astype(np.float64)
    parts = spca.gemm_nt_shape(P.cuda()[:, :K], Q.cuda()[:, :K], shape, splits)
    torch.cuda.synchronize()
    C = parts.cpu().numpy().astype(np.float64).sum(axis=0)
    ref = P64 @ Q64.T
    bound = (np.abs(P64) @ np.abs(Q64).T) * ((K + splits) * 2.0 ** -24) * 1.01 + 1e-30
    assert np.all(np.abs(C - ref) <= bound)


def test_host_bf16_rounding_matches_torch():
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy().astype(np.float64)
    assert np.array_equal(_bf16_round(x), ref)


def _param(fid, A, s):
    return workloads.s_or_gamma_for(fid, A, s, "scaled" if fid in (6, 8) else "literal")


@pytest.mark.parametrize("fid", range(1, 9))
def test_bf16_polish_solve_matches_oracle(spca, fid):
    print(f"bf16 solve fid={fid}", flush=True)
    sp = workloads.spiked_matrix(workloads.SEED_BASE + 300 + fid, 400, 2000,
                                 thetas=(60.0, 40.0, 25.0), spike_nnz=30)
    A_np = sp.A
    par = _param(fid, A_np, 30)
    X0 = workloads.random_unit_starts(workloads.SEED_BASE + 400 + fid, 64, 2000)
    got = spca.am_solve(to_device_colmajor(A_np), fid, par, to_device_rows(X0), tol=1e-8,
                        maxit=200, precision=spca.PREC_BF16_POLISH, polish_maxit=200)
    ref = oracle.am_multi(A_np, fid, par, X0, 1e-8, 200, nthreads=8, want_x=False)
    f_ref = ref["f"][ref["best"]]
    scale = abs(f_ref)
    # signed: positive when the GPU result is above the oracle's best
    pre = (got["objective_pre_polish"] - f_ref) / scale
    post = (got["objective"] - f_ref) / scale
    srt = np.sort(ref["f"])[::-1]
    gap = (srt[0] - srt[1]) / abs(srt[0]) if len(srt) > 1 else 1.0
    print(f"F{fid}: pre-polish rel gap {pre:+.2e}, post-polish {post:+.2e}, "
          f"polish iters {got['polish_iters']}, oracle top-2 gap {gap:.2e}", flush=True)
    # before the polish: within BF16 resolution of the oracle's best
    assert abs(pre) <= 1e-3
    # the result is an FP64 stationary point of Algorithm 2
    cert = fixed_point_certificate(A_np, fid, par, got["x"], got["objective"])
    assert cert["ok"], cert
    # after the polish: no worse than the oracle's best by more than 1e-5,
    # except at a documented near-tie of the oracle's own stationary points
    # (top-2 gap below the BF16 resolution 1e-3, where BF16 rounding can
    # steer every start to the second one): then at least the oracle's
    # second best
    if post < -1e-5:
        assert gap < 1e-3, (post, gap)
        assert got["objective"] >= srt[1] * (1 - 1e-9), (got["objective"], srt[:3])
        print(f"F{fid}: near-tie of the oracle's top stationary points (gap {gap:.2e}); "
              f"the result lies between its best and second best", flush=True)
    # the returned vector is unit norm and its objective is the reported one
    x = got["x"]
    assert abs(np.linalg.norm(x) - 1.0) < 1e-12 or not x.any()
    f_chk, _ = oracle.objective(fid, A_np, x, par)
    assert rel_err(got["objective"], f_chk) <= 1e-9
