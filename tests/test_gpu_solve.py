"""Parity of the batched GPU solve (spca_am_solve_ex) with the FP64 oracle on
the same seeded inputs and starts, for all 8 formulations of Table 1, plus
edge cases, determinism and closed forms."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import (compare_solve, gpu_stepper, per_start_parity, rel_err, subset,
                         support_near_tie_margin, to_device_colmajor, to_device_rows)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def spca():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1212_4137_amd as m

    m.load()
    return m


def _param(fid, A, s, gamma_mode=None):
    mode = gamma_mode or ("scaled" if fid in (6, 8) else "literal")
    return workloads.s_or_gamma_for(fid, A, s, mode)


# n = 300 (2 tiles + 44), p = 1500 (11 tiles + 92): several tiles and ragged
# tails in both products; r = 40 and 130 exercise the small-M and multi-M
# GEMM paths.  F6 / F8 run with both readings of gamma: the literal
# 0.1 max ||a_i||_2 of the graded workloads (iterates mostly dense: the dense
# A x and the FP64 MFMA evaluation) and the scale-consistent one (sparse).
CASES = [(fid, r, None) for fid in range(1, 9) for r in (40, 130)]
CASES += [(fid, r, "literal") for fid in (6, 8) for r in (40, 130)]


@pytest.mark.parametrize("fid,r,gamma_mode", CASES)
def test_all_formulations_match_oracle(spca, fid, r, gamma_mode):
    print(f"solve case fid={fid} r={r} gamma={gamma_mode}", flush=True)
    sp = workloads.spiked_matrix(workloads.SEED_BASE + 100 + fid, 300, 1500,
                                 thetas=(45.0, 30.0, 20.0), spike_nnz=25)
    A_np = sp.A
    par = _param(fid, A_np, 25, gamma_mode)
    X0 = workloads.random_unit_starts(workloads.SEED_BASE + 200 + fid, r, 1500)
    Ad, X0d = to_device_colmajor(A_np), to_device_rows(X0)
    got = spca.am_solve(Ad, fid, par, X0d, tol=1e-8, maxit=300, return_X=True)
    ref = oracle.am_multi(A_np, fid, par, X0, 1e-8, 300, nthreads=8)
    compare_solve(got, ref, f"F{fid} r={r}", A_np, fid, par, X0=X0,
                  stepper=gpu_stepper(spca.am_solve, Ad, fid, par, X0d, tol=1e-8))
    xb = ref["X"][ref["best"]]
    sup_ref = np.flatnonzero(xb)
    margin = support_near_tie_margin(A_np, xb, fid, par)
    if margin > 1e-5:
        assert np.array_equal(got["support"], sup_ref), (margin, got["support"][:10],
                                                          sup_ref[:10])
        np.testing.assert_allclose(got["x"], xb * np.sign(xb @ got["x"] or 1.0),
                                   atol=3e-5)
    else:
        print(f"near-tie at the best support (margin {margin:.2e}); support not compared")
    np.testing.assert_allclose(got["explained_variance"], ref["ev"][ref["best"]], rtol=2e-5)


def test_small_single_start_workload(spca):
    """Gaussian 100 x 500, L2 variance / L0 constraint, s = 10, start e_i at the
    column of largest norm, tol 1e-8, maxit 500 (stored oracle result)."""
    with open(os.path.join(GOLDEN, "gauss_100x500_F1_s10.json")) as fh:
        g = json.load(fh)
    cfg = workloads.SMALL_SINGLE_START
    A_np = workloads.gaussian_matrix(cfg["seed"], cfg["n"], cfg["p"])
    A = to_device_colmajor(A_np)
    got = spca.am_solve(A, 1, cfg["s"], None, tol=cfg["tol"], maxit=cfg["maxit"])
    assert rel_err(got["objective"], g["f"]) <= 1e-5
    assert got["support"].tolist() == g["support"]
    # Iteration counts are not pinned: tol = 1e-8 is below FP32 resolution, so
    # the FP32 path may meet the ratio test on rounding noise a few steps
    # before the FP64 oracle; it never runs longer.
    assert got["iters"] <= g["iters"] + 2
    assert got["status"] == g["status"]
    # the one-call entry point agrees with the context entry point
    simple = spca.am_solve_simple(A, 1, cfg["s"], None, tol=cfg["tol"], maxit=cfg["maxit"])
    assert simple["objective"] == got["objective"]
    assert np.array_equal(simple["x"], got["x"])


def test_power_method_reduction_s_equals_p(spca):
    rng = np.random.default_rng(3)
    A_np = rng.standard_normal((200, 301)).astype(np.float32)
    sig = np.linalg.svd(A_np.astype(np.float64), compute_uv=False)[0]
    X0 = workloads.random_unit_starts(9, 4, 301)
    A = to_device_colmajor(A_np)
    for fid, par, want in ((1, 301, sig), (3, 301.0, sig), (7, 0.0, sig), (5, 0.0, sig ** 2)):
        got = spca.am_solve(A, fid, par, to_device_rows(X0), tol=1e-12, maxit=3000)
        assert rel_err(got["objective"], want) <= 1e-5, (fid, got["objective"], want)


def test_phi_monotone_per_step(spca):
    sp = workloads.spiked_matrix(17, 200, 900, thetas=(30.0, 20.0), spike_nnz=15)
    X0 = to_device_rows(workloads.random_unit_starts(18, 32, 900))
    A = to_device_colmajor(sp.A)
    for fid in range(1, 9):
        par = _param(fid, sp.A, 15)
        prev = None
        for k in range(1, 9):
            got = spca.am_solve(A, fid, par, X0, tol=-1.0, maxit=k)
            phi = got["phi_per_start"]
            live = got["status_per_start"] == spca.MAXIT
            if prev is not None:
                ok = phi[live] >= prev[live] * (1 - 2e-6) - 1e-12
                assert np.all(ok), (fid, k)
            assert np.all(got["iters_per_start"][live] == k)
            prev = phi


def test_repeat_runs_are_bitwise_identical(spca):
    sp = workloads.spiked_matrix(19, 333, 2001, thetas=(40.0, 20.0), spike_nnz=20)
    A = to_device_colmajor(sp.A)
    X0 = to_device_rows(workloads.random_unit_starts(20, 70, 2001))
    for fid in (1, 4, 6, 7):
        par = _param(fid, sp.A, 20)
        a = spca.am_solve(A, fid, par, X0, tol=1e-7, maxit=100, return_X=True)
        b = spca.am_solve(A, fid, par, X0, tol=1e-7, maxit=100, return_X=True)
        assert np.array_equal(a["f_per_start"], b["f_per_start"])
        assert np.array_equal(a["x"], b["x"])
        assert torch.equal(a["X_final"], b["X_final"])


def test_dense_and_sparse_products_agree(spca):
    sp = workloads.spiked_matrix(21, 256, 1024, thetas=(40.0, 20.0), spike_nnz=10)
    A = to_device_colmajor(sp.A)
    X0 = to_device_rows(workloads.random_unit_starts(22, 64, 1024))
    for fid in (1, 2, 5):
        par = _param(fid, sp.A, 10)
        a = spca.am_solve(A, fid, par, X0, tol=1e-9, maxit=200)
        b = spca.am_solve(A, fid, par, X0, tol=1e-9, maxit=200, flags=spca.FLAG_DENSE_ONLY)
        assert rel_err(a["objective"], b["objective"]) <= 1e-5
        assert np.array_equal(a["support"], b["support"])


def test_unaligned_leading_dimension_and_odd_sizes(spca):
    rng = np.random.default_rng(23)
    A_np = rng.standard_normal((37, 53)).astype(np.float32)
    X0 = workloads.random_unit_starts(24, 3, 53)
    for lda in (37, 41):
        A = to_device_colmajor(A_np, lda=lda)
        for fid in (1, 4, 5, 8):
            par = {1: 5, 4: 5.0, 5: 2.0, 8: 3.0}[fid]
            got = spca.am_solve(A, fid, par, to_device_rows(X0), tol=1e-10, maxit=500,
                                return_X=True)
            ref = oracle.am_multi(A_np, fid, par, X0, 1e-10, 500)
            compare_solve(got, ref, f"odd lda={lda} F{fid}", A_np, fid, par, X0=X0,
                          stepper=gpu_stepper(spca.am_solve, A, fid, par, to_device_rows(X0),
                                              tol=1e-10))


def test_degenerate_and_zero_starts(spca):
    A_np = np.zeros((40, 60), np.float32)
    A_np[:, :10] = np.random.default_rng(25).standard_normal((40, 10))
    X0 = np.zeros((3, 60), np.float32)
    X0[0, 30] = 1.0                       # A x0 = 0: DEGENERATE
    X0[1, 2] = 1.0
    X0[2, :] = 1.0
    A = to_device_colmajor(A_np)
    got = spca.am_solve(A, 1, 3, to_device_rows(X0), tol=1e-9, maxit=50)
    assert got["status_per_start"][0] == spca.DEGENERATE
    assert got["f_per_start"][0] == 0.0 and got["iters_per_start"][0] == 0
    ref = oracle.am_multi(A_np, 1, 3, X0, 1e-9, 50)
    assert rel_err(got["objective"], ref["f"][ref["best"]]) <= 1e-5
    assert got["warning"] == spca.WARN_NONE  # the others converged
    # the same with one x-update: no start can meet the stop test
    got = spca.am_solve(A, 1, 3, to_device_rows(X0), tol=1e-9, maxit=1)
    assert got["warning"] == spca.WARN_NO_CONVERGED
    got = spca.am_solve(A, 1, 3, to_device_rows(X0), tol=-1.0, maxit=1)
    assert got["warning"] == spca.WARN_NONE  # stop test off: no warning
    # gamma above the zero-solution threshold: every start ends ZERO (one
    # DEGENERATE start among them)
    thr = float(np.max(np.linalg.norm(A_np.astype(np.float64), axis=0)))
    got = spca.am_solve(A, 7, thr * 1.01, to_device_rows(X0[1:]), tol=1e-9, maxit=50)
    assert np.all(got["status_per_start"] == spca.ZERO)
    assert got["objective"] == 0.0 and got["nnz"] == 0 and not np.any(got["x"])
    assert got["warning"] == spca.WARN_ALL_ZERO
    got = spca.am_solve(A, 7, thr * 1.01, to_device_rows(X0), tol=1e-9, maxit=50)
    assert got["warning"] == spca.WARN_ALL_ZERO
    # an all-zero matrix: every start DEGENERATE
    got = spca.am_solve(to_device_colmajor(np.zeros((8, 9), np.float32)), 2, 2,
                        to_device_rows(np.ones((2, 9), np.float32)), tol=1e-9, maxit=5)
    assert np.all(got["status_per_start"] == spca.DEGENERATE)
    assert got["warning"] == spca.WARN_ALL_DEGENERATE


def test_check_finite_flag_rejects_nan(spca):
    A_np = np.ones((16, 20), np.float32)
    A_np[3, 4] = np.nan
    with pytest.raises(spca.SpcaError) as e:
        spca.am_solve(to_device_colmajor(A_np), 1, 2, None, flags=spca.FLAG_CHECK_FINITE)
    assert e.value.code == -1


def test_budget_is_enforced(spca):
    ctx = spca.Context(0, hbm_budget_bytes=1 << 20)
    A = to_device_colmajor(np.ones((500, 800), np.float32))
    X0 = to_device_rows(np.ones((64, 800), np.float32))
    with pytest.raises(spca.SpcaError) as e:
        spca.am_solve(A, 1, 5, X0, ctx=ctx)
    assert e.value.code == -2
    ctx.close()


@pytest.mark.parametrize("fid", [1, 2, 3, 4])
def test_row_block_list_product(spca, fid):
    # few starts on tall columns, union product off: the planner picks the
    # row-block list kernel (many workgroups per start); results keep parity
    # with the oracle and agree with the dense product
    sp = workloads.spiked_matrix(71, 8200, 1500, thetas=(200.0, 120.0), spike_nnz=20)
    X0n = workloads.random_unit_starts(72, 12, 1500)
    A, X0 = to_device_colmajor(sp.A), to_device_rows(X0n)
    par = _param(fid, sp.A, 20)
    got = spca.am_solve(A, fid, par, X0, tol=1e-8, maxit=200, kernel_times=True,
                        flags=spca.FLAG_NO_UNION, return_X=True)
    assert got["kernel_times"]["iters_list_rows"] > 0, got["kernel_times"]
    assert got["kernel_times"]["iters_union"] == 0
    ref = oracle.am_multi(sp.A.astype(np.float64), fid, par, X0n.astype(np.float64),
                          1e-8, 200, nthreads=6)
    compare_solve(got, ref, f"row-block list F{fid}", sp.A, fid, par, X0=X0n,
                  stepper=gpu_stepper(spca.am_solve, A, fid, par, X0, tol=1e-8,
                                      flags=spca.FLAG_NO_UNION))
    dense = spca.am_solve(A, fid, par, X0, tol=1e-8, maxit=200, flags=spca.FLAG_DENSE_ONLY)
    assert rel_err(got["objective"], dense["objective"]) <= 1e-5


def test_row_block_list_product_many_starts(spca):
    """More starts than the row-block kernel's capped grid height (256), so
    each workgroup row serves several starts: per-start results agree with
    the dense product on the same starts."""
    sp = workloads.spiked_matrix(73, 8200, 1500, thetas=(200.0, 120.0), spike_nnz=20)
    X0n = workloads.random_unit_starts(74, 300, 1500)
    A, X0 = to_device_colmajor(sp.A), to_device_rows(X0n)
    got = spca.am_solve(A, 1, 20.0, X0, tol=1e-8, maxit=100, kernel_times=True,
                        flags=spca.FLAG_NO_UNION)
    assert got["kernel_times"]["iters_list_rows"] > 0, got["kernel_times"]
    dense = spca.am_solve(A, 1, 20.0, X0, tol=1e-8, maxit=100, flags=spca.FLAG_DENSE_ONLY)
    assert rel_err(got["objective"], dense["objective"]) <= 1e-5
    ok = [rel_err(a, b) <= 1e-5 for a, b in zip(got["f_per_start"], dense["f_per_start"])]
    assert np.mean(ok) >= 0.98


@pytest.mark.parametrize("fid", [1, 6])
def test_k_split_aty_product(spca, fid):
    """Few starts and a long p: the planner splits the K = n loop of
    V = A^T Y and the partials are summed before the x-update.  Parity with
    the oracle, and with the same solve forced to one split through the
    tuning table."""
    n, p, r = 2000, 8000, 16
    print(f"k-split A^T Y case fid={fid}", flush=True)
    assert spca.gemm_plan(r, p, n, 16)[1] > 1
    sp = workloads.spiked_matrix(workloads.SEED_BASE + 120 + fid, n, p,
                                 thetas=(80.0, 60.0, 40.0), spike_nnz=40)
    A_np = sp.A
    par = _param(fid, A_np, 40)
    X0 = workloads.random_unit_starts(workloads.SEED_BASE + 220 + fid, r, p)
    A = to_device_colmajor(A_np)
    got = spca.am_solve(A, fid, par, to_device_rows(X0), tol=1e-8, maxit=120,
                        return_X=True)
    ref = oracle.am_multi(A_np, fid, par, X0, 1e-8, 120, nthreads=8)
    compare_solve(got, ref, f"k-split F{fid}", A_np, fid, par, X0=X0,
                  stepper=gpu_stepper(spca.am_solve, A, fid, par, to_device_rows(X0),
                                      tol=1e-8))
    shape = spca.gemm_plan(r, p, n, 16)[0]
    # bucket(x) = round(2 log2 x): 16 -> 8, 8000 -> 26, 2000 -> 22
    spca.tune_table_import(f"4 16 8 26 22 {shape} 1\n")
    try:
        assert spca.gemm_plan(r, p, n, 16) == (shape, 1)
        one = spca.am_solve(A, fid, par, to_device_rows(X0), tol=1e-8, maxit=120)
    finally:
        spca.tune_table_clear()
    assert rel_err(got["objective"], one["objective"]) <= 1e-5


def test_union_product_used_and_agrees(spca):
    """512 starts made of four distinct ones, so that their supports
    overlap almost entirely: the planner moves A x to the union-of-supports
    product (which the host keeps launching while it is picked); per-start
    results agree with the dense product, and the graph replays the same
    adaptive launch sequence bit for bit."""
    sp = workloads.spiked_matrix(75, 2000, 4000, thetas=(300.0,), spike_nnz=20)
    X0n = np.ascontiguousarray(np.repeat(workloads.random_unit_starts(76, 4, 4000), 128, axis=0))
    A, X0 = to_device_colmajor(sp.A), to_device_rows(X0n)
    kw = dict(tol=-1.0, maxit=64, return_X=True)
    got = spca.am_solve(A, 1, 20.0, X0, kernel_times=True, **kw)
    assert got["kernel_times"]["iters_union"] > 0, got["kernel_times"]
    # the oracle from the four distinct starts, per start and best of all
    ref4 = oracle.am_multi(sp.A, 1, 20.0, X0n[::128], -1.0, 64, nthreads=4)
    ref = {k: np.repeat(ref4[k], 128, axis=0) for k in ("f", "status", "iters")}
    ref["best"] = ref4["best"] * 128
    compare_solve(got, ref, "union product", sp.A, 1, 20.0, X0=X0n,
                  stepper=gpu_stepper(spca.am_solve, A, 1, 20.0, X0, tol=-1.0))
    dense = spca.am_solve(A, 1, 20.0, X0, flags=spca.FLAG_DENSE_ONLY, **kw)
    ok = [rel_err(a, b) <= 1e-5 for a, b in zip(got["f_per_start"], dense["f_per_start"])]
    assert np.mean(ok) >= 0.98
    g = spca.am_solve(A, 1, 20.0, X0, flags=spca.FLAG_GRAPH, **kw)
    assert np.array_equal(g["f_per_start"], got["f_per_start"])
    assert torch.equal(g["X_final"], got["X_final"])


def test_union_product_returns_when_supports_converge(spca):
    """Random starts on a moderate spike: their supports differ at first
    (the list product serves, and the host stops launching the union
    product) and converge later, when the probes bring the union product
    back.  Per-start results agree with the dense product, and the graph
    replays the same launch decisions bit for bit."""
    sp = workloads.spiked_matrix(75, 2000, 4000, thetas=(600.0,), spike_nnz=20)
    X0n = workloads.random_unit_starts(77, 512, 4000)
    A, X0 = to_device_colmajor(sp.A), to_device_rows(X0n)
    kw = dict(tol=-1.0, maxit=96, return_X=True)
    got = spca.am_solve(A, 1, 20.0, X0, kernel_times=True, **kw)
    kt = got["kernel_times"]
    assert kt["iters_list"] > 8 and kt["iters_union"] > 0, kt
    # a sample of the starts against the oracle from the same starts
    idx = np.r_[0:24, 100:512:64]
    ref = oracle.am_multi(sp.A, 1, 20.0, X0n[idx], -1.0, 96, nthreads=8)
    per_start_parity(subset(got, idx), ref, "union product (sample)", sp.A, 1, 20.0,
                     X0=X0n[idx], stepper=gpu_stepper(spca.am_solve, A, 1, 20.0, X0,
                                                      tol=-1.0, rows=idx))
    dense = spca.am_solve(A, 1, 20.0, X0, flags=spca.FLAG_DENSE_ONLY, **kw)
    ok = [rel_err(a, b) <= 1e-5 for a, b in zip(got["f_per_start"], dense["f_per_start"])]
    assert np.mean(ok) >= 0.98
    g = spca.am_solve(A, 1, 20.0, X0, flags=spca.FLAG_GRAPH, **kw)
    assert np.array_equal(g["f_per_start"], got["f_per_start"])
    assert torch.equal(g["X_final"], got["X_final"])


def test_work_counters_and_sampled_events(spca):
    """The device's work counters (running starts and iterate nonzeros per
    iteration, the algorithmic work of the two products) and the sampled
    event timing: fixed work gives r maxit running-start iterations and,
    for T_s, nonzeros r p (the dense starts) plus r s per later iteration;
    with the stop test the running starts sum to the iterations done."""
    sp = workloads.spiked_matrix(81, 200, 900, thetas=(40.0, 20.0), spike_nnz=10)
    A = to_device_colmajor(sp.A)
    X0 = to_device_rows(workloads.random_unit_starts(82, 40, 900))
    got = spca.am_solve(A, 1, 12.0, X0, tol=-1.0, maxit=20, kernel_times=True)
    kt = got["kernel_times"]
    assert kt["active_starts_sum"] == 40 * 20
    assert kt["ax_nnz_sum"] == 40 * 900 + 40 * 19 * 12
    assert kt["aty_launches"] == 20
    got = spca.am_solve(A, 1, 12.0, X0, tol=-1.0, maxit=20, kernel_times=True,
                        flags=spca.FLAG_TIME_SAMPLED)
    kt = got["kernel_times"]
    assert kt["aty_launches"] == 3 and kt["x_update_launches"] == 3  # iterations 0, 8, 16
    assert kt["active_starts_sum"] == 40 * 20
    got = spca.am_solve(A, 3, 8.0, X0, tol=1e-6, maxit=300, kernel_times=True)
    assert got["kernel_times"]["active_starts_sum"] == got["iters_per_start"].sum()
    assert got["kernel_times"]["ax_nnz_sum"] >= 40 * 900


def test_concurrent_solves_on_several_streams_are_identical(spca):
    """Independent solves on 4 streams at once (a context and a host thread
    each, as bench.py --streams runs them) give the same bits as one after
    another on one stream."""
    import threading

    sp = workloads.spiked_matrix(workloads.SEED_BASE + 77, 300, 3000, thetas=(40.0, 20.0),
                                 spike_nnz=20)
    A = to_device_colmajor(sp.A)
    X0 = to_device_rows(workloads.random_unit_starts(workloads.SEED_BASE + 78, 96, 3000))
    fids = list(range(1, 9))
    par = {f: _param(f, sp.A, 20, "literal") for f in fids}
    seq = {f: spca.am_solve(A, f, par[f], X0, tol=-1.0, maxit=60, return_X=True) for f in fids}
    ctxs = [spca.Context(0) for _ in range(4)]
    streams = [torch.cuda.Stream() for _ in range(4)]
    conc = {}

    def lane(w):
        for f in fids[w::4]:
            conc[f] = spca.am_solve(A, f, par[f], X0, tol=-1.0, maxit=60, ctx=ctxs[w],
                                    stream=streams[w], return_X=True)
    threads = [threading.Thread(target=lane, args=(w,)) for w in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    for f in fids:
        assert np.array_equal(seq[f]["f_per_start"], conc[f]["f_per_start"]), f
        assert torch.equal(seq[f]["X_final"], conc[f]["X_final"]), f
        assert np.array_equal(seq[f]["x"], conc[f]["x"]), f
