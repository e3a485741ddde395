"""Pins for the oracle's Algorithm 2 and multi-start driver.

Checks against what the paper and the mathematics fix, never against the
oracle itself: the reduction to classical / robust PCA at s = p or gamma = 0
(Section 1.1, with a dense SVD or exhaustive sign enumeration as reference),
brute force over supports or sign vectors on tiny inputs (OPT = max over y of
F_X(y), proof of Theorem 1), the monotone interleaving of phi and f (Section
1.2 and Theorem 1), closed forms at s = 1, for rank-one A and for gamma above
the zero-solution threshold, and metamorphic invariances.
"""
import itertools

import numpy as np
import pytest

import oracle

L2_FIDS = (1, 3, 5, 7)
L1_FIDS = (2, 4, 6, 8)


def _starts(r, p, seed):
    X = np.random.default_rng(seed).standard_normal((r, p))
    return X / np.linalg.norm(X, axis=1, keepdims=True)


def _sigma_max(A):
    return float(np.linalg.svd(A, compute_uv=False)[0])


# -- reduction to classical PCA (s = p, gamma = 0) ---------------------------

@pytest.mark.parametrize("fid,par,power", [(1, None, 1), (3, None, 1), (7, 0.0, 1),
                                           (5, 0.0, 2)])
def test_power_method_reduction(fid, par, power):
    r = np.random.default_rng(7)
    A = r.standard_normal((40, 25))
    p = A.shape[1]
    par = float(p) if par is None else par
    res = oracle.am_multi(A, fid, par, _starts(4, p, 1), tol=1e-15, maxit=5000)
    assert res["f"][res["best"]] == pytest.approx(_sigma_max(A) ** power, rel=1e-10)
    assert res["ev"][res["best"]] == pytest.approx(_sigma_max(A) ** 2, rel=1e-10)


def _robust_pca_opt(A):
    """max_{||x||_2<=1} ||Ax||_1 = max over y in {-1,1}^n of ||A^T y||_2."""
    n = A.shape[0]
    return max(np.linalg.norm(A.T @ np.array(y)) for y in itertools.product((-1, 1), repeat=n))


@pytest.mark.parametrize("fid", L1_FIDS)
def test_robust_pca_reduction(fid):
    r = np.random.default_rng(11)
    A = r.standard_normal((9, 6))
    p = A.shape[1]
    par = float(p) if fid <= 4 else 0.0
    res = oracle.am_multi(A, fid, par, _starts(64, p, 2), tol=1e-14, maxit=2000)
    opt = _robust_pca_opt(A)
    best = res["f"][res["best"]]
    want = opt ** 2 if fid == 6 else opt
    assert best <= want * (1 + 1e-12)
    assert best == pytest.approx(want, rel=1e-9)
    # the explained variance of L1 variance is ||Ax||_1 itself (not squared):
    # at s = p / gamma = 0 it is the robust-PCA optimum for every formulation
    assert res["ev"][res["best"]] == pytest.approx(opt, rel=1e-9)


# -- brute force on tiny inputs -------------------------------------------------

def _opt_F1(A, s):
    p = A.shape[1]
    return max(_sigma_max(A[:, list(S)]) for S in itertools.combinations(range(p), s))


def _opt_F5(A, gamma):
    p = A.shape[1]
    best = 0.0
    for k in range(1, p + 1):
        for S in itertools.combinations(range(p), k):
            best = max(best, _sigma_max(A[:, list(S)]) ** 2 - gamma * k)
    return best


def _phi_l1_var(fid, v, par):
    """F_X(y) at v = A^T y for the L1-variance formulations, from the
    definitions of the x-subproblems, written with numpy."""
    if fid == 2:
        return np.sqrt(np.sum(np.sort(v ** 2)[::-1][: int(par)]))
    if fid == 6:
        return np.sum(np.maximum(v ** 2 - par, 0))
    if fid == 8:
        return np.linalg.norm(np.maximum(np.abs(v) - par, 0))
    if fid == 4:  # dual of S4: min over lambda >= 0 (fine grid plus refinement)
        from scipy import optimize
        g = lambda t: t * np.sqrt(par) + np.linalg.norm(np.maximum(np.abs(v) - t, 0))
        top = np.max(np.abs(v))
        grid = np.linspace(0, top, 2001)
        t0 = grid[np.argmin([g(t) for t in grid])]
        lo, hi = max(0, t0 - top / 2000), min(top, t0 + top / 2000)
        res = optimize.minimize_scalar(g, bounds=(lo, hi), method="bounded",
                                       options={"xatol": 1e-14})
        return min(res.fun, g(t0))
    raise ValueError(fid)


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_F1(seed):
    r = np.random.default_rng(20 + seed)
    A = r.standard_normal((8, 12))
    s = 3
    opt = _opt_F1(A, s)
    res = oracle.am_multi(A, 1, s, _starts(200, 12, seed), tol=1e-12, maxit=500)
    assert np.all(res["f"] <= opt * (1 + 1e-12))
    assert res["f"][res["best"]] == pytest.approx(opt, rel=1e-9)


@pytest.mark.parametrize("seed", range(3))
def test_brute_force_F5(seed):
    r = np.random.default_rng(30 + seed)
    A = r.standard_normal((8, 10))
    gamma = 1.5
    opt = _opt_F5(A, gamma)
    res = oracle.am_multi(A, 5, gamma, _starts(200, 10, seed), tol=1e-12, maxit=500)
    assert np.all(res["f"] <= opt + 1e-9 * abs(opt))
    assert res["f"][res["best"]] == pytest.approx(opt, rel=1e-9)


@pytest.mark.parametrize("fid", L1_FIDS)
def test_brute_force_L1_variance(fid):
    r = np.random.default_rng(40 + fid)
    A = r.standard_normal((9, 8))
    par = 3.0 if fid <= 4 else (2.0 if fid == 6 else 0.6)
    opt = max(_phi_l1_var(fid, A.T @ np.array(y), par)
              for y in itertools.product((-1, 1), repeat=A.shape[0]))
    res = oracle.am_multi(A, fid, par, _starts(300, 8, fid), tol=1e-12, maxit=500)
    # F_X(y) equals the objective at the optimal x for that y
    assert np.all(res["f"] <= opt * (1 + 1e-9))
    assert res["f"][res["best"]] == pytest.approx(opt, rel=1e-7)
    # explained variance at the optimum, from the maximising sign vector y*
    # alone: there y* = sgn(A x*), so ||A x*||_1 = y*^T A x* = v*^T x* with
    # v* = A^T y* and x* the normalised image of v* under the x-operator
    ys = [np.array(y) for y in itertools.product((-1, 1), repeat=A.shape[0])]
    vals = [_phi_l1_var(fid, A.T @ y, par) for y in ys]
    v = A.T @ ys[int(np.argmax(vals))]
    w, _ = oracle.x_operator(fid, v, par)
    x_star = w / np.linalg.norm(w)
    assert res["ev"][res["best"]] == pytest.approx(float(v @ x_star), rel=1e-6)


@pytest.mark.parametrize("fid", (1, 3, 5, 7))
def test_brute_force_angular_sweep_n2(fid):
    """n = 2: OPT = max over y on the unit circle of F_X(y); a fine sweep
    brackets it within the Lipschitz bound of F_X."""
    r = np.random.default_rng(50 + fid)
    A = r.standard_normal((2, 7))
    par = {1: 2, 3: 2.0, 5: 0.8, 7: 0.4}[fid]
    th = np.linspace(0, 2 * np.pi, 200001)
    Y = np.stack([np.cos(th), np.sin(th)])
    V = A.T @ Y  # p x m
    if fid == 1:
        vals = np.sqrt(np.sum(np.sort(V ** 2, axis=0)[::-1][:par], axis=0))
    elif fid == 5:
        vals = np.sum(np.maximum(V ** 2 - par, 0), axis=0)
    elif fid == 7:
        vals = np.linalg.norm(np.maximum(np.abs(V) - par, 0), axis=0)
    else:
        vals = np.array([_phi_l1_var(4, V[:, k], par) for k in range(0, V.shape[1], 400)])
        th = th[::400]
    opt_lo = vals.max()
    L = _sigma_max(A) * (2 * _sigma_max(A) if fid == 5 else 1)
    opt_hi = opt_lo + L * (th[1] - th[0])
    res = oracle.am_multi(A, fid, par, _starts(100, 7, fid), tol=1e-13, maxit=1000)
    best = res["f"][res["best"]]
    assert best <= opt_hi * (1 + 1e-12)
    assert best >= opt_lo * (1 - 1e-9)


# -- monotone interleaving: phi_{k-1} <= f(x^k) <= phi_k ----------------------

@pytest.mark.parametrize("fid", range(1, 9))
def test_interleaving(fid):
    r = np.random.default_rng(60 + fid)
    A = r.standard_normal((15, 40))
    par = 5 if fid <= 4 else {5: 4.0, 6: 20.0, 7: 0.5, 8: 2.0}[fid]
    x0 = _starts(1, 40, fid)[0]
    K = 12
    full = oracle.am_single(A, fid, par, x0, tol=-1.0, maxit=K)
    phi = full["phi_trace"]
    assert full["iters"] == K and full["status"] == oracle.MAXIT
    for k in range(1, K):
        xk = oracle.am_single(A, fid, par, x0, tol=-1.0, maxit=k)["x"]
        fk, _ = oracle.objective(fid, A, xk, par)
        eps = 1e-12 * abs(phi[k])
        assert phi[k - 1] - eps <= fk <= phi[k] + eps, (k, phi[k - 1], fk, phi[k])


# -- closed forms ---------------------------------------------------------------

def test_s1_from_max_norm_column_is_global_optimum():
    r = np.random.default_rng(70)
    A = r.standard_normal((20, 60))
    x0 = oracle.unit_vector_start(A)
    out = oracle.am_single(A, 1, 1, x0, tol=1e-12, maxit=50)
    assert out["f"] == pytest.approx(np.max(np.linalg.norm(A, axis=0)), rel=1e-14)
    assert out["iters"] == 2 and out["status"] == oracle.CONVERGED
    # F3 with s = 1 has the same optimum (the L1 ball of radius 1 has vertices +-e_i)
    res = oracle.am_multi(A, 3, 1.0, _starts(64, 60, 3), tol=1e-12, maxit=500)
    assert res["f"].max() <= np.max(np.linalg.norm(A, axis=0)) * (1 + 1e-12)
    # L1 variance, s = 1: OPT = max_i ||a_i||_1
    for fid in (2, 4):
        res = oracle.am_multi(A, fid, 1.0, _starts(64, 60, 4), tol=1e-12, maxit=500)
        assert res["f"].max() == pytest.approx(np.max(np.abs(A).sum(axis=0)), rel=1e-12)


@pytest.mark.parametrize("fid", range(1, 9))
def test_rank_one_closed_form(fid):
    r = np.random.default_rng(80 + fid)
    n, p = 30, 50
    u = r.standard_normal(n)
    u /= np.linalg.norm(u)
    v = r.standard_normal(p)
    v /= np.linalg.norm(v)
    sigma = 3.0
    A = sigma * np.outer(u, v)
    c = sigma if fid % 2 else sigma * np.sum(np.abs(u))  # ||A x|| = c |v^T x|
    av = np.abs(c * v)
    if fid in (1, 2):
        s = 7
        want = np.sqrt(np.sum(np.sort(av ** 2)[::-1][:s]))
        par = s
    elif fid in (3, 4):
        par = 7.0
        from scipy import optimize
        g = lambda t: t * np.sqrt(par) + np.linalg.norm(np.maximum(av - t, 0))
        want = optimize.minimize_scalar(g, bounds=(0, av.max()), method="bounded",
                                        options={"xatol": 1e-14}).fun
    elif fid in (5, 6):
        par = 0.02 * c * c
        want = np.sum(np.maximum(av ** 2 - par, 0))
    else:
        par = 0.1 * c
        want = np.linalg.norm(np.maximum(av - par, 0))
    res = oracle.am_multi(A, fid, par, _starts(3, p, fid), tol=1e-14, maxit=100)
    assert res["f"][res["best"]] == pytest.approx(want, rel=1e-9)
    assert np.all(res["iters"] <= 3)


@pytest.mark.parametrize("fid", (5, 6, 7, 8))
def test_gamma_above_zero_threshold_gives_zero(fid):
    r = np.random.default_rng(90 + fid)
    A = r.standard_normal((12, 30))
    c2 = np.max(np.linalg.norm(A, axis=0))
    c1 = np.max(np.abs(A).sum(axis=0))
    thr = {5: c2 ** 2, 6: c1 ** 2, 7: c2, 8: c1}[fid]
    res = oracle.am_multi(A, fid, thr * 1.0001, _starts(8, 30, fid), tol=1e-8, maxit=50)
    assert np.all(res["status"] == oracle.ZERO)
    assert np.all(res["f"] == 0.0) and np.all(res["X"] == 0.0)
    # just below the threshold, the start e_i on the column attaining it gives
    # v_i = ||a_i||_2 (L2 variance) or ||a_i||_1 (L1 variance) and survives
    col = np.argmax(np.linalg.norm(A, axis=0) if fid % 2 else np.abs(A).sum(axis=0))
    x0 = np.zeros(30)
    x0[col] = 1.0
    out = oracle.am_single(A, fid, thr * 0.999, x0, tol=1e-8, maxit=50)
    assert out["f"] > 0 and out["status"] != oracle.ZERO


def test_degenerate_start():
    A = np.zeros((5, 8))
    A[:, :4] = np.random.default_rng(0).standard_normal((5, 4))
    x0 = np.zeros(8)
    x0[6] = 1.0  # A x0 = 0 (Theorem 1 assumes ||A x0|| != 0)
    for fid in range(1, 9):
        out = oracle.am_single(A, fid, 2 if fid <= 4 else 0.1, x0, 1e-8, 10)
        assert out["status"] == oracle.DEGENERATE and out["f"] == 0.0 and out["iters"] == 0


# -- metamorphic invariances ------------------------------------------------------

@pytest.mark.parametrize("fid", range(1, 9))
def test_permutation_and_sign_invariance(fid):
    r = np.random.default_rng(100 + fid)
    A = r.standard_normal((12, 20))
    par = 4 if fid <= 4 else {5: 3.0, 6: 10.0, 7: 0.4, 8: 1.5}[fid]
    X0 = _starts(5, 20, fid)
    base = oracle.am_multi(A, fid, par, X0, tol=1e-10, maxit=300)
    perm = r.permutation(20)
    sign = r.choice([-1.0, 1.0], size=20)
    A2 = A[:, perm] * sign
    X02 = X0[:, perm] * sign
    other = oracle.am_multi(A2, fid, par, X02, tol=1e-10, maxit=300)
    np.testing.assert_allclose(other["f"], base["f"], rtol=1e-9)
    np.testing.assert_allclose(other["X"], base["X"][:, perm] * sign, atol=1e-9)


@pytest.mark.parametrize("fid", L2_FIDS)
def test_orthogonal_row_mixing_invariance(fid):
    r = np.random.default_rng(110 + fid)
    A = r.standard_normal((10, 18))
    Q, _ = np.linalg.qr(r.standard_normal((10, 10)))
    par = 4 if fid <= 4 else {5: 3.0, 7: 0.4}[fid]
    X0 = _starts(4, 18, fid)
    a = oracle.am_multi(A, fid, par, X0, tol=1e-10, maxit=300)
    b = oracle.am_multi(Q @ A, fid, par, X0, tol=1e-10, maxit=300)
    np.testing.assert_allclose(a["f"], b["f"], rtol=1e-9)


def test_tol_negative_runs_maxit_and_threads_do_not_change_results():
    r = np.random.default_rng(120)
    A = r.standard_normal((20, 30))
    X0 = _starts(7, 30, 5)
    one = oracle.am_multi(A, 3, 4.0, X0, tol=-1.0, maxit=17, nthreads=1)
    four = oracle.am_multi(A, 3, 4.0, X0, tol=-1.0, maxit=17, nthreads=4)
    assert np.all(one["iters"] == 17) and np.all(one["status"] == oracle.MAXIT)
    assert np.array_equal(one["X"], four["X"]) and one["best"] == four["best"]
