"""Pins for the oracle's operators (Section 2.1 and Table 3).

Every check here is independent of the oracle's own arithmetic: the paper's
worked example, brute-force enumeration, a generic constrained optimiser
(scipy SLSQP) and a bounded scalar minimiser on the dual of S4.
"""
import itertools
import json
import os

import numpy as np
import pytest
from scipy import optimize

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_T_s_worked_example():
    with open(os.path.join(GOLDEN, "ts_worked_example.json")) as fh:
        ex = json.load(fh)
    out, phi = oracle.T_s(ex["a"], ex["s"])
    assert out.tolist() == ex["T_s"]
    assert phi == pytest.approx(np.linalg.norm(ex["T_s"]), rel=1e-15)


@pytest.mark.parametrize("seed", range(20))
def test_T_s_brute_force(seed):
    r = np.random.default_rng(seed)
    m = int(r.integers(1, 9))
    s = int(r.integers(0, m + 1))
    a = r.standard_normal(m)
    out, phi = oracle.T_s(a, s)
    # S3: max over ||z||_2 <= 1, ||z||_0 <= s of a^T z = max_{|S|=s} ||a_S||_2
    best = max((np.linalg.norm(a[list(S)]) for S in itertools.combinations(range(m), s)),
               default=0.0)
    assert phi == pytest.approx(best, rel=1e-14, abs=1e-300)
    assert np.count_nonzero(out) == min(s, m)
    kept = out != 0
    assert np.all(out[kept] == a[kept])
    if kept.any() and (~kept).any():
        assert np.min(np.abs(a[kept])) >= np.max(np.abs(a[~kept]))


def test_T_s_ties_go_to_lower_index():
    out, _ = oracle.T_s([3.0, -3.0, 1.0, 3.0], 2)
    assert out.tolist() == [3.0, -3.0, 0.0, 0.0]
    out, _ = oracle.T_s([0.5, 2.0, -2.0, 2.0], 1)
    assert out.tolist() == [0.0, 2.0, 0.0, 0.0]


@pytest.mark.parametrize("seed", range(20))
def test_U_gamma_brute_force(seed):
    r = np.random.default_rng(100 + seed)
    m = int(r.integers(1, 9))
    a = r.standard_normal(m) * 2
    gamma = float(r.uniform(0, 3))
    out, phi = oracle.U_gamma(a, gamma)
    # S5: max over ||z||_2 <= 1 of (a^T z)^2 - gamma ||z||_0
    #   = max over supports S (incl. empty) of ||a_S||^2 - gamma |S|
    best = 0.0
    for k in range(1, m + 1):
        for S in itertools.combinations(range(m), k):
            best = max(best, float(np.sum(a[list(S)] ** 2)) - gamma * k)
    assert phi == pytest.approx(best, rel=1e-13, abs=1e-13)
    # z* = U/||U|| attains it
    if np.any(out):
        z = out / np.linalg.norm(out)
        assert (a @ z) ** 2 - gamma * np.count_nonzero(z) == pytest.approx(phi, rel=1e-12)


def test_U_gamma_boundary_is_strict():
    out, phi = oracle.U_gamma([2.0, -1.0, 0.5], 1.0)
    assert out.tolist() == [2.0, 0.0, 0.0]  # a_i^2 = gamma is dropped: sgn(0) = 0
    assert phi == pytest.approx(3.0)


def _slsqp_max(fun, grad, x0, cons):
    res = optimize.minimize(lambda z: -fun(z), x0, jac=lambda z: -grad(z),
                            constraints=cons, method="SLSQP",
                            options={"ftol": 1e-14, "maxiter": 500})
    return -res.fun


@pytest.mark.parametrize("seed", range(12))
def test_V_gamma_against_slsqp(seed):
    r = np.random.default_rng(200 + seed)
    m = int(r.integers(2, 7))
    a = r.standard_normal(m)
    gamma = float(r.uniform(0, 0.8) * np.max(np.abs(a)))
    out, phi = oracle.V_gamma(a, gamma)
    # S6: max a^T z - gamma ||z||_1 s.t. ||z||_2 <= 1; split z = zp - zn
    fun = lambda w: a @ (w[:m] - w[m:]) - gamma * np.sum(w)
    grad = lambda w: np.concatenate([a - gamma, -a - gamma])
    cons = [{"type": "ineq", "fun": lambda w: 1 - np.sum((w[:m] - w[m:]) ** 2)}]
    best = -np.inf
    for trial in range(4):
        w0 = np.abs(r.standard_normal(2 * m)) * 0.1
        res = optimize.minimize(lambda w: -fun(w), w0, jac=lambda w: -grad(w),
                                bounds=[(0, None)] * (2 * m), constraints=cons,
                                method="SLSQP", options={"ftol": 1e-15, "maxiter": 1000})
        best = max(best, -res.fun)
    assert phi == pytest.approx(best, rel=1e-6, abs=1e-9)
    if np.any(out):
        z = out / np.linalg.norm(out)
        assert a @ z - gamma * np.sum(np.abs(z)) == pytest.approx(phi, rel=1e-12)


def _dual_S4(a, s, lam):
    return lam * np.sqrt(s) + np.linalg.norm(np.sign(a) * np.maximum(np.abs(a) - lam, 0))


@pytest.mark.parametrize("seed", range(25))
def test_lambda_s_minimises_the_dual(seed):
    r = np.random.default_rng(300 + seed)
    m = int(r.integers(1, 40))
    a = r.standard_normal(m)
    if seed % 5 == 0:
        a[r.integers(0, m, size=max(1, m // 3))] = 0.0
    s = float(r.uniform(1, m + 2)) if seed % 3 else float(r.integers(1, m + 1))
    lam = oracle.lambda_s(a, s)
    assert lam >= 0
    top = float(np.max(np.abs(a)))
    grid = np.linspace(0, top, 20001)
    g = np.array([_dual_S4(a, s, t) for t in grid])
    ref = optimize.minimize_scalar(lambda t: _dual_S4(a, s, t), bounds=(0, top),
                                   method="bounded", options={"xatol": 1e-13})
    dual_min = min(g.min(), ref.fun)
    assert _dual_S4(a, s, lam) <= dual_min + 1e-12 * max(1.0, dual_min)


@pytest.mark.parametrize("seed", range(15))
def test_V_lambda_s_primal_dual_and_slsqp(seed):
    r = np.random.default_rng(400 + seed)
    m = int(r.integers(2, 8))
    a = r.standard_normal(m)
    s = float(r.uniform(1, m))
    out, phi = oracle.V_lambda_s(a, s)
    lam = oracle.lambda_s(a, s)
    z = out / np.linalg.norm(out)
    # feasibility and primal value = dual value (Table 3, S4)
    assert np.sum(np.abs(z)) <= np.sqrt(s) * (1 + 1e-12)
    assert a @ z == pytest.approx(phi, rel=1e-12)
    if lam > 0:  # KKT: the L1 constraint is tight
        assert np.sum(np.abs(z)) == pytest.approx(np.sqrt(s), rel=1e-12)
    # generic solver on max a^T z, ||z||_2 <= 1, ||z||_1 <= sqrt(s)
    fun = lambda w: a @ (w[:m] - w[m:])
    grad = lambda w: np.concatenate([a, -a])
    cons = [{"type": "ineq", "fun": lambda w: 1 - np.sum((w[:m] - w[m:]) ** 2)},
            {"type": "ineq", "fun": lambda w: np.sqrt(s) - np.sum(w)}]
    best = -np.inf
    for trial in range(4):
        w0 = np.abs(r.standard_normal(2 * m)) * 0.1
        res = optimize.minimize(lambda w: -fun(w), w0, jac=lambda w: -grad(w),
                                bounds=[(0, None)] * (2 * m), constraints=cons,
                                method="SLSQP", options={"ftol": 1e-15, "maxiter": 1000})
        best = max(best, -res.fun)
    assert phi == pytest.approx(best, rel=1e-6)


def test_lambda_s_special_cases():
    a = np.array([3.0, -1.0, 2.0, 0.5])
    # s = 1: the L1 ball of radius 1 inside the unit L2 ball; z* = sign e_argmax
    out, phi = oracle.V_lambda_s(a, 1)
    assert np.count_nonzero(out) == 1 and out[0] > 0
    assert phi == pytest.approx(3.0, rel=1e-14)
    # constraint inactive when ||a||_1 <= sqrt(s) ||a||_2: lambda = 0
    assert oracle.lambda_s(a, 4.0) == 0.0
    out, phi = oracle.V_lambda_s(a, 4.0)
    assert np.allclose(out, a) and phi == pytest.approx(np.linalg.norm(a), rel=1e-14)
    assert oracle.lambda_s(np.zeros(5), 2.0) == 0.0


@pytest.mark.parametrize("seed", range(6))
def test_x_operator_dispatch(seed):
    r = np.random.default_rng(500 + seed)
    v = r.standard_normal(30)
    for fid in range(1, 9):
        par = 4 if fid <= 4 else 0.3
        w, phi = oracle.x_operator(fid, v, par)
        if fid in (1, 2):
            ref = oracle.T_s(v, 4)
        elif fid in (3, 4):
            ref = oracle.V_lambda_s(v, 4)
        elif fid in (5, 6):
            ref = oracle.U_gamma(v, 0.3)
        else:
            ref = oracle.V_gamma(v, 0.3)
        assert np.array_equal(w, ref[0]) and phi == ref[1]
