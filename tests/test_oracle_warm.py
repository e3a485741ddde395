"""Pins of the oracle's sparsity-targeted warm-up (Section 4.1): the
parameter follows v for warm_iters x-updates, then is frozen.

* warm_iters = 0 is the plain algorithm, bit for bit;
* gamma re-targeted to s nonzeros on every iteration turns U_gamma into T_s,
  so the warm L0 penalties reproduce the L0 constraints (F5 = F1, F6 = F2);
* each warm iterate of V_gamma has exactly s nonzeros with gamma the
  (s+1)-th largest |v_i| of that iteration, recomputed here from the
  previous iterate;
* after the warm-up the iteration is the plain penalty / soft-threshold AM
  with the frozen value (checked by restarting a plain run from the iterate
  and parameter at the freeze);
* no start stops before the parameter is frozen; the best start has the
  largest explained variance."""
import numpy as np
import pytest

import oracle
import workloads


@pytest.fixture(scope="module")
def prob():
    sp = workloads.spiked_matrix(91, 60, 400, thetas=(30.0, 15.0), spike_nnz=10)
    X0 = workloads.random_unit_starts(92, 5, 400)
    return sp.A.astype(np.float64), X0


def _y(A, x, fid):
    u = A @ x
    return np.sign(u) if fid % 2 == 0 else u / np.linalg.norm(u)


@pytest.mark.parametrize("fid,par", [(3, 5.0), (4, 7.5), (5, 0.5), (6, 40.0), (7, 0.6),
                                     (8, 9.0)])
def test_zero_warmup_is_the_plain_algorithm(prob, fid, par):
    A, X0 = prob
    a = oracle.am_multi(A, fid, par, X0, 1e-9, 100)
    b = oracle.am_multi_warm(A, fid, par, X0, 1e-9, 100, 0, 12)
    assert np.array_equal(a["X"], b["X"])
    assert np.array_equal(a["f"], b["f"]) and np.array_equal(a["iters"], b["iters"])


@pytest.mark.parametrize("pen,con", [(5, 1), (6, 2)])
def test_warm_l0_penalty_reproduces_l0_constraint(prob, pen, con):
    A, X0 = prob
    s = 12
    a = oracle.am_multi(A, con, s, X0, -1.0, 30)
    b = oracle.am_multi_warm(A, pen, 0.0, X0, -1.0, 30, 1000, s)
    assert np.array_equal(a["X"], b["X"])
    assert np.all((b["X"] != 0).sum(axis=1) == s)


@pytest.mark.parametrize("fid", [7, 8])
def test_warm_soft_threshold_targets_s(prob, fid):
    A, X0 = prob
    s, m = 9, 12
    full = oracle.am_multi_warm(A, fid, 0.0, X0, -1.0, m, 1000, s)
    prev = oracle.am_multi_warm(A, fid, 0.0, X0, -1.0, m - 1, 1000, s)
    for j in range(len(X0)):
        x = full["X"][j]
        assert np.count_nonzero(x) == s
        v = A.T @ _y(A, prev["X"][j], fid)
        g = np.sort(np.abs(v))[::-1][s]
        # numpy's product sums in another order: agreement to rounding
        assert abs(full["param"][j] - g) <= 1e-13 * g
        w = np.sign(v) * np.maximum(np.abs(v) - g, 0.0)
        np.testing.assert_allclose(x, w / np.linalg.norm(w), rtol=0, atol=1e-12)


@pytest.mark.parametrize("fid,plain,par", [(3, 7, 5.0), (4, 8, 5.0), (5, 5, None),
                                           (7, 7, None)])
def test_after_warmup_parameter_is_frozen(prob, fid, plain, par):
    A, X0 = prob
    K, m, s = 3, 15, 10
    warm = oracle.am_multi_warm(A, fid, par if par else 0.0, X0, -1.0, m, K, s)
    at_k = oracle.am_multi_warm(A, fid, par if par else 0.0, X0, -1.0, K, K, s)
    for j in range(len(X0)):
        # the frozen value is the one of the K-th x-update
        assert warm["param"][j] == at_k["param"][j]
        rest = oracle.am_multi(A, plain, at_k["param"][j], at_k["X"][j:j + 1], -1.0, m - K)
        np.testing.assert_allclose(warm["X"][j], rest["X"][0], rtol=0, atol=1e-13)


@pytest.mark.parametrize("fid", [7, 6, 8])
def test_no_stop_before_freeze_and_best_by_explained_variance(prob, fid):
    A, X0 = prob
    res = oracle.am_multi_warm(A, fid, 0.0, X0, 1e-3, 200, 6, 10)
    assert np.all(res["iters"] >= 7)
    assert res["best"] == int(np.argmax(res["ev"]))
    # each start's explained variance is that of its returned x: ||Ax||_2^2
    # for L2 variance, ||Ax||_1 (the value y^T A x at y = sgn(Ax)) for L1
    for j in range(len(X0)):
        x = res["X"][j]
        u = A @ x
        want = float(np.sign(u) @ u) if fid % 2 == 0 else float(u @ u)
        assert res["ev"][j] == pytest.approx(want, rel=1e-12)
