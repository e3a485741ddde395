"""The parity protocol the GPU tests use (tests/gpu_helpers.py), checked on
the CPU with the oracle on both sides: an exact copy of the oracle's results
passes; a start whose objective or status differs passes only when its
final iterate is a fixed point of Algorithm 2 (another stationary point, as
several correct results allow, Section 4); planted mistakes (an iterate
that is not a fixed point, a wrong objective, a best start above the
oracle's, a differing start with no iterate to certify) fail."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import (compare_solve, fixed_point_certificate, per_start_parity,
                         support_near_tie_margin)


@pytest.fixture(scope="module")
def case():
    sp = workloads.spiked_matrix(workloads.SEED_BASE + 500, 60, 300, thetas=(20.0, 12.0),
                                 spike_nnz=8)
    A = sp.A.astype(np.float64)
    X0 = workloads.random_unit_starts(workloads.SEED_BASE + 501, 12, 300)
    return A, X0


def _as_got(ref):
    return {"f_per_start": ref["f"].copy(), "status_per_start": ref["status"].copy(),
            "objective": float(ref["f"][ref["best"]]), "X_final": ref["X"].copy()}


@pytest.mark.parametrize("fid,par", [(1, 8), (2, 8), (3, 6.0), (4, 6.0), (5, 2.0),
                                     (6, 200.0), (7, 1.0), (8, 10.0)])
def test_oracle_against_itself_passes(case, fid, par):
    A, X0 = case
    ref = oracle.am_multi(A, fid, par, X0, 1e-10, 400)
    info = compare_solve(_as_got(ref), ref, f"self F{fid}", A, fid, par)
    assert info["certified"] == 0 and info["start_match"] == 1.0


@pytest.mark.parametrize("fid,par", [(1, 8), (4, 6.0), (5, 2.0), (8, 10.0)])
def test_converged_iterates_pass_the_certificate(case, fid, par):
    A, X0 = case
    ref = oracle.am_multi(A, fid, par, X0, 1e-12, 1000)
    for j in range(len(X0)):
        if ref["f"][j] == 0:
            continue
        c = fixed_point_certificate(A, fid, par, ref["X"][j], ref["f"][j])
        assert c["ok"], (j, c)


def test_another_stationary_point_is_certified(case):
    """Start 0 reported at the stationary point reached from start 1 (as if
    its trajectory had split at a near-tie): certified, so it passes."""
    A, X0 = case
    ref = oracle.am_multi(A, 1, 8, X0, 1e-12, 1000)
    got = _as_got(ref)
    order = np.argsort(ref["f"])
    lo, hi = order[0], order[-1]
    assert ref["f"][hi] > ref["f"][lo] * (1 + 1e-4)
    got["f_per_start"][lo] = ref["f"][hi]
    got["X_final"][lo] = ref["X"][hi]
    info = compare_solve(got, ref, "split", A, 1, 8)
    assert info["certified"] == 1


def test_status_difference_needs_certificate(case):
    A, X0 = case
    ref = oracle.am_multi(A, 3, 6.0, X0, 1e-12, 1000)
    got = _as_got(ref)
    got["status_per_start"][2] = 1 - got["status_per_start"][2] if got[
        "status_per_start"][2] in (0, 1) else 0
    assert compare_solve(got, ref, "status", A, 3, 6.0)["certified"] == 1
    got["X_final"] = None
    with pytest.raises(AssertionError):
        compare_solve(got, ref, "status, no iterate", A, 3, 6.0)


def test_planted_iterate_that_is_not_a_fixed_point_fails(case):
    """A differing start whose iterate is the one after a single AM step
    from its start: one more step still gains, so it is rejected."""
    A, X0 = case
    ref = oracle.am_multi(A, 1, 8, X0, 1e-12, 1000)
    early = oracle.am_multi(A, 1, 8, X0, -1.0, 1)
    got = _as_got(ref)
    j = int(np.argmax(ref["f"] - early["f"]))
    assert ref["f"][j] - early["f"][j] > 1e-3 * ref["f"][j]
    got["f_per_start"][j] = early["f"][j]
    got["X_final"][j] = early["X"][j]
    with pytest.raises(AssertionError):
        compare_solve(got, ref, "planted non-fixed point", A, 1, 8)


def test_planted_wrong_objective_fails(case):
    """The iterate is right but the reported objective is not its f."""
    A, X0 = case
    ref = oracle.am_multi(A, 5, 2.0, X0, 1e-12, 1000)
    got = _as_got(ref)
    got["f_per_start"][4] *= 1 + 1e-4
    with pytest.raises(AssertionError):
        compare_solve(got, ref, "planted objective", A, 5, 2.0)


def test_planted_best_above_oracle_fails(case):
    A, X0 = case
    ref = oracle.am_multi(A, 7, 1.0, X0, 1e-12, 1000)
    got = _as_got(ref)
    got["objective"] = float(ref["f"][ref["best"]]) * (1 + 1e-4)
    with pytest.raises(AssertionError):
        compare_solve(got, ref, "planted best", A, 7, 1.0)


def test_near_tie_margin_of_a_planted_tie():
    """Two equal columns give equal |v_i|: at s = 1 they compete for the
    one place of T_s and the margin of that decision is zero; at s = 3 the
    cut falls between distinct values."""
    A = np.eye(4)
    A[:, 3] = A[:, 2]
    x = np.array([0.6, 0.5, 0.4, 0.4])  # v is proportional to (0.6, 0.5, 0.8, 0.8)
    assert support_near_tie_margin(A, x, 1, 1) == 0.0
    assert support_near_tie_margin(A, x, 1, 3) == pytest.approx(1 / 6)


def test_per_start_parity_counts(case):
    A, X0 = case
    ref = oracle.am_multi(A, 2, 8, X0, 1e-12, 1000)
    got = _as_got(ref)
    match, n_cert = per_start_parity(got, ref, "counts", A, 2, 8)
    assert match == 1.0 and n_cert == 0


def test_early_stop_on_the_same_trajectory_passes(case):
    """A start reported CONVERGED a few x-updates before the oracle stops
    (as when the FP32 ratio test meets a tolerance below its resolution):
    its iterate is the oracle's after the same number of x-updates, so it
    passes; the same iterate reported with another iteration count fails."""
    A, X0 = case
    ref = oracle.am_multi(A, 5, 2.0, X0, 1e-12, 1000)
    j = int(np.argmax(ref["iters"]))
    k = int(ref["iters"][j])
    while True:  # the last x-update count whose iterate is clearly short of the end
        k -= 1
        early = oracle.am_single(A, 5, 2.0, X0[j], -1.0, k)
        if ref["f"][j] - early["f"] > 1e-4 * ref["f"][j]:
            break
    assert not fixed_point_certificate(A, 5, 2.0, early["x"], early["f"])["ok"]
    got = _as_got(ref)
    got["iters_per_start"] = ref["iters"].copy()
    got["iters_per_start"][j] = k
    got["f_per_start"][j] = early["f"]
    got["X_final"][j] = early["x"]
    got["status_per_start"][j] = 0
    info = compare_solve(got, ref, "early stop", A, 5, 2.0, X0=X0)
    assert info["certified"] == 1
    got["iters_per_start"][j] = k + 3
    with pytest.raises(AssertionError):
        compare_solve(got, ref, "early stop, wrong count", A, 5, 2.0, X0=X0)


def _trajectory(A, fid, par, x0, K):
    xs, x = [], np.asarray(x0, np.float64)
    for _ in range(K):
        x = oracle.am_single(A, fid, par, x, -1.0, 1)["x"]
        xs.append(x.copy())
    return xs


def test_stepwise_check_accepts_a_valid_trajectory_and_rejects_a_wrong_step(case):
    """Step-by-step certificate: a trajectory whose every step is the FP64
    map of its predecessor (here from a start perturbed at rounding level,
    and not yet converged) passes; the same trajectory with one step taken
    by a wrong operator (T_s with s - 1) fails at that step."""
    from gpu_helpers import plain_step, stepwise_check

    A, X0 = case
    fid, par, K = 1, 8, 12
    x0 = X0[3] * (1 + 1e-9 * np.random.default_rng(0).standard_normal(X0.shape[1]))
    xs = _trajectory(A, fid, par, x0, K)
    step, margin = plain_step(A, fid, par)
    assert stepwise_check(A, X0[3], xs, step, margin)["ok"]
    bad = list(xs)
    w, _ = oracle.x_operator(fid, A.T @ (A @ xs[4] / np.linalg.norm(A @ xs[4])), par - 1)
    bad[5] = w / np.linalg.norm(w)
    r = stepwise_check(A, X0[3], bad, step, margin)
    assert not r["ok"] and r["k"] == 6


def test_unconverged_differing_start_needs_the_stepwise_check(case, monkeypatch):
    """Fixed work too short to converge, and a start reported at the end of
    another valid trajectory (as after a split at a near-tie): the
    fixed-point certificate does not cover it and, with the oracle's
    trajectory check made to miss (a split), only the stepwise check
    does; a planted wrong step then fails."""
    import gpu_helpers

    A, X0 = case
    fid, par, K = 3, 6.0, 4
    ref = oracle.am_multi(A, fid, par, X0, -1.0, K)
    j = 5
    X0b = X0.copy()
    X0b[j] = X0[(j + 1) % len(X0)]
    xs = _trajectory(A, fid, par, X0b[j], K)
    got = _as_got(ref)
    got["iters_per_start"] = ref["iters"].copy()
    got["f_per_start"][j] = oracle.objective(fid, A, xs[-1], par)[0]
    got["X_final"][j] = xs[-1]
    got["objective"] = float(np.max(got["f_per_start"]))
    if got["objective"] > ref["f"][ref["best"]]:
        pytest.skip("the planted trajectory beats the oracle's best")
    assert not fixed_point_certificate(A, fid, par, xs[-1], got["f_per_start"][j])["ok"]
    monkeypatch.setattr(gpu_helpers, "trajectory_check",
                        lambda *a, **k: {"ok": False, "why": "split"})
    with pytest.raises(AssertionError):
        compare_solve(got, ref, "unconverged, no stepper", A, fid, par, X0=X0b)

    def stepper(k):
        Xk = oracle.am_multi(A, fid, par, X0, -1.0, k)["X"]
        Xk[j] = xs[k - 1]
        return Xk
    info = compare_solve(got, ref, "unconverged, stepwise", A, fid, par, X0=X0b,
                         stepper=stepper)
    assert info["certified"] == 1

    def bad_stepper(k):
        Xk = stepper(k)
        if k == 2:
            Xk[j] = np.roll(Xk[j], 1)
        return Xk
    with pytest.raises(AssertionError):
        compare_solve(got, ref, "unconverged, wrong step", A, fid, par, X0=X0b,
                      stepper=bad_stepper)
