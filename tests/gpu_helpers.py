"""Helpers shared by the GPU tests: device upload in the library's layout and
the parity protocol used to compare a batched solve with the FP64 oracle.

The protocol (several correct results, Section 4: trajectories from
different starts, or from one start under different rounding, may split at
a near-tie and end at different stationary points of Algorithm 2):

1. the best-of-r objective agrees with the oracle's best-of-r on the same
   starts within the tolerance;
2. every start agrees with the oracle's run from the same start (objective
   within the tolerance and the same status), or else
   a. its final iterate is the oracle's iterate from the same start after
      the same number of x-updates (same support, objective within the
      tolerance): the trajectories agree and only the stop test fired at
      another iteration (the ratio test reads phi to FP32 resolution, so a
      tolerance below it can stop earlier or later; iteration counts are
      not pinned), or
   b. its final iterate passes the FP64 fixed-point certificate: one more
      FP64 step of Algorithm 2 from it keeps its support (up to a
      near-tie, whose margin is printed) and raises the objective by no
      more than the tolerance (another stationary point), or
   c. every step of its GPU trajectory is the FP64 step of Algorithm 2
      from the GPU's previous iterate: the same support, unless that
      step's decision was a near-tie (relative margin below 1e-5, printed:
      the place where the trajectories split), and values within FP32
      rounding.  The GPU iterates come from re-running the solve with
      maxit = 1, 2, ... (the solve is deterministic, and a start's
      arithmetic does not depend on the other starts).
   No start is let through without one of them;
3. no start exceeds the oracle's best by more than the tolerance.
"""
import numpy as np

import oracle

REL_TOL_FP32 = 1e-5  # relative objective error allowed for the FP32 path
NEAR_TIE = 1e-5      # relative margin below which a support decision is a tie


def to_device_colmajor(A_np, device="cuda:0", lda=None):
    """Upload an n x p matrix as a column-major (n, p) tensor, strides (1, lda)."""
    import torch

    n, p = A_np.shape
    lda = lda or n
    buf = torch.zeros((p, lda), dtype=torch.float32)
    buf[:, :n] = torch.from_numpy(np.ascontiguousarray(np.asarray(A_np, np.float32).T))
    dev = buf.to(device)
    return dev[:, :n].t()


def to_device_rows(X_np, device="cuda:0"):
    import torch

    return torch.from_numpy(np.ascontiguousarray(np.asarray(X_np, np.float32))).to(device)


def rel_err(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _image(A, fid, x):
    """v = A^T y(x) in FP64 (the argument of the x-operator one step on)."""
    u = A @ x
    if not np.any(u):
        return None
    y = np.sign(u) if fid % 2 == 0 else u / np.linalg.norm(u)
    return A.T @ y


def support_near_tie_margin(A, x, fid, s_or_gamma):
    """Relative margin of the decision that fixes the support of the image of
    x: for T_s the gap between the s-th and (s+1)-th |v_i| (relative to the
    s-th), for U_gamma / V_gamma / V_lambda the smallest distance of v_i^2 or
    |v_i| to the threshold, relative to the threshold (FP64)."""
    A = np.asarray(A, np.float64)
    v = _image(A, fid, np.asarray(x, np.float64))
    if v is None:
        return np.inf
    v = np.abs(v)
    if fid <= 2:
        srt = np.sort(v)[::-1]
        s = int(s_or_gamma)
        if s >= v.size:
            return np.inf
        return (srt[s - 1] - srt[s]) / max(srt[s - 1], 1e-300)
    if fid <= 4:
        lam = oracle.lambda_s(v, s_or_gamma)
        if lam <= 0:
            return np.inf
        return np.min(np.abs(v - lam)) / lam
    if s_or_gamma <= 0:
        return np.inf
    if fid in (5, 6):
        return np.min(np.abs(v * v - s_or_gamma)) / s_or_gamma
    return np.min(np.abs(v - s_or_gamma)) / s_or_gamma


def fixed_point_certificate(A, fid, s_or_gamma, x, f_reported, rel_tol=REL_TOL_FP32):
    """FP64 certificate that x (a final iterate of the GPU path) is a
    stationary point of Algorithm 2: one more FP64 step from x keeps its
    support (or the decision is a near-tie) and raises f by at most rel_tol
    relative; also f(x) in FP64 agrees with the reported objective.
    Returns a dict with 'ok' and the figures."""
    A = np.asarray(A, np.float64)
    x = np.asarray(x, np.float64)
    nx = np.linalg.norm(x)
    if nx == 0:
        return {"ok": False, "why": "zero iterate"}
    x = x / nx
    f0, _ = oracle.objective(fid, A, x, s_or_gamma)
    step = oracle.am_single(A, fid, s_or_gamma, x, -1.0, 1)
    f1 = step["f"]
    scale = max(abs(f0), 1e-300)
    gain = (f1 - f0) / scale
    same = np.array_equal(np.flatnonzero(step["x"]), np.flatnonzero(x))
    margin = support_near_tie_margin(A, x, fid, s_or_gamma)
    consistent = abs(f0 - f_reported) <= 1e-6 * scale
    ok = bool(gain <= rel_tol and (same or margin < NEAR_TIE) and consistent)
    return {"ok": ok, "gain": gain, "same_support": bool(same), "margin": margin,
            "f_x": f0, "f_reported": f_reported}


def trajectory_check(A, fid, s_or_gamma, x0, iters, x, f_reported, rel_tol=REL_TOL_FP32):
    """Does the final iterate x (reported objective f_reported, after
    ``iters`` x-updates) coincide with the oracle's iterate from the same
    start x0 after the same number of x-updates (stop test off)?"""
    run = oracle.am_single(A, fid, s_or_gamma, x0, -1.0, int(iters))
    x = np.asarray(x, np.float64)
    same = np.array_equal(np.flatnonzero(run["x"]), np.flatnonzero(x))
    scale = max(abs(run["f"]), 1e-300)
    close = abs(run["f"] - f_reported) <= rel_tol * scale
    return {"ok": bool(same and close), "f_oracle_same_iters": run["f"],
            "same_support": bool(same), "iters": int(iters)}


def y_tie_margin(A, fid, x):
    """Relative margin of the sign decisions of the L1-variance y-update at x:
    min |u_i| over max |u_i| with u = A x (infinite for L2 variance)."""
    if fid % 2 == 1:
        return np.inf
    u = np.abs(np.asarray(A, np.float64) @ np.asarray(x, np.float64))
    top = u.max()
    return np.inf if top == 0 else float(u.min() / top)


def stepwise_check(A, x0, iterates, step, margin, x_tol=1e-4):
    """Check a GPU trajectory step by step: ``iterates[k-1]`` is the GPU
    iterate after k x-updates, ``step(prev, k)`` the FP64 image of prev
    under the k-th x-update, ``margin(prev, k)`` the relative margin of that
    step's support decision.  Every step must give the FP64 image's support
    (or be a near-tie: a split) and its values within x_tol."""
    prev = np.asarray(x0, np.float64)
    splits = []
    for k, xg in enumerate(iterates, 1):
        xg = np.asarray(xg, np.float64)
        ng = np.linalg.norm(xg)
        xo = step(prev, k)
        no = np.linalg.norm(xo)
        if ng == 0 or no == 0:
            if not (ng == 0 and no == 0):
                m = margin(prev, k)
                if m >= NEAR_TIE:
                    return {"ok": False, "k": k, "why": "zero on one side", "margin": m}
                splits.append((k, m))
            break
        xg = xg / ng
        if not np.array_equal(xg != 0, xo != 0):
            m = margin(prev, k)
            if m >= NEAR_TIE:
                return {"ok": False, "k": k, "why": "support", "margin": m,
                        "nnz_gpu": int(np.count_nonzero(xg)), "nnz_fp64": int(np.count_nonzero(xo))}
            splits.append((k, m))
        else:
            dx = float(np.max(np.abs(xg - xo)))
            if dx > x_tol:
                m = margin(prev, k)
                if m >= NEAR_TIE:
                    return {"ok": False, "k": k, "why": "values", "dx": dx, "margin": m}
                splits.append((k, m))
        prev = xg
    return {"ok": True, "steps": len(iterates), "splits": splits}


def plain_step(A, fid, par):
    """The k-th x-update of Algorithm 2 and the margin of its decisions."""
    def step(prev, k):
        return oracle.am_single(A, fid, par, prev, -1.0, 1)["x"]

    def margin(prev, k):
        return min(support_near_tie_margin(A, prev, fid, par), y_tie_margin(A, fid, prev))
    return step, margin


def per_start_parity(got, ref, label, A=None, fid=None, s_or_gamma=None,
                     rel_tol=REL_TOL_FP32, params=None, cert_fid=None, X0=None,
                     stepper=None, step_fns=None):
    """Step 2 of the protocol: every start agrees with the oracle's run from
    the same start (objective within rel_tol, same status) or its final
    iterate ``got['X_final'][j]`` passes the FP64 fixed-point certificate on
    (A, fid, s_or_gamma).  Under the warm-up the map after the freeze is the
    one to certify: ``params`` gives each start's frozen parameter and
    ``cert_fid`` the formulation whose x-operator it parameterises (the
    objective is then not compared, as the two formulations' f differ).
    With the starts ``X0`` (host, one per row) a differing start is first
    checked against the oracle's trajectory from its start (2a above).
    ``stepper(k)`` re-runs the GPU solve for k x-updates and returns its
    final iterates (rows as in got); with it, a start that fails 2a and 2b
    is checked step by step (2c); ``step_fns(j)`` gives that start's
    (step, margin) pair when it is not the plain map of (fid, s_or_gamma).
    Returns (fraction of agreeing starts, number certified)."""
    f_ref = np.asarray(ref["f"])
    f_got = np.asarray(got["f_per_start"])
    scale_best = max(abs(f_ref[ref["best"]]), 1e-300)
    f_ok = np.array([abs(a - b) <= rel_tol * max(abs(b), 1e-300)
                     or abs(a - b) <= rel_tol * scale_best for a, b in zip(f_got, f_ref)])
    st_ok = np.asarray(got["status_per_start"]) == np.asarray(ref["status"])
    both_zero = (f_got == 0) & (f_ref == 0)
    agree = (f_ok & st_ok) | both_zero
    X = got.get("X_final")
    n_cert = 0
    pending = []
    for j in np.flatnonzero(~agree):
        assert X is not None and A is not None, (
            f"{label}: start {j} differs from the oracle (gpu f {f_got[j]!r} status "
            f"{got['status_per_start'][j]}, oracle f {f_ref[j]!r} status "
            f"{ref['status'][j]}) and no final iterate was given to certify it")
        xj = X[j].detach().cpu().numpy() if hasattr(X, "detach") else np.asarray(X[j])
        par = s_or_gamma if params is None else float(params[j])
        n_cert += 1
        if X0 is not None and params is None and "iters_per_start" in got:
            t = trajectory_check(A, fid, par, X0[j], got["iters_per_start"][j], xj,
                                 f_got[j], rel_tol)
            print(f"{label}: start {j} gpu f {f_got[j]:.10g} oracle f {f_ref[j]:.10g} "
                  f"-> trajectory {t}", flush=True)
            if t["ok"]:
                continue
        cf = cert_fid or fid
        c = fixed_point_certificate(A, cf, par, xj, f_got[j], rel_tol)
        if cf != fid:
            c["ok"] = c["ok"] or (c.get("gain", np.inf) <= rel_tol and
                                  (c["same_support"] or c["margin"] < NEAR_TIE))
        print(f"{label}: start {j} gpu f {f_got[j]:.10g} oracle f {f_ref[j]:.10g} "
              f"-> certificate {c}", flush=True)
        if c["ok"]:
            continue
        assert stepper is not None and X0 is not None, (label, j, c)
        pending.append(int(j))
    if pending:
        kmax = int(max(got["iters_per_start"][j] for j in pending))
        traj = {j: [] for j in pending}
        for k in range(1, kmax + 1):
            Xk = stepper(k)
            Xk = Xk.detach().cpu().numpy() if hasattr(Xk, "detach") else np.asarray(Xk)
            for j in pending:
                if k <= got["iters_per_start"][j]:
                    traj[j].append(Xk[j].astype(np.float64))
        for j in pending:
            step, margin = (step_fns(j) if step_fns is not None
                            else plain_step(A, fid, s_or_gamma))
            r = stepwise_check(np.asarray(A, np.float64), X0[j], traj[j], step, margin)
            print(f"{label}: start {j} -> stepwise {r}", flush=True)
            assert r["ok"], (label, j, r)
    return float(agree.mean()), n_cert


def compare_solve(got, ref, label, A=None, fid=None, s_or_gamma=None,
                  rel_tol=REL_TOL_FP32, X0=None, stepper=None):
    """Parity of a batched GPU solve against the oracle on the same starts
    (the protocol in the module docstring).  ``A``, ``fid`` and
    ``s_or_gamma`` (the problem, FP64 or FP32 host array) and
    ``got['X_final']`` (the GPU's final iterates) are needed to certify a
    start that differs, and ``X0`` (host starts) to check it against the
    oracle's trajectory.  Returns a dict of diagnostics."""
    f_ref = np.asarray(ref["f"])
    f_got = np.asarray(got["f_per_start"])
    best_ref = f_ref[ref["best"]]
    scale_best = max(abs(best_ref), 1e-300)
    err_best = rel_err(got["objective"], best_ref)
    match, n_cert = per_start_parity(got, ref, label, A, fid, s_or_gamma, rel_tol, X0=X0,
                                     stepper=stepper)
    info = {"label": label, "best_rel_err": err_best, "start_match": match,
            "certified": n_cert, "gpu_best": got["objective"], "oracle_best": best_ref}
    print("parity", info, flush=True)
    assert err_best <= rel_tol, info
    assert np.all(f_got <= best_ref + rel_tol * scale_best), info
    return info


def gpu_stepper(solve, *args, rows=None, **kw):
    """stepper(k) for per_start_parity: the final iterates of the same GPU
    solve (``solve``: spca.am_solve or spca.am_solve_sparse, with its
    arguments) run for k x-updates; ``rows`` selects the starts compared."""
    kw = dict(kw)
    kw["return_X"] = True

    def run(k):
        kw["maxit"] = k
        X = solve(*args, **kw)["X_final"]
        return X if rows is None else X[rows]
    return run


def subset(got, idx):
    """The per-start outputs of a GPU solve restricted to the starts idx
    (to compare a sample of starts with the oracle run on those starts)."""
    idx = np.asarray(idx)
    out = {k: np.asarray(got[k])[idx] for k in ("f_per_start", "status_per_start",
                                                 "iters_per_start", "ev_per_start")}
    out["X_final"] = got["X_final"][idx] if got.get("X_final") is not None else None
    out["objective"] = float(np.max(out["f_per_start"]))
    return out
