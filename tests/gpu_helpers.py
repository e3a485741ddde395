"""Helpers shared by the GPU tests: device upload in the library's layout and
the parity protocol used to compare a batched solve with the FP64 oracle."""
import numpy as np

REL_TOL_FP32 = 1e-5  # relative objective error allowed for the FP32 path


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


def compare_solve(got, ref, label, rel_tol=REL_TOL_FP32, min_start_match=0.9):
    """Parity of a batched GPU solve against the oracle on the same starts.

    * the best objective agrees within rel_tol;
    * per start, the objective agrees within rel_tol for at least
      ``min_start_match`` of the starts (trajectories may split at near-ties
      and end at different stationary points; no GPU start may exceed the
      oracle's best by more than the tolerance);
    * per-start status agrees for the matching starts.
    Returns a dict of diagnostics.
    """
    f_ref = ref["f"]
    f_got = got["f_per_start"]
    best_ref = f_ref[ref["best"]]
    err_best = rel_err(got["objective"], best_ref)
    match = np.array([rel_err(a, b) <= rel_tol or abs(a - b) <= rel_tol * abs(best_ref)
                      for a, b in zip(f_got, f_ref)])
    info = {"label": label, "best_rel_err": err_best, "start_match": float(match.mean()),
            "gpu_best": got["objective"], "oracle_best": best_ref}
    print("parity", info, flush=True)
    assert err_best <= rel_tol, info
    assert match.mean() >= min_start_match, info
    assert np.all(f_got <= best_ref + rel_tol * max(abs(best_ref), 1e-300)), info
    st_ok = got["status_per_start"][match] == ref["status"][match]
    assert st_ok.mean() >= 0.9, (info, got["status_per_start"], ref["status"])
    return info


def support_near_tie_margin(A, x_best, fid, s_or_gamma):
    """Relative margin of the decision that fixed the oracle's best support:
    for T_s the gap between the s-th and (s+1)-th |v_i|, for the thresholds
    the smallest | |v_i| - lambda | relative to lambda (FP64)."""
    A = np.asarray(A, np.float64)
    u = A @ x_best
    if not np.any(u):
        return np.inf
    y = np.sign(u) if fid % 2 == 0 else u / np.linalg.norm(u)
    v = np.abs(A.T @ y)
    if fid <= 2:
        srt = np.sort(v)[::-1]
        s = int(s_or_gamma)
        if s >= v.size:
            return np.inf
        return (srt[s - 1] - srt[s]) / max(srt[s - 1], 1e-300)
    if fid in (5, 6):
        return np.min(np.abs(v * v - s_or_gamma)) / max(s_or_gamma, 1e-300)
    if fid in (7, 8):
        return np.min(np.abs(v - s_or_gamma)) / max(s_or_gamma, 1e-300)
    return np.inf
