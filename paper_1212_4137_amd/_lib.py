"""ctypes binding of ``libspca.so`` (argument marshalling only).

Every step of the AM iteration runs in the HIP library; this module only
turns torch tensors into pointers and host arrays back into numpy.  It never
falls back to a CPU implementation: if the library is missing or the device
is not a GPU, it raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libspca.so")

SPCA_OK, SPCA_EINVAL, SPCA_ENOMEM, SPCA_EHIP = 0, -1, -2, -3
CONVERGED, MAXIT, DEGENERATE, ZERO = 0, 1, 2, 3
WARN_NONE, WARN_ALL_DEGENERATE, WARN_ALL_ZERO, WARN_NO_CONVERGED = 0, 1, 2, 3
PREC_FP32, PREC_BF16_POLISH = 0, 1
FLAG_GRAPH, FLAG_CHECK_FINITE, FLAG_DENSE_ONLY, FLAG_AUTOTUNE, FLAG_NO_UNION = 1, 2, 4, 8, 16
FLAG_SPARSE_PANELS, FLAG_SPARSE_NO_PANELS, FLAG_TIME_SAMPLED = 32, 64, 128

EXPORTED = ("spca_am_solve", "spca_am_solve_ex", "spca_ctx_create",
            "spca_ctx_destroy", "spca_workspace_bytes", "spca_last_error",
            "spca_gemm_nt_f32", "spca_gemm_nt_bf16", "spca_gemm_nt_f32_shape",
            "spca_gemm_nt_f32_plan", "spca_x_update", "spca_generate_spiked",
            "spca_ctx_set_workspace", "spca_request_footprint", "spca_server_create",
            "spca_server_submit", "spca_server_poll", "spca_server_stats",
            "spca_server_destroy", "spca_tune_table_export", "spca_tune_table_import",
            "spca_tune_table_clear", "spca_gemm_nt_bf16_shape", "spca_am_components",
            "spca_am_solve_sparse", "spca_am_components_sparse", "spca_x_update_noalloc",
            "spca_am_solve_group", "spca_group_workspace_bytes", "spca_server_set_group_limit")
GROUP_MAX_REQUESTS, GROUP_MAX_P, GROUP_MAX_STARTS = 1024, 12288, 65536


class SpcaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libspca error {code}: {msg}")
        self.code = code


class Result(ctypes.Structure):
    _fields_ = [("objective", ctypes.c_double), ("explained_var", ctypes.c_double),
                ("phi", ctypes.c_double), ("iters_x_starts", ctypes.c_double),
                ("best_start", ctypes.c_int32), ("nnz", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("objective_pre_polish", ctypes.c_double),
                ("polish_iters", ctypes.c_int32), ("warning", ctypes.c_int32)]


class Problem(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("n", ctypes.c_int64), ("p", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("formulation", ctypes.c_int32),
                ("s_or_gamma", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("X0", ctypes.c_void_p), ("r", ctypes.c_int32), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("polish_maxit", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("total_starts", ctypes.c_int32),
                ("warmup_iters", ctypes.c_int32), ("target_nnz", ctypes.c_int32),
                ("deflate_X", ctypes.c_void_p), ("deflate_k", ctypes.c_int32)]


class Outputs(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("support", ctypes.c_void_p),
                ("res", ctypes.POINTER(Result)),
                ("f_per_start", ctypes.c_void_p), ("ev_per_start", ctypes.c_void_p),
                ("phi_per_start", ctypes.c_void_p), ("iters_per_start", ctypes.c_void_p),
                ("status_per_start", ctypes.c_void_p), ("nnz_per_start", ctypes.c_void_p),
                ("X_final", ctypes.c_void_p), ("kernel_times", ctypes.c_void_p),
                ("param_per_start", ctypes.c_void_p)]


class SparseProblem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("p", ctypes.c_int64), ("col_ptr", ctypes.c_void_p),
                ("row_idx", ctypes.c_void_p), ("col_val", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("row_val", ctypes.c_void_p), ("formulation", ctypes.c_int32),
                ("s_or_gamma", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("n", ctypes.c_int64), ("p", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("seed", ctypes.c_uint64), ("k", ctypes.c_int32),
                ("formulation", ctypes.c_int32), ("thetas", ctypes.c_void_p),
                ("U", ctypes.c_void_p), ("V", ctypes.c_void_p),
                ("start_seed", ctypes.c_uint64), ("s_or_gamma", ctypes.c_double),
                ("gamma_rel", ctypes.c_double), ("r", ctypes.c_int32),
                ("maxit", ctypes.c_int32), ("tol", ctypes.c_double),
                ("precision", ctypes.c_int32), ("polish_maxit", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("x_out", ctypes.c_void_p), ("support_out", ctypes.c_void_p)]


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("rc", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("res", Result), ("s_or_gamma", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_solve", ctypes.c_double), ("t_done", ctypes.c_double), ("footprint", ctypes.c_size_t),
                ("error", ctypes.c_char * 160)]


class ServerStats(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_size_t), ("in_use_bytes", ctypes.c_size_t),
                ("peak_in_use_bytes", ctypes.c_size_t), ("queued", ctypes.c_int64),
                ("running", ctypes.c_int32), ("peak_running", ctypes.c_int32),
                ("completed", ctypes.c_int64), ("now", ctypes.c_double)]


_lib = None
_lock = threading.Lock()


def load():
    """Loads libspca.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1212_4137_amd.build` (no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        P, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.spca_last_error.restype = ctypes.c_char_p
        lib.spca_last_error.argtypes = []
        lib.spca_ctx_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, ctypes.c_size_t]
        lib.spca_ctx_create.restype = ctypes.c_int
        lib.spca_ctx_destroy.argtypes = [P]
        lib.spca_ctx_destroy.restype = ctypes.c_int
        lib.spca_workspace_bytes.argtypes = [i64, i64, i32, ctypes.c_int]
        lib.spca_workspace_bytes.restype = ctypes.c_size_t
        lib.spca_am_solve.argtypes = [P, i64, i64, i64, ctypes.c_int, d, P, i32, d, i32,
                                      P, P, ctypes.POINTER(Result)]
        lib.spca_am_solve.restype = ctypes.c_int
        lib.spca_am_solve_ex.argtypes = [P, P, ctypes.POINTER(Problem),
                                         ctypes.POINTER(SolveOpts), ctypes.POINTER(Outputs)]
        lib.spca_am_solve_ex.restype = ctypes.c_int
        lib.spca_am_solve_group.argtypes = [P, P, i32, ctypes.POINTER(Problem),
                                            ctypes.POINTER(SolveOpts), ctypes.POINTER(Outputs)]
        lib.spca_am_solve_group.restype = ctypes.c_int
        lib.spca_group_workspace_bytes.argtypes = [i32, ctypes.POINTER(Problem),
                                                   ctypes.POINTER(SolveOpts)]
        lib.spca_group_workspace_bytes.restype = ctypes.c_size_t
        lib.spca_server_set_group_limit.argtypes = [P, i32]
        lib.spca_server_set_group_limit.restype = ctypes.c_int
        lib.spca_gemm_nt_f32.argtypes = [P, P, i64, P, i64, P, i64, i64, i64, i64]
        lib.spca_gemm_nt_f32.restype = ctypes.c_int
        lib.spca_gemm_nt_bf16.argtypes = [P, P, i64, P, i64, P, i64, i64, i64, i64]
        lib.spca_gemm_nt_bf16.restype = ctypes.c_int
        lib.spca_generate_spiked.argtypes = [P, ctypes.c_uint64, i64, i64, P, i64, i32,
                                             P, P, i64, P, i64]
        lib.spca_generate_spiked.restype = ctypes.c_int
        lib.spca_gemm_nt_f32_shape.argtypes = [P, P, i64, P, i64, P, i64, i64, i64, i64,
                                               ctypes.c_int, ctypes.c_int]
        lib.spca_gemm_nt_f32_shape.restype = ctypes.c_int
        lib.spca_gemm_nt_bf16_shape.argtypes = [P, P, i64, P, i64, P, i64, i64, i64, i64,
                                                ctypes.c_int, ctypes.c_int]
        lib.spca_gemm_nt_bf16_shape.restype = ctypes.c_int
        lib.spca_gemm_nt_f32_plan.argtypes = [i64, i64, i64, ctypes.c_int,
                                              ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_int)]
        lib.spca_gemm_nt_f32_plan.restype = ctypes.c_int
        lib.spca_x_update.argtypes = [P, ctypes.c_int, P, i64, i64, i64, d, P, i64, P, P]
        lib.spca_x_update.restype = ctypes.c_int
        lib.spca_x_update_noalloc.argtypes = [P, ctypes.c_int, P, i64, i64, i64, d, P, i64,
                                              P, P]
        lib.spca_x_update_noalloc.restype = ctypes.c_int
        lib.spca_tune_table_export.argtypes = [ctypes.c_char_p, ctypes.c_size_t,
                                               ctypes.POINTER(ctypes.c_size_t)]
        lib.spca_tune_table_export.restype = ctypes.c_int
        lib.spca_tune_table_import.argtypes = [ctypes.c_char_p]
        lib.spca_tune_table_import.restype = ctypes.c_int
        lib.spca_tune_table_clear.argtypes = []
        lib.spca_tune_table_clear.restype = ctypes.c_int
        lib.spca_am_solve_sparse.argtypes = [P, P, ctypes.POINTER(SparseProblem),
                                             ctypes.POINTER(SolveOpts),
                                             ctypes.POINTER(Outputs)]
        lib.spca_am_solve_sparse.restype = ctypes.c_int
        lib.spca_am_components.argtypes = [P, P, ctypes.POINTER(Problem),
                                           ctypes.POINTER(SolveOpts), i32, P,
                                           ctypes.POINTER(Result)]
        lib.spca_am_components.restype = ctypes.c_int
        lib.spca_am_components_sparse.argtypes = [P, P, ctypes.POINTER(SparseProblem),
                                                  ctypes.POINTER(SolveOpts), i32, P,
                                                  ctypes.POINTER(Result)]
        lib.spca_am_components_sparse.restype = ctypes.c_int
        lib.spca_ctx_set_workspace.argtypes = [P, P, ctypes.c_size_t]
        lib.spca_ctx_set_workspace.restype = ctypes.c_int
        lib.spca_request_footprint.argtypes = [ctypes.POINTER(Request)]
        lib.spca_request_footprint.restype = ctypes.c_size_t
        lib.spca_server_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, ctypes.c_size_t,
                                           i32]
        lib.spca_server_create.restype = ctypes.c_int
        lib.spca_server_submit.argtypes = [P, ctypes.POINTER(Request),
                                           ctypes.POINTER(ctypes.c_int64)]
        lib.spca_server_submit.restype = ctypes.c_int
        lib.spca_server_poll.argtypes = [P, ctypes.POINTER(Completion), i32,
                                         ctypes.POINTER(i32), i32]
        lib.spca_server_poll.restype = ctypes.c_int
        lib.spca_server_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
        lib.spca_server_stats.restype = ctypes.c_int
        lib.spca_server_destroy.argtypes = [P]
        lib.spca_server_destroy.restype = ctypes.c_int
        _lib = lib
        return lib


def _check(code):
    if code != SPCA_OK:
        raise SpcaError(code, load().spca_last_error().decode())


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _require_gpu_tensor(t, name, dtype=None):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")


def _stream_ptr(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """An ``spca_ctx``: device binding, workspace and HBM budget."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.spca_ctx_create(ctypes.byref(h), int(device), int(hbm_budget_bytes)))
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            load().spca_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def default_context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def workspace_bytes(n, p, r, precision=PREC_FP32):
    return int(load().spca_workspace_bytes(int(n), int(p), int(r), int(precision)))


def colmajor_view(A):
    """(n, p, lda) of a torch tensor holding A column-major: shape (n, p) with
    strides (1, lda)."""
    n, p = A.shape
    if A.stride(0) != 1 or (p > 1 and A.stride(1) < n):
        raise ValueError("A must be column-major: shape (n, p), strides (1, lda>=n)")
    lda = A.stride(1) if p > 1 else max(n, 1)
    return n, p, lda


def am_solve(A, formulation, s_or_gamma, X0=None, tol=1e-8, maxit=200, *,
             precision=PREC_FP32, polish_maxit=0, check_every=8, flags=0,
             ctx=None, stream=None, return_X=False, kernel_times=False, slots=None,
             warmup_iters=0, target_nnz=0):
    """Batched AM solve (``spca_am_solve_ex``).

    slots: run the rows of X0 through this many slots with on-the-fly
        replacement (``total_starts`` = rows of X0); None runs them all at once.
    warmup_iters, target_nnz: the sparsity-targeted warm-up of lambda / gamma.

    A : torch.float32 GPU tensor (n, p), column-major (strides (1, lda)).
    precision: PREC_FP32 / PREC_BF16_POLISH, or "fp32" / "bf16".
    X0: torch.float32 GPU tensor (r, p), contiguous, one start per row; or
        None for the single start e_i at the column of largest norm.
    Returns a dict of host (numpy) results.
    """
    import torch

    if isinstance(precision, str):
        precision = {"fp32": PREC_FP32, "bf16": PREC_BF16_POLISH}[precision]
    _require_gpu_tensor(A, "A", torch.float32)
    n, p, lda = colmajor_view(A)
    if X0 is not None:
        _require_gpu_tensor(X0, "X0", torch.float32)
        if X0.dim() != 2 or X0.shape[1] != p or not X0.is_contiguous():
            raise ValueError("X0 must be a contiguous (r, p) tensor")
        r = X0.shape[0]
    else:
        r = 1
    total = r
    if slots is not None and slots < r:
        r = int(slots)
    ctx = ctx or default_context(A.device.index or 0)
    x = np.zeros(p, dtype=np.float64)
    sup = np.zeros(p, dtype=np.int32)
    res = Result()
    f = np.zeros(total)
    ev = np.zeros(total)
    phi = np.zeros(total)
    iters = np.zeros(total, dtype=np.int32)
    status = np.zeros(total, dtype=np.int32)
    nnz = np.zeros(total, dtype=np.int32)
    Xf = torch.empty((total, p), dtype=torch.float32, device=A.device) if return_X else None
    kt = np.zeros(12) if kernel_times else None
    prob = Problem(A.data_ptr(), n, p, lda, int(formulation), float(s_or_gamma))
    opts = SolveOpts(X0.data_ptr() if X0 is not None else None, r, float(tol), int(maxit),
                     int(precision), int(polish_maxit), int(check_every), int(flags),
                     int(total if total > r else 0), int(warmup_iters), int(target_nnz))
    par = np.zeros(total)
    out = Outputs(_np_ptr(x), _np_ptr(sup), ctypes.pointer(res), _np_ptr(f), _np_ptr(ev),
                  _np_ptr(phi), _np_ptr(iters), _np_ptr(status), _np_ptr(nnz),
                  Xf.data_ptr() if Xf is not None else None, _np_ptr(kt), _np_ptr(par))
    _check(load().spca_am_solve_ex(ctx.handle, _stream_ptr(stream), ctypes.byref(prob),
                                   ctypes.byref(opts), ctypes.byref(out)))
    return {"x": x, "support": sup[: res.nnz].copy(), "objective": res.objective,
            "explained_variance": res.explained_var, "phi": res.phi,
            "best_start": res.best_start, "nnz": res.nnz, "iters": res.iters,
            "status": res.status, "warning": res.warning, "iters_x_starts": res.iters_x_starts,
            "objective_pre_polish": res.objective_pre_polish,
            "polish_iters": res.polish_iters,
            "f_per_start": f, "ev_per_start": ev, "phi_per_start": phi,
            "iters_per_start": iters, "status_per_start": status,
            "nnz_per_start": nnz, "X_final": Xf, "param_per_start": par,
            "kernel_times": None if kt is None else {
                "aty_ms": kt[0], "aty_launches": int(kt[1]), "x_update_ms": kt[2],
                "x_update_launches": int(kt[3]), "ax_dense_ms": kt[4],
                "ax_dense_launches": int(kt[5]), "iters_dense": int(kt[6]),
                "iters_list": int(kt[7]), "iters_union": int(kt[8]),
                "iters_list_rows": int(kt[9]), "active_starts_sum": float(kt[10]),
                "ax_nnz_sum": float(kt[11])}}


def _group_args(requests):
    import torch

    count = len(requests)
    probs = (Problem * count)()
    opts = (SolveOpts * count)()
    for q, rq in enumerate(requests):
        A, X0 = rq["A"], rq.get("X0")
        _require_gpu_tensor(A, "A", torch.float32)
        n, p, lda = colmajor_view(A)
        if X0 is not None:
            _require_gpu_tensor(X0, "X0", torch.float32)
            if X0.dim() != 2 or X0.shape[1] != p or not X0.is_contiguous():
                raise ValueError("X0 must be a contiguous (r, p) tensor")
        r = 1 if X0 is None else X0.shape[0]
        probs[q] = Problem(A.data_ptr(), n, p, lda, int(rq["formulation"]),
                           float(rq["s_or_gamma"]))
        opts[q] = SolveOpts(X0.data_ptr() if X0 is not None else None, r,
                            float(rq.get("tol", 1e-8)), int(rq.get("maxit", 200)), PREC_FP32, 0,
                            int(rq.get("check_every", 8)), 0, 0, 0, 0)
    return probs, opts


def group_workspace_bytes(requests):
    probs, opts = _group_args(requests)
    return int(load().spca_group_workspace_bytes(len(requests), probs, opts))


def am_solve_group(requests, *, ctx=None, stream=None, return_X=False):
    """Grouped solve (``spca_am_solve_group``): the requests iterate together,
    every launch of an iteration covering all of them.

    requests: list of dicts with A (column-major float32 GPU tensor), X0
        ((r, p) float32 GPU tensor or None for r = 1), formulation,
        s_or_gamma and optionally tol, maxit, check_every.
    Returns one result dict per request (the keys of ``am_solve``)."""
    import torch

    count = len(requests)
    probs, opts = _group_args(requests)
    outs = (Outputs * count)()
    keep = []
    for q, rq in enumerate(requests):
        p, r = probs[q].p, opts[q].r
        d = {"x": np.zeros(p), "sup": np.zeros(p, dtype=np.int32), "res": Result(),
             "f": np.zeros(r), "ev": np.zeros(r), "phi": np.zeros(r),
             "iters": np.zeros(r, dtype=np.int32), "status": np.zeros(r, dtype=np.int32),
             "nnz": np.zeros(r, dtype=np.int32),
             "Xf": torch.empty((r, p), dtype=torch.float32, device=rq["A"].device)
             if return_X else None}
        keep.append(d)
        outs[q] = Outputs(_np_ptr(d["x"]), _np_ptr(d["sup"]), ctypes.pointer(d["res"]),
                          _np_ptr(d["f"]), _np_ptr(d["ev"]), _np_ptr(d["phi"]),
                          _np_ptr(d["iters"]), _np_ptr(d["status"]), _np_ptr(d["nnz"]),
                          d["Xf"].data_ptr() if d["Xf"] is not None else None, None, None)
    ctx = ctx or default_context(requests[0]["A"].device.index or 0)
    _check(load().spca_am_solve_group(ctx.handle, _stream_ptr(stream), count, probs, opts, outs))
    results = []
    for d in keep:
        res = d["res"]
        results.append({
            "x": d["x"], "support": d["sup"][: res.nnz].copy(), "objective": res.objective,
            "explained_variance": res.explained_var, "phi": res.phi,
            "best_start": res.best_start, "nnz": res.nnz, "iters": res.iters,
            "status": res.status, "warning": res.warning,
            "iters_x_starts": res.iters_x_starts, "f_per_start": d["f"],
            "ev_per_start": d["ev"], "phi_per_start": d["phi"],
            "iters_per_start": d["iters"], "status_per_start": d["status"],
            "nnz_per_start": d["nnz"], "X_final": d["Xf"]})
    return results


def am_solve_simple(A, formulation, s_or_gamma, X0=None, tol=1e-8, maxit=200):
    """The one-call entry point ``spca_am_solve`` (default context, null
    stream)."""
    import torch

    _require_gpu_tensor(A, "A", torch.float32)
    n, p, lda = colmajor_view(A)
    r = 1 if X0 is None else X0.shape[0]
    x = np.zeros(p, dtype=np.float64)
    sup = np.zeros(p, dtype=np.int32)
    res = Result()
    torch.cuda.synchronize()
    _check(load().spca_am_solve(ctypes.c_void_p(A.data_ptr()), n, p, lda, int(formulation),
                                float(s_or_gamma),
                                ctypes.c_void_p(X0.data_ptr()) if X0 is not None else None,
                                r, float(tol), int(maxit), _np_ptr(x), _np_ptr(sup),
                                ctypes.byref(res)))
    return {"x": x, "support": sup[: res.nnz].copy(), "objective": res.objective,
            "explained_variance": res.explained_var, "best_start": res.best_start,
            "nnz": res.nnz, "iters": res.iters, "status": res.status, "warning": res.warning}


def gemm_nt(P, Q, stream=None):
    """C = P Q^T on the MFMA kernel (``spca_gemm_nt_f32``)."""
    import torch

    _require_gpu_tensor(P, "P", torch.float32)
    _require_gpu_tensor(Q, "Q", torch.float32)
    M, K = P.shape
    N, K2 = Q.shape
    if K2 != K:
        raise ValueError("inner dimensions differ")
    if P.stride(1) != 1 or Q.stride(1) != 1:
        raise ValueError("P and Q must be row-major")
    C = torch.empty((M, N), dtype=torch.float32, device=P.device)
    _check(load().spca_gemm_nt_f32(_stream_ptr(stream), ctypes.c_void_p(P.data_ptr()),
                                   P.stride(0), ctypes.c_void_p(Q.data_ptr()), Q.stride(0),
                                   ctypes.c_void_p(C.data_ptr()), N, M, N, K))
    return C


def generate_spiked(seed, n, p, thetas=(), U=None, V=None, lda=None, device="cuda:0",
                    stream=None):
    """Device-generated spiked matrix (``spca_generate_spiked``) as a
    column-major (n, p) float32 tensor.  U (n x k) and V (p x k) are host
    float64 arrays of the spike directions."""
    import torch

    lda = lda or n
    buf = torch.empty((p, lda), dtype=torch.float32, device=device)
    k = len(thetas)
    th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64))
    Ud = Vd = None
    if k:
        Ud = torch.from_numpy(np.asfortranarray(U, dtype=np.float64).T.copy()).to(device)
        Vd = torch.from_numpy(np.asfortranarray(V, dtype=np.float64).T.copy()).to(device)
    _check(load().spca_generate_spiked(_stream_ptr(stream), int(seed), n, p,
                                       ctypes.c_void_p(buf.data_ptr()), lda, k,
                                       _np_ptr(th) if k else None,
                                       ctypes.c_void_p(Ud.data_ptr()) if k else None, n,
                                       ctypes.c_void_p(Vd.data_ptr()) if k else None, p))
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    return buf[:, :n].t()


def gemm_nt_bf16(P, Q, stream=None):
    """C = P Q^T from BF16 operands with FP32 accumulation
    (``spca_gemm_nt_bf16``); P and Q are torch.bfloat16 row-major tensors
    whose leading dimensions are multiples of 8."""
    import torch

    _require_gpu_tensor(P, "P", torch.bfloat16)
    _require_gpu_tensor(Q, "Q", torch.bfloat16)
    M, K = P.shape
    N, K2 = Q.shape
    if K2 != K:
        raise ValueError("inner dimensions differ")
    C = torch.empty((M, N), dtype=torch.float32, device=P.device)
    _check(load().spca_gemm_nt_bf16(_stream_ptr(stream), ctypes.c_void_p(P.data_ptr()),
                                    P.stride(0), ctypes.c_void_p(Q.data_ptr()), Q.stride(0),
                                    ctypes.c_void_p(C.data_ptr()), N, M, N, K))
    return C


def gemm_nt_shape(P, Q, shape, splits=1, stream=None):
    """Partial products of P Q^T with a forced tile shape and K split
    (``spca_gemm_nt_f32_shape``, or ``spca_gemm_nt_bf16_shape`` for
    torch.bfloat16 operands); returns a (splits, M, N) tensor whose sum over
    the first axis is the product."""
    import torch

    if P.dtype == torch.bfloat16:
        _require_gpu_tensor(Q, "Q", torch.bfloat16)
        M, K = P.shape
        N, _ = Q.shape
        C = torch.empty((splits, M, N), dtype=torch.float32, device=P.device)
        _check(load().spca_gemm_nt_bf16_shape(
            _stream_ptr(stream), ctypes.c_void_p(P.data_ptr()), P.stride(0),
            ctypes.c_void_p(Q.data_ptr()), Q.stride(0), ctypes.c_void_p(C.data_ptr()), N,
            M, N, K, int(shape), int(splits)))
        return C
    _require_gpu_tensor(P, "P", torch.float32)
    _require_gpu_tensor(Q, "Q", torch.float32)
    M, K = P.shape
    N, _ = Q.shape
    C = torch.empty((splits, M, N), dtype=torch.float32, device=P.device)
    _check(load().spca_gemm_nt_f32_shape(_stream_ptr(stream), ctypes.c_void_p(P.data_ptr()),
                                         P.stride(0), ctypes.c_void_p(Q.data_ptr()),
                                         Q.stride(0), ctypes.c_void_p(C.data_ptr()), N,
                                         M, N, K, int(shape), int(splits)))
    return C


def gemm_plan(M, N, K, max_splits=1):
    """(shape, splits) the library picks for an M x N x K product."""
    sh, sp = ctypes.c_int(), ctypes.c_int()
    _check(load().spca_gemm_nt_f32_plan(int(M), int(N), int(K), int(max_splits),
                                        ctypes.byref(sh), ctypes.byref(sp)))
    return sh.value, sp.value


def x_update(formulation, V, s_or_gamma, stream=None, out=None, noalloc=False):
    """The x-update operator on each row of V (``spca_x_update``, or
    ``spca_x_update_noalloc`` with noalloc=True); returns (X, phi, nnz) as
    GPU tensors, written into ``out`` when given."""
    import torch

    _require_gpu_tensor(V, "V", torch.float32)
    r, p = V.shape
    if V.stride(1) != 1:
        raise ValueError("V must be row-major")
    if out is None:
        X = torch.empty((r, p), dtype=torch.float32, device=V.device)
        phi = torch.empty(r, dtype=torch.float64, device=V.device)
        nnz = torch.empty(r, dtype=torch.int32, device=V.device)
    else:
        X, phi, nnz = out
        if (X.shape != (r, p) or X.dtype != torch.float32 or not X.is_contiguous()
                or phi.dtype != torch.float64 or phi.numel() < r
                or nnz.dtype != torch.int32 or nnz.numel() < r):
            raise ValueError("out must be (X (r, p) float32, phi float64 >= r, nnz int32 >= r)")
    fn = load().spca_x_update_noalloc if noalloc else load().spca_x_update
    _check(fn(_stream_ptr(stream), int(formulation),
                                ctypes.c_void_p(V.data_ptr()), V.stride(0), r, p,
                                float(s_or_gamma), ctypes.c_void_p(X.data_ptr()), p,
                                ctypes.c_void_p(phi.data_ptr()),
                                ctypes.c_void_p(nnz.data_ptr())))
    return X, phi, nnz


def _request(spec):
    """spca_request from a dict; returns (Request, arrays to keep alive)."""
    keep = []
    q = Request()
    A = spec.get("A")
    if A is not None:
        n, p, lda = colmajor_view(A)
        q.A, q.n, q.p, q.lda = A.data_ptr(), n, p, lda
        keep.append(A)
    else:
        q.n, q.p = int(spec["n"]), int(spec["p"])
        q.seed = int(spec.get("seed", 0))
        thetas = np.ascontiguousarray(spec.get("thetas", ()), dtype=np.float64)
        q.k = len(thetas)
        if q.k:
            U = np.asfortranarray(spec["U"], dtype=np.float64)
            V = np.asfortranarray(spec["V"], dtype=np.float64)
            if U.shape != (q.n, q.k) or V.shape != (q.p, q.k):
                raise ValueError("U must be (n, k) and V (p, k)")
            keep += [thetas, U, V]
            q.thetas, q.U, q.V = _np_ptr(thetas), _np_ptr(U), _np_ptr(V)
    q.start_seed = int(spec.get("start_seed", 1))
    q.formulation = int(spec["formulation"])
    q.s_or_gamma = float(spec.get("s_or_gamma", 0.0))
    q.gamma_rel = float(spec.get("gamma_rel", 0.0))
    q.r = int(spec.get("r", 16))
    q.maxit = int(spec.get("maxit", 200))
    q.tol = float(spec.get("tol", 1e-6))
    prec = spec.get("precision", PREC_FP32)
    q.precision = {"fp32": PREC_FP32, "bf16": PREC_BF16_POLISH}.get(prec, prec)
    q.polish_maxit = int(spec.get("polish_maxit", q.maxit))
    q.check_every = int(spec.get("check_every", 8))
    q.flags = int(spec.get("flags", 0))
    if spec.get("want_x", False):
        x = np.zeros(q.p, dtype=np.float64)
        sup = np.zeros(q.p, dtype=np.int32)
        keep += [x, sup]
        q.x_out, q.support_out = _np_ptr(x), _np_ptr(sup)
    return q, keep


def request_footprint(spec):
    """Bytes of server memory the request holds while it runs."""
    q, _ = _request(spec)
    return int(load().spca_request_footprint(ctypes.byref(q)))


class Server:
    """Continuous-batching request server (``spca_server_*``): an HBM arena
    of ``hbm_bytes`` and ``workers`` concurrent solves.  ``submit`` takes a
    dict with the fields of spca_request (``want_x=True`` asks for x and
    the support); ``poll`` returns finished requests as dicts."""

    def __init__(self, hbm_bytes, workers=4, device=0, group_limit=None):
        self.handle = ctypes.c_void_p()
        _check(load().spca_server_create(ctypes.byref(self.handle), device,
                                         int(hbm_bytes), int(workers)))
        self._keep = {}
        if group_limit is not None:
            # 0: every request alone (spca_am_solve_ex); k: groups of <= k
            try:
                _check(load().spca_server_set_group_limit(self.handle, int(group_limit)))
            except Exception:
                self.close()
                raise

    def submit(self, spec):
        q, keep = _request(spec)
        rid = ctypes.c_int64()
        _check(load().spca_server_submit(self.handle, ctypes.byref(q), ctypes.byref(rid)))
        self._keep[rid.value] = (q, keep)
        return rid.value

    def poll(self, wait_ms=0, max_items=256):
        buf = (Completion * max_items)()
        cnt = ctypes.c_int32()
        _check(load().spca_server_poll(self.handle, buf, max_items, ctypes.byref(cnt),
                                       int(wait_ms)))
        out = []
        for c in buf[: cnt.value]:
            q, keep = self._keep.pop(c.id)
            d = {"id": c.id, "rc": c.rc, "error": c.error.decode(errors="replace"),
                 "objective": c.res.objective, "explained_variance": c.res.explained_var,
                 "objective_pre_polish": c.res.objective_pre_polish,
                 "nnz": c.res.nnz, "iters": c.res.iters, "status": c.res.status, "warning": c.res.warning,
                 "best_start": c.res.best_start, "iters_x_starts": c.res.iters_x_starts,
                 "polish_iters": c.res.polish_iters, "s_or_gamma": c.s_or_gamma,
                 "t_submit": c.t_submit, "t_admit": c.t_admit, "t_solve": c.t_solve,
                 "t_done": c.t_done,
                 "footprint": c.footprint}
            if q.x_out:
                x, sup = keep[-2], keep[-1]
                d["x"] = x
                d["support"] = sup[: c.res.nnz].copy()
            out.append(d)
        return out

    def stats(self):
        st = ServerStats()
        _check(load().spca_server_stats(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if self.handle:
            _check(load().spca_server_destroy(self.handle))
            self.handle = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def tune_table_export():
    """The tuning table as text (``spca_tune_table_export``)."""
    n = ctypes.c_size_t()
    _check(load().spca_tune_table_export(None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(load().spca_tune_table_export(buf, n.value + 1, ctypes.byref(n)))
    return buf.value.decode()


def tune_table_import(text):
    _check(load().spca_tune_table_import(text.encode()))


def tune_table_clear():
    _check(load().spca_tune_table_clear())


def am_components(A, formulation, s_or_gamma, X0, ncomp, tol=1e-8, maxit=200, *,
                  check_every=8, flags=0, ctx=None, stream=None, warmup_iters=0,
                  target_nnz=0):
    """Several components (``spca_am_components``): component c solves the
    problem on A deflated by the loadings of components 0..c-1, from the
    same starts.  Returns a list of dicts (objective, explained variance,
    best start, nnz, iterations, status, x, support)."""
    import torch

    _require_gpu_tensor(A, "A", torch.float32)
    n, p, lda = colmajor_view(A)
    _require_gpu_tensor(X0, "X0", torch.float32)
    if X0.dim() != 2 or X0.shape[1] != p or not X0.is_contiguous():
        raise ValueError("X0 must be a contiguous (r, p) tensor")
    r = X0.shape[0]
    ctx = ctx or default_context(A.device.index or 0)
    X = np.zeros((ncomp, p), dtype=np.float64)
    res = (Result * ncomp)()
    prob = Problem(A.data_ptr(), n, p, lda, int(formulation), float(s_or_gamma))
    opts = SolveOpts(X0.data_ptr(), r, float(tol), int(maxit), PREC_FP32, 0,
                     int(check_every), int(flags), 0, int(warmup_iters), int(target_nnz),
                     None, 0)
    _check(load().spca_am_components(ctx.handle, _stream_ptr(stream), ctypes.byref(prob),
                                     ctypes.byref(opts), int(ncomp), _np_ptr(X), res))
    out = []
    for c in range(ncomp):
        x = X[c]
        out.append({"objective": res[c].objective, "explained_variance": res[c].explained_var,
                    "best_start": res[c].best_start, "nnz": res[c].nnz,
                    "iters": res[c].iters, "status": res[c].status, "x": x.copy(),
                    "support": np.flatnonzero(x)})
    return out


def am_components_sparse(D, formulation, s_or_gamma, X0, ncomp, tol=1e-8, maxit=200, *,
                         check_every=8, flags=0, ctx=None, stream=None, warmup_iters=0,
                         target_nnz=0):
    """Several components on a sparse A (``spca_am_components_sparse``); D
    from sparse_to_device, X0 a contiguous (r, p) float32 GPU tensor.
    Returns the same list of dicts as am_components."""
    import torch

    n, p = D["n"], D["p"]
    _require_gpu_tensor(X0, "X0", torch.float32)
    if X0.dim() != 2 or X0.shape[1] != p or not X0.is_contiguous():
        raise ValueError("X0 must be a contiguous (r, p) tensor")
    r = X0.shape[0]
    ctx = ctx or default_context(X0.device.index or 0)
    X = np.zeros((ncomp, p), dtype=np.float64)
    res = (Result * ncomp)()
    prob = SparseProblem(n, p, D["col_ptr"].data_ptr(), D["row_idx"].data_ptr(),
                         D["col_val"].data_ptr(), D["row_ptr"].data_ptr(),
                         D["col_idx"].data_ptr(), D["row_val"].data_ptr(), int(formulation),
                         float(s_or_gamma))
    opts = SolveOpts(X0.data_ptr(), r, float(tol), int(maxit), PREC_FP32, 0,
                     int(check_every), int(flags), 0, int(warmup_iters), int(target_nnz),
                     None, 0)
    _check(load().spca_am_components_sparse(ctx.handle, _stream_ptr(stream),
                                            ctypes.byref(prob), ctypes.byref(opts),
                                            int(ncomp), _np_ptr(X), res))
    out = []
    for c in range(ncomp):
        x = X[c]
        out.append({"objective": res[c].objective, "explained_variance": res[c].explained_var,
                    "best_start": res[c].best_start, "nnz": res[c].nnz,
                    "iters": res[c].iters, "status": res[c].status, "x": x.copy(),
                    "support": np.flatnonzero(x)})
    return out


def sparse_to_device(mat, device="cuda:0"):
    """Device copies of a sparse matrix's two layouts (an object with n, p,
    col_ptr, row_idx, col_val, row_ptr, col_idx, row_val host arrays)."""
    import torch

    dev = {"n": int(mat.n), "p": int(mat.p)}
    for name, dt in (("col_ptr", np.int64), ("row_idx", np.int32), ("col_val", np.float32),
                     ("row_ptr", np.int64), ("col_idx", np.int32), ("row_val", np.float32)):
        dev[name] = torch.from_numpy(np.ascontiguousarray(getattr(mat, name), dtype=dt)).to(device)
    return dev


def am_solve_sparse(D, formulation, s_or_gamma, X0, tol=1e-8, maxit=200, *, check_every=8,
                    flags=0, ctx=None, stream=None, warmup_iters=0, target_nnz=0,
                    return_X=False, kernel_times=False):
    """Batched AM solve on a sparse A (``spca_am_solve_sparse``); D from
    sparse_to_device, X0 a contiguous (r, p) float32 GPU tensor."""
    import torch

    n, p = D["n"], D["p"]
    _require_gpu_tensor(X0, "X0", torch.float32)
    if X0.dim() != 2 or X0.shape[1] != p or not X0.is_contiguous():
        raise ValueError("X0 must be a contiguous (r, p) tensor")
    r = X0.shape[0]
    ctx = ctx or default_context(X0.device.index or 0)
    x = np.zeros(p, dtype=np.float64)
    sup = np.zeros(p, dtype=np.int32)
    res = Result()
    f, ev, phi = np.zeros(r), np.zeros(r), np.zeros(r)
    iters = np.zeros(r, dtype=np.int32)
    status = np.zeros(r, dtype=np.int32)
    nnz = np.zeros(r, dtype=np.int32)
    par = np.zeros(r)
    Xf = torch.empty((r, p), dtype=torch.float32, device=X0.device) if return_X else None
    prob = SparseProblem(n, p, D["col_ptr"].data_ptr(), D["row_idx"].data_ptr(),
                         D["col_val"].data_ptr(), D["row_ptr"].data_ptr(),
                         D["col_idx"].data_ptr(), D["row_val"].data_ptr(), int(formulation),
                         float(s_or_gamma))
    opts = SolveOpts(X0.data_ptr(), r, float(tol), int(maxit), PREC_FP32, 0, int(check_every),
                     int(flags), 0, int(warmup_iters), int(target_nnz), None, 0)
    kt = np.zeros(12) if kernel_times else None
    out = Outputs(_np_ptr(x), _np_ptr(sup), ctypes.pointer(res), _np_ptr(f), _np_ptr(ev),
                  _np_ptr(phi), _np_ptr(iters), _np_ptr(status), _np_ptr(nnz),
                  Xf.data_ptr() if Xf is not None else None,
                  _np_ptr(kt) if kt is not None else None, _np_ptr(par))
    _check(load().spca_am_solve_sparse(ctx.handle, _stream_ptr(stream), ctypes.byref(prob),
                                       ctypes.byref(opts), ctypes.byref(out)))
    return {"x": x, "support": sup[: res.nnz].copy(), "objective": res.objective,
            "explained_variance": res.explained_var, "best_start": res.best_start,
            "nnz": res.nnz, "iters": res.iters, "status": res.status, "warning": res.warning,
            "iters_x_starts": res.iters_x_starts, "f_per_start": f, "ev_per_start": ev,
            "iters_per_start": iters, "status_per_start": status, "nnz_per_start": nnz,
            "param_per_start": par, "X_final": Xf,
            "kernel_times": None if kt is None else {
                "aty_ms": kt[0], "aty_launches": int(kt[1]), "x_update_ms": kt[2],
                "x_update_launches": int(kt[3]), "ax_dense_ms": kt[4],
                "ax_dense_launches": int(kt[5]), "iters_dense": int(kt[6]),
                "iters_list": int(kt[7] - kt[9]), "iters_list_rows": int(kt[9]),
                "active_starts_sum": float(kt[10]), "ax_nnz_sum": float(kt[11])}}
