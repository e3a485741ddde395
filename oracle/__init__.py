"""FP64 CPU oracle for the AM sparse PCA method (arXiv:1212.4137).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline
leg of ``bench.py`` may call it; the product path never does.  The numerics
live in ``spca_oracle.c`` (plain C, FP64, no BLAS); this module is the ctypes
shim plus numpy conveniences.  It imports nothing from the GPU package.

Each function cites the passage of the paper it follows:
  * operators T_s, U_gamma, V_gamma, lambda_s -- Section 2.1 (definitions
    after Table 3) and Table 3 (rows S3-S6, optimal values phi(z*));
  * x_operator -- Algorithm 2, the four x-update branches;
  * objective -- Table 1, column f(x); explained variance as defined in
    Section 4.1 (||Ax||_2^2 for L2 variance, ||Ax||_1 for L1 variance);
  * am_single / am_multi -- Algorithm 2 with the stop test of Section 2.2,
    and the multi-start scheme of Section 4 (keep the largest objective).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

CONVERGED, MAXIT, DEGENERATE, ZERO = 0, 1, 2, 3

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build

        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    d = ctypes.c_double
    i64 = ctypes.c_int64
    i32 = ctypes.c_int32
    P = ctypes.c_void_p
    lib.orc_T_s.argtypes = [P, i64, i64, P]
    lib.orc_T_s.restype = d
    lib.orc_U_gamma.argtypes = [P, i64, d, P]
    lib.orc_U_gamma.restype = d
    lib.orc_V_gamma.argtypes = [P, i64, d, P]
    lib.orc_V_gamma.restype = d
    lib.orc_lambda_s.argtypes = [P, i64, d]
    lib.orc_lambda_s.restype = d
    lib.orc_V_lambda_s.argtypes = [P, i64, d, P]
    lib.orc_V_lambda_s.restype = d
    lib.orc_x_operator.argtypes = [ctypes.c_int, P, i64, d, P]
    lib.orc_x_operator.restype = d
    lib.orc_objective.argtypes = [ctypes.c_int, P, i64, i64, i64, P, d, P]
    lib.orc_objective.restype = d
    lib.orc_am_single.argtypes = [P, i64, i64, i64, ctypes.c_int, d, P, d, i32,
                                  P, P, P, P, P]
    lib.orc_am_single.restype = ctypes.c_int
    lib.orc_am_multi.argtypes = [P, i64, i64, i64, ctypes.c_int, d, P, i32, d,
                                 i32, ctypes.c_int, P, P, P, P, P, P]
    lib.orc_am_multi.restype = i32
    lib.orc_am_multi_warm.argtypes = [P, i64, i64, i64, ctypes.c_int, d, i64, i32, P, i32,
                                      d, i32, ctypes.c_int, P, P, P, P, P, P]
    lib.orc_am_multi_warm.restype = i32
    lib.orc_am_multi_csc.argtypes = [P, P, P, i64, i64, ctypes.c_int, d, P, i32, d, i32,
                                     ctypes.c_int, P, P, P, P, P]
    lib.orc_am_multi_csc.restype = i32
    lib.orc_deflate.argtypes = [P, i64, i64, i64, P, P, i64]
    lib.orc_deflate.restype = None
    lib.orc_max_norm_column.argtypes = [P, i64, i64, i64]
    lib.orc_max_norm_column.restype = i64
    _lib = lib
    return lib


def _vec(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _colmajor(A):
    """FP64 Fortran-ordered copy of A (n x p) and its leading dimension."""
    A64 = np.asfortranarray(np.asarray(A, dtype=np.float64))
    return A64, A64.shape[0]


# -- operators (Section 2.1, Table 3) ---------------------------------------

def T_s(a, s):
    """T_s(a) and ||T_s(a)||_2 (Table 3, S3); ties go to the lower index."""
    a = _vec(a)
    out = np.zeros_like(a)
    phi = _load().orc_T_s(_ptr(a), a.size, int(s), _ptr(out))
    return out, phi


def U_gamma(a, gamma):
    """U_gamma(a) and the S5 optimum sum over kept i of (a_i^2 - gamma)."""
    a = _vec(a)
    out = np.zeros_like(a)
    phi = _load().orc_U_gamma(_ptr(a), a.size, float(gamma), _ptr(out))
    return out, phi


def V_gamma(a, gamma):
    """V_gamma(a) (soft threshold) and the S6 optimum ||V_gamma(a)||_2."""
    a = _vec(a)
    out = np.zeros_like(a)
    phi = _load().orc_V_gamma(_ptr(a), a.size, float(gamma), _ptr(out))
    return out, phi


def lambda_s(a, s):
    """lambda_s(a) = argmin_{l >= 0} l sqrt(s) + ||V_l(a)||_2, exactly."""
    a = _vec(a)
    return _load().orc_lambda_s(_ptr(a), a.size, float(s))


def V_lambda_s(a, s):
    """V_{lambda_s(a)}(a) and the S4 optimum lambda sqrt(s) + ||V||_2."""
    a = _vec(a)
    out = np.zeros_like(a)
    phi = _load().orc_V_lambda_s(_ptr(a), a.size, float(s), _ptr(out))
    return out, phi


def x_operator(fid, v, s_or_gamma):
    """The x-update operator of Algorithm 2 for formulation ``fid``."""
    v = _vec(v)
    w = np.zeros_like(v)
    phi = _load().orc_x_operator(int(fid), _ptr(v), v.size, float(s_or_gamma),
                                 _ptr(w))
    return w, phi


# -- objective and Algorithm 2 ----------------------------------------------

def objective(fid, A, x, s_or_gamma):
    """(f(x) of Table 1, explained variance) in FP64."""
    A64, lda = _colmajor(A)
    n, p = A64.shape
    x = _vec(x)
    ev = ctypes.c_double()
    f = _load().orc_objective(int(fid), _ptr(A64), n, p, lda, _ptr(x),
                              float(s_or_gamma), ctypes.byref(ev))
    return f, ev.value


def am_single(A, fid, s_or_gamma, x0, tol, maxit):
    """Algorithm 2 from one start; returns a dict with x, phi trace, etc."""
    A64, lda = _colmajor(A)
    n, p = A64.shape
    x0 = _vec(x0)
    x = np.zeros(p)
    trace = np.zeros(max(int(maxit), 1))
    it = ctypes.c_int32()
    f = ctypes.c_double()
    ev = ctypes.c_double()
    st = _load().orc_am_single(_ptr(A64), n, p, lda, int(fid), float(s_or_gamma),
                               _ptr(x0), float(tol), int(maxit), _ptr(x),
                               _ptr(trace), ctypes.byref(it), ctypes.byref(f),
                               ctypes.byref(ev))
    return {"x": x, "phi_trace": trace[: it.value].copy(), "iters": it.value,
            "f": f.value, "ev": ev.value, "status": st}


def am_multi(A, fid, s_or_gamma, X0, tol, maxit, nthreads=1, want_x=True):
    """Multi-start AM (Section 4): every row of X0 is a start.

    Returns a dict with the best start index, per-start f, EV, final phi,
    iteration count and status, and (if ``want_x``) all final x (r x p).
    """
    A64, lda = _colmajor(A)
    n, p = A64.shape
    X0 = np.ascontiguousarray(np.asarray(X0, dtype=np.float64))
    if X0.ndim == 1:
        X0 = X0[None, :]
    r = X0.shape[0]
    assert X0.shape[1] == p
    X = np.zeros((r, p)) if want_x else None
    f = np.zeros(r)
    ev = np.zeros(r)
    phi = np.zeros(r)
    iters = np.zeros(r, dtype=np.int32)
    status = np.zeros(r, dtype=np.int32)
    best = _load().orc_am_multi(_ptr(A64), n, p, lda, int(fid), float(s_or_gamma),
                                _ptr(X0), r, float(tol), int(maxit), int(nthreads),
                                _ptr(X) if want_x else None, _ptr(f), _ptr(ev),
                                _ptr(phi), _ptr(iters), _ptr(status))
    return {"best": int(best), "X": X, "f": f, "ev": ev, "phi": phi,
            "iters": iters, "status": status}


def am_multi_warm(A, fid, s_or_gamma, X0, tol, maxit, warm_iters, target_s=0,
                  nthreads=1):
    """Multi-start AM with the sparsity-targeted warm-up of Section 4.1:
    the parameter (lambda for the L1 constraint, gamma for the penalties,
    targeting target_s nonzeros) follows v for warm_iters x-updates and is
    frozen afterwards.  The best start has the largest explained variance.
    Returns the best start, per-start f, EV, final parameter, iterations,
    status and final x (r x p)."""
    A64, lda = _colmajor(A)
    n, p = A64.shape
    X0 = np.ascontiguousarray(np.asarray(X0, dtype=np.float64))
    if X0.ndim == 1:
        X0 = X0[None, :]
    r = X0.shape[0]
    assert X0.shape[1] == p
    X = np.zeros((r, p))
    f = np.zeros(r)
    ev = np.zeros(r)
    par = np.zeros(r)
    iters = np.zeros(r, dtype=np.int32)
    status = np.zeros(r, dtype=np.int32)
    best = _load().orc_am_multi_warm(_ptr(A64), n, p, lda, int(fid), float(s_or_gamma),
                                     int(target_s), int(warm_iters), _ptr(X0), r, float(tol),
                                     int(maxit), int(nthreads), _ptr(X), _ptr(f), _ptr(ev),
                                     _ptr(par), _ptr(iters), _ptr(status))
    return {"best": int(best), "X": X, "f": f, "ev": ev, "param": par, "iters": iters,
            "status": status}


def am_multi_csc(col_ptr, row_idx, val, n, p, fid, s_or_gamma, X0, tol, maxit,
                 nthreads=1):
    """Multi-start AM on a sparse A in compressed sparse columns (int64
    col_ptr of length p + 1, int32 row indices, values as FP64)."""
    cp = np.ascontiguousarray(col_ptr, dtype=np.int64)
    ri = np.ascontiguousarray(row_idx, dtype=np.int32)
    vv = np.ascontiguousarray(val, dtype=np.float64)
    assert cp.shape == (p + 1,) and ri.shape == vv.shape == (cp[-1],)
    X0 = np.ascontiguousarray(np.asarray(X0, dtype=np.float64))
    if X0.ndim == 1:
        X0 = X0[None, :]
    r = X0.shape[0]
    X = np.zeros((r, p))
    f = np.zeros(r)
    ev = np.zeros(r)
    iters = np.zeros(r, dtype=np.int32)
    status = np.zeros(r, dtype=np.int32)
    best = _load().orc_am_multi_csc(_ptr(cp), _ptr(ri), _ptr(vv), int(n), int(p), int(fid),
                                    float(s_or_gamma), _ptr(X0), r, float(tol), int(maxit),
                                    int(nthreads), _ptr(X), _ptr(f), _ptr(ev), _ptr(iters),
                                    _ptr(status))
    return {"best": int(best), "X": X, "f": f, "ev": ev, "iters": iters, "status": status}


def deflate(A, x):
    """A (I - x x^T) for a unit loading x (projection deflation)."""
    A64, lda = _colmajor(A)
    n, p = A64.shape
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    out = np.zeros((p, n)).T  # column-major n x p
    _load().orc_deflate(_ptr(A64), n, p, lda, _ptr(x), _ptr(out), n)
    return out


def am_components(A, fid, s_or_gamma, X0, ncomp, tol, maxit, nthreads=1):
    """Several sparse loadings: component t is the multi-start AM solution
    on A deflated by the loadings found before it (projection deflation),
    from the same starts.  Returns per component the best start, f and
    explained variance on its deflated matrix, and the loading."""
    At = np.asfortranarray(np.asarray(A, dtype=np.float64))
    comps = []
    for _ in range(ncomp):
        res = am_multi(At, fid, s_or_gamma, X0, tol, maxit, nthreads=nthreads)
        b = res["best"]
        x = res["X"][b].copy()
        comps.append({"best": b, "f": res["f"][b], "ev": res["ev"][b], "x": x,
                      "f_all": res["f"]})
        if np.any(x):
            At = deflate(At, x)
    return comps


def max_norm_column(A):
    """argmax_i ||a_i||_2 (ties to the lowest i)."""
    A64, lda = _colmajor(A)
    n, p = A64.shape
    return int(_load().orc_max_norm_column(_ptr(A64), n, p, lda))


def unit_vector_start(A):
    """x0 = e_{i*} with i* the column of largest norm (start of the small
    single-start workload: y0 is then that column, normalised)."""
    p = np.asarray(A).shape[1]
    x0 = np.zeros(p)
    x0[max_norm_column(A)] = 1.0
    return x0
