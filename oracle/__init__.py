"""FP64 CPU oracle for similarity-based fuzzy clustering (test infrastructure).

This package is the slow, independent reference the HIP path is checked
against.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import it; the library itself never does, and the two share no
code.  Every function here is a thin ctypes wrapper over ``fcref.c`` (plain C,
IEEE double), which computes what the paper's formulas and algorithms define:

* ``x_s``               -- the products X s_i of eq. (gradient_column), section 3
* ``share``             -- share = X X^T, Alg. 2
* ``project_simplex``   -- the Euclidean projection onto the simplex (section 2),
                           from its optimality conditions (the result Alg. 1 computes)
* ``loss``              -- the structured loss of Alg. 3
* ``gradient``          -- eq. (gradient_column), column by column
* ``spectral_norm``     -- power iteration for ||S||_2 (Theorem 3.1's bound)
* ``solve``             -- parallel GPA (Alg. 2/3) or parallel FISTA (Alg. 4),
                           with a constant step, a step schedule, or
                           backtracking on L

Layout: the paper's C x N matrix X with column x_i stored contiguously, i.e. a
row-major ``(N, C)`` numpy array whose row i is x_i.  S is symmetric CSR
(``row_ptr`` int64, ``col_idx`` int32, ``val`` float64).  ``diag_unit=True``
means the similarity is S + I with no diagonal stored (the paper's
adjacency-plus-ones convention).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fcref.c")
_LIB_PATH = os.path.join(_HERE, "libfcref.so")
_lib = None

STOP_MAXITER, STOP_LOSS, STOP_PGRAD, STOP_STEP = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile fcref.c into oracle/libfcref.so with gcc and OpenMP."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-std=c99", "-Wall", "-shared", "-fPIC",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Opts(ctypes.Structure):
    _fields_ = [
        ("accelerate", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("backtrack", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("step", ctypes.c_double),
        ("L0", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("tol_loss", ctypes.c_double),
        ("tol_pgrad", ctypes.c_double),
        ("step_schedule", ctypes.POINTER(ctypes.c_double)),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.fcref_num_threads.restype = ctypes.c_int
        lib.fcref_norm_s_sq.argtypes = [i64, P, P, ctypes.c_int]
        lib.fcref_norm_s_sq.restype = f64
        lib.fcref_x_s.argtypes = [i64, P, P, P, ctypes.c_int, ctypes.c_int, P, P]
        lib.fcref_share.argtypes = [i64, ctypes.c_int, P, P]
        lib.fcref_x_s_rows.argtypes = [i64, P, P, P, P, ctypes.c_int, ctypes.c_int, P, P]
        lib.fcref_hvp.argtypes = [i64, P, P, P, ctypes.c_int, ctypes.c_int, P, P, P]
        lib.fcref_project_simplex.argtypes = [ctypes.c_int, P, P]
        lib.fcref_project_columns.argtypes = [i64, ctypes.c_int, P, P]
        lib.fcref_loss.argtypes = [i64, P, P, P, ctypes.c_int, ctypes.c_int, P]
        lib.fcref_loss.restype = f64
        lib.fcref_gradient.argtypes = [i64, P, P, P, ctypes.c_int, ctypes.c_int, P, P]
        lib.fcref_spectral_norm.argtypes = [i64, P, P, P, ctypes.c_int, ctypes.c_int,
                                            f64, ctypes.POINTER(ctypes.c_int)]
        lib.fcref_spectral_norm.restype = f64
        lib.fcref_solve.argtypes = [i64, P, P, P, ctypes.c_int, ctypes.c_int, P,
                                    ctypes.POINTER(_Opts), P, P, P, P, P,
                                    ctypes.POINTER(i32)]
        lib.fcref_solve.restype = ctypes.c_int
        lib.fcref_solve_timed.argtypes = lib.fcref_solve.argtypes + [P]
        lib.fcref_solve_timed.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().fcref_num_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(row_ptr, col_idx, val):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    n = rp.shape[0] - 1
    if ci.shape[0] != rp[-1] or v.shape[0] != rp[-1]:
        raise ValueError("CSR arrays disagree on nnz")
    return n, rp, ci, v


def _mat(X, n):
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim != 2 or X.shape[0] != n:
        raise ValueError(f"X must be (N, C) with N={n}, got {X.shape}")
    return X


def norm_s_sq(row_ptr, col_idx, val, diag_unit: bool) -> float:
    n, rp, ci, v = _csr(row_ptr, col_idx, val)
    return float(_load().fcref_norm_s_sq(n, _ptr(rp), _ptr(v), int(diag_unit)))


def x_s(row_ptr, col_idx, val, diag_unit: bool, X) -> np.ndarray:
    """Row i of the result is X s_i (section 3, eq. gradient_column)."""
    n, rp, ci, v = _csr(row_ptr, col_idx, val)
    X = _mat(X, n)
    out = np.empty_like(X)
    _load().fcref_x_s(n, _ptr(rp), _ptr(ci), _ptr(v), int(diag_unit), X.shape[1],
                      _ptr(X), _ptr(out))
    return out


def share(X) -> np.ndarray:
    """share = X X^T (C x C), Alg. 2."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    C = X.shape[1]
    out = np.empty((C, C), dtype=np.float64)
    _load().fcref_share(X.shape[0], C, _ptr(X), _ptr(out))
    return out


def x_s_rows(rows, sub_row_ptr, sub_col_idx, sub_val, diag_unit: bool, X) -> np.ndarray:
    """X s_i (section 3, eq. gradient_column) for the listed articles only.
    sub_row_ptr/sub_col_idx/sub_val hold the rows of S of those articles, in
    the order of `rows`; X is the full (N, C) membership matrix."""
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    m, rp, ci, v = _csr(sub_row_ptr, sub_col_idx, sub_val)
    if rows.shape[0] != m:
        raise ValueError("one CSR row per listed article")
    X = np.ascontiguousarray(X, dtype=np.float64)
    out = np.empty((m, X.shape[1]), dtype=np.float64)
    _load().fcref_x_s_rows(m, _ptr(rows), _ptr(rp), _ptr(ci), _ptr(v), int(diag_unit),
                           X.shape[1], _ptr(X), _ptr(out))
    return out


def step_rows(rows, sub_row_ptr, sub_col_idx, sub_val, diag_unit: bool, X, tau: float) -> np.ndarray:
    """One projected gradient step X -> P_Omega(X - tau grad f(X)) (Alg. 2)
    evaluated at the listed articles only: column i of the gradient is
    -4 (X s_i - share x_i) (eq. gradient_column) with share = X X^T over all
    N articles, and each updated column is projected onto the simplex (Alg. 1)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    G = share(X)
    XS = x_s_rows(rows, sub_row_ptr, sub_col_idx, sub_val, diag_unit, X)
    xr = X[np.asarray(rows, dtype=np.int64)]
    grad = -4.0 * (XS - xr @ G)
    return project_columns(xr - tau * grad)


def project_simplex(x) -> np.ndarray:
    """Euclidean projection of one vector onto the unit simplex (section 2;
    the threshold of its optimality conditions found by bisection, then
    formed exactly from the support)."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    y = np.empty_like(x)
    _load().fcref_project_simplex(x.shape[0], _ptr(x), _ptr(y))
    return y


def project_columns(V) -> np.ndarray:
    """P_Omega: the simplex projection applied to every row of an (N, C) array."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    out = np.empty_like(V)
    _load().fcref_project_columns(V.shape[0], V.shape[1], _ptr(V), _ptr(out))
    return out


def loss(row_ptr, col_idx, val, diag_unit: bool, X) -> float:
    """Structured loss of Alg. 3."""
    n, rp, ci, v = _csr(row_ptr, col_idx, val)
    X = _mat(X, n)
    return float(_load().fcref_loss(n, _ptr(rp), _ptr(ci), _ptr(v), int(diag_unit),
                                    X.shape[1], _ptr(X)))


def gradient(row_ptr, col_idx, val, diag_unit: bool, X) -> np.ndarray:
    """Gradient of f, column by column (eq. gradient_column)."""
    n, rp, ci, v = _csr(row_ptr, col_idx, val)
    X = _mat(X, n)
    out = np.empty_like(X)
    _load().fcref_gradient(n, _ptr(rp), _ptr(ci), _ptr(v), int(diag_unit), X.shape[1],
                           _ptr(X), _ptr(out))
    return out


def hvp(row_ptr, col_idx, val, diag_unit: bool, X, V) -> np.ndarray:
    """Hessian of f at X applied to V (Theorem 4.1, eq. hessian), rows as X."""
    n, rp, ci, v = _csr(row_ptr, col_idx, val)
    X = _mat(X, n)
    V = _mat(V, n)
    if V.shape != X.shape:
        raise ValueError("V must have the shape of X")
    out = np.empty_like(X)
    _load().fcref_hvp(n, _ptr(rp), _ptr(ci), _ptr(v), int(diag_unit), X.shape[1], _ptr(X),
                      _ptr(V), _ptr(out))
    return out


def face_basis(X, zero_tol: float = 0.0) -> np.ndarray:
    """Orthonormal basis (columns, flattened in the layout of X) of the
    directions V whose rows sum to zero and vanish where x_ki <= zero_tol:
    the tangent directions of Omega at X (eq. 1st_tangent_cone) that keep
    every zero component at zero.  They satisfy <grad f(X), V> = 0 at a
    critical point, so Theorem 4.1 asks <Hess f(X) V, V> >= 0 on them."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    n, C = X.shape
    cols = []
    for i in range(n):
        sup = np.flatnonzero(X[i] > zero_tol)
        m = sup.size
        for t in range(1, m):            # Helmert contrasts on the support
            w = np.zeros(C)
            w[sup[:t]] = 1.0 / t
            w[sup[t]] = -1.0
            w /= np.linalg.norm(w)
            col = np.zeros(n * C)
            col[i * C:(i + 1) * C] = w
            cols.append(col)
    return np.array(cols).T if cols else np.zeros((n * C, 0))


def curvature_dense(row_ptr, col_idx, val, diag_unit: bool, X, zero_tol: float = 0.0):
    """Smallest eigenvalue of the Hessian restricted to face_basis(X), and a
    unit eigen-direction (layout of X), from the dense restricted matrix
    B^T H B built column by column with hvp (small instances only)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    B = face_basis(X, zero_tol)
    if B.shape[1] == 0:
        return float("inf"), np.zeros_like(X)
    HB = np.stack([hvp(row_ptr, col_idx, val, diag_unit, X, B[:, j].reshape(X.shape)).ravel()
                   for j in range(B.shape[1])], axis=1)
    K = B.T @ HB
    K = 0.5 * (K + K.T)
    w, Q = np.linalg.eigh(K)
    return float(w[0]), (B @ Q[:, 0]).reshape(X.shape)


def spectral_norm(row_ptr, col_idx, val, diag_unit: bool, max_iter: int = 1000,
                  rtol: float = 1e-12):
    """(||S||_2, iterations) by power iteration."""
    n, rp, ci, v = _csr(row_ptr, col_idx, val)
    it = ctypes.c_int(0)
    est = _load().fcref_spectral_norm(n, _ptr(rp), _ptr(ci), _ptr(v), int(diag_unit),
                                      int(max_iter), float(rtol), ctypes.byref(it))
    return float(est), int(it.value)


def lipschitz_bound(spec_norm: float, n: int) -> float:
    """L = 4 ||S||_2 + 12 N from the proof of Theorem 3.1."""
    return 4.0 * spec_norm + 12.0 * n


@dataclass
class SolveResult:
    X: np.ndarray          # output Xbar of the last completed iteration
    iters: int             # completed iterations
    f: np.ndarray          # f[0..iters]: loss of Xbar_0 .. Xbar_iters
    tau: np.ndarray        # tau[1..iters] (tau[0] unused)
    trials: np.ndarray     # backtracking trials per iteration
    r: np.ndarray          # gradient-mapping norms ||Y_n - Xbar_n|| / tau_n
    stop_reason: int
    seconds: np.ndarray | None = None   # wall time of iterations 1..iters (timed=True)


def solve(row_ptr, col_idx, val, diag_unit: bool, X0, *, accelerate: bool = True,
          max_iter: int = 100, step: float | None = None, step_schedule=None,
          backtrack: bool = False, L0: float = 1.0, eta: float = 2.0,
          tol_loss: float = math.nan, tol_pgrad: float = 0.0,
          timed: bool = False) -> SolveResult:
    """Parallel FISTA (Alg. 4) or parallel GPA (Alg. 2/3, accelerate=False).
    timed=True also records each iteration's wall time (seconds[1..iters])."""
    n, rp, ci, v = _csr(row_ptr, col_idx, val)
    X0 = _mat(X0, n)
    C = X0.shape[1]
    sched = None
    if step_schedule is not None:
        sched = np.ascontiguousarray(step_schedule, dtype=np.float64)
        if sched.shape[0] < max_iter:
            raise ValueError("step_schedule shorter than max_iter")
    if not backtrack and sched is None and (step is None or step <= 0):
        raise ValueError("a positive constant step, a schedule, or backtracking is required")
    opts = _Opts(int(accelerate), int(max_iter), int(backtrack), 0,
                 float(step or 0.0), float(L0), float(eta), float(tol_loss),
                 float(tol_pgrad),
                 sched.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if sched is not None
                 else ctypes.POINTER(ctypes.c_double)())
    X = np.empty_like(X0)
    f = np.full(max_iter + 1, np.nan)
    tau = np.full(max_iter + 1, np.nan)
    trials = np.zeros(max_iter + 1, dtype=np.int32)
    r = np.full(max_iter + 1, np.nan)
    reason = ctypes.c_int32(0)
    args = (n, _ptr(rp), _ptr(ci), _ptr(v), int(diag_unit), C, _ptr(X0), ctypes.byref(opts),
            _ptr(X), _ptr(f), _ptr(tau), _ptr(trials), _ptr(r), ctypes.byref(reason))
    secs = None
    if timed:
        secs = np.full(max_iter + 1, np.nan)
        it = _load().fcref_solve_timed(*args, _ptr(secs))
        secs = secs[: it + 1]
    else:
        it = _load().fcref_solve(*args)
    return SolveResult(X, int(it), f[: it + 1], tau[: it + 1], trials[: it + 1],
                       r[: it + 1], int(reason.value), secs)
