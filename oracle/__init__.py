"""CPU FP64 oracle for the asynchronous block ILU(0) preconditioner: ctypes wrappers.

TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the benchmark's CPU-baseline leg
may import this package. It shares no code with the HIP library (paper_1912_00539_amd).

Every function takes the BSR case as (n, rowptr int32[N+1], colidx int32[Z], A float64[Z,4,4])
and returns fresh numpy arrays. The C source (abilu_oracle.c) cites the passage each routine
follows.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

FLAG_MODIFIED = 1
FLAG_NONFINITE = 2
PC_EXACT = -1


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build(verbose=False)
        L = C.CDLL(path)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        vp = C.c_void_p
        L.oracle_inv4.argtypes = [f64p, f64p]; L.oracle_inv4.restype = C.c_int
        L.oracle_check_pattern.argtypes = [C.c_int, i32p, i32p]; L.oracle_check_pattern.restype = C.c_int
        L.oracle_pairs.argtypes = [C.c_int, i32p, i32p, i64p, vp, vp]; L.oracle_pairs.restype = C.c_long
        L.oracle_depth.argtypes = [C.c_int, i32p, i32p, i32p]; L.oracle_depth.restype = C.c_int
        L.oracle_levels.argtypes = [C.c_int, i32p, i32p, i32p, i32p, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.oracle_levels.restype = None
        for name in ("oracle_ilu0_seq",):
            getattr(L, name).argtypes = [C.c_int, i32p, i32p, f64p, f64p, f64p]
            getattr(L, name).restype = C.c_uint
        for name in ("oracle_factor_sync", "oracle_factor_gs"):
            getattr(L, name).argtypes = [C.c_int, i32p, i32p, f64p, vp, C.c_int, f64p, f64p]
            getattr(L, name).restype = C.c_uint
        L.oracle_factor_chunked.argtypes = [C.c_int, i32p, i32p, f64p, vp, C.c_int, C.c_int, C.c_int, f64p, f64p]
        L.oracle_factor_chunked.restype = C.c_uint
        L.oracle_apply_chunked.argtypes = [C.c_int, i32p, i32p, f64p, f64p, f64p, f64p, C.c_int, C.c_int, C.c_int]
        L.oracle_apply_chunked.restype = None
        L.oracle_apply_sync.argtypes = [C.c_int, i32p, i32p, f64p, f64p, f64p, f64p, C.c_int]
        L.oracle_apply_sync.restype = None
        L.oracle_trisolve_exact.argtypes = [C.c_int, i32p, i32p, f64p, f64p, f64p, f64p]
        L.oracle_trisolve_exact.restype = None
        L.oracle_spmv.argtypes = [C.c_int, i32p, i32p, f64p, f64p, f64p]; L.oracle_spmv.restype = None
        L.oracle_fgmres.argtypes = [C.c_int, i32p, i32p, f64p, f64p, f64p, C.c_int, C.c_int, C.c_double,
                                    f64p, f64p, C.c_int, vp, vp]
        L.oracle_fgmres.restype = C.c_int
        L.oracle_ilu_residual.argtypes = [C.c_int, i32p, i32p, f64p, f64p]; L.oracle_ilu_residual.restype = C.c_double
        L.oracle_fixed_point_residual.argtypes = [C.c_int, i32p, i32p, f64p, f64p]
        L.oracle_fixed_point_residual.restype = C.c_double
        L.oracle_jacobi_norms.argtypes = [C.c_int, i32p, i32p, f64p, f64p, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_jacobi_norms.restype = None
        L.oracle_factor_error.argtypes = [C.c_int, i32p, i32p, f64p, f64p, f64p, C.POINTER(C.c_double),
                                          C.POINTER(C.c_double)]
        L.oracle_factor_error.restype = None
        L.oracle_num_threads.argtypes = []; L.oracle_num_threads.restype = C.c_int
        _LIB = L
    return _LIB


class _FgmresResult(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("rel_true_residual", C.c_double)]


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _pat(rowptr, colidx):
    return _c(rowptr, np.int32), _c(colidx, np.int32)


def num_threads() -> int:
    return int(_lib().oracle_num_threads())


def inv4(M):
    out = np.empty(16)
    flag = _lib().oracle_inv4(_c(M, np.float64).reshape(16), out)
    return out.reshape(4, 4), int(flag)


def check_pattern(n, rowptr, colidx) -> int:
    rp, ci = _pat(rowptr, colidx)
    return int(_lib().oracle_check_pattern(n, rp, ci))


def pairs(n, rowptr, colidx):
    """(pair_ptr int64[Z+1], pik int32[P], pkj int32[P]) of the update sets K(i,j)."""
    rp, ci = _pat(rowptr, colidx)
    z = int(rp[n]) if n > 0 else 0
    ptr = np.zeros(z + 1, np.int64)
    cnt = _lib().oracle_pairs(n, rp, ci, ptr, None, None)
    pik = np.zeros(max(cnt, 1), np.int32); pkj = np.zeros(max(cnt, 1), np.int32)
    _lib().oracle_pairs(n, rp, ci, ptr, pik.ctypes.data_as(C.c_void_p), pkj.ctypes.data_as(C.c_void_p))
    return ptr, pik[:cnt], pkj[:cnt]


def depth(n, rowptr, colidx):
    """(D, depth int32[Z]) of the block unknowns' dependency DAG."""
    rp, ci = _pat(rowptr, colidx)
    d = np.zeros(max(int(rp[n]), 1), np.int32)
    D = _lib().oracle_depth(n, rp, ci, d)
    return int(D), d[: int(rp[n])]


def levels(n, rowptr, colidx):
    """(levels of L, levels of U, per-row lower levels, per-row upper levels)."""
    rp, ci = _pat(rowptr, colidx)
    ll = np.zeros(max(n, 1), np.int32); lu = np.zeros(max(n, 1), np.int32)
    nl = C.c_int(0); nu = C.c_int(0)
    _lib().oracle_levels(n, rp, ci, ll, lu, C.byref(nl), C.byref(nu))
    return nl.value, nu.value, ll[:n], lu[:n]


def _out(n, z):
    return np.zeros(max(z, 1) * 16), np.zeros(max(n, 1) * 16)


def _shape(X, D, n, z):
    return X[: z * 16].reshape(z, 4, 4), D[: n * 16].reshape(n, 4, 4)


def ilu0_seq(n, rowptr, colidx, A):
    """Sequential block ILU(0): returns (X, Dinv, flags)."""
    rp, ci = _pat(rowptr, colidx); z = int(rp[n]) if n else 0
    X, D = _out(n, z)
    f = _lib().oracle_ilu0_seq(n, rp, ci, _c(A, np.float64).reshape(-1) if z else np.zeros(16), X, D)
    return (*_shape(X, D, n, z), int(f))


def _factor(fn, n, rowptr, colidx, A, nsw, X0):
    rp, ci = _pat(rowptr, colidx); z = int(rp[n]) if n else 0
    X, D = _out(n, z)
    Af = _c(A, np.float64).reshape(-1) if z else np.zeros(16)
    x0 = None
    if X0 is not None:
        X0 = _c(X0, np.float64).reshape(-1)
        x0 = X0.ctypes.data_as(C.c_void_p)
    f = fn(n, rp, ci, Af, x0, int(nsw), X, D)
    return (*_shape(X, D, n, z), int(f))


def factor_sync(n, rowptr, colidx, A, nsw, X0=None):
    """nsw synchronous sweeps x^{p+1} = h(x^p) from X0 (default A): (X, Dinv, flags)."""
    return _factor(_lib().oracle_factor_sync, n, rowptr, colidx, A, nsw, X0)


def factor_gs(n, rowptr, colidx, A, nsw, X0=None):
    """nsw in-place row-major sweeps (one worker): (X, Dinv, flags)."""
    return _factor(_lib().oracle_factor_gs, n, rowptr, colidx, A, nsw, X0)


def factor_chunked(n, rowptr, colidx, A, nsw, R, X0=None, descending=False):
    """nsw chunked sweeps (chunks of R rows, Gauss-Seidel within a chunk, other chunks read from
    the previous sweep) from X0 (default A): (X, Dinv, flags)."""
    rp, ci = _pat(rowptr, colidx); z = int(rp[n]) if n else 0
    X, D = _out(n, z)
    Af = _c(A, np.float64).reshape(-1) if z else np.zeros(16)
    x0 = None
    if X0 is not None:
        X0 = _c(X0, np.float64).reshape(-1)
        x0 = X0.ctypes.data_as(C.c_void_p)
    f = _lib().oracle_factor_chunked(n, rp, ci, Af, x0, int(nsw), int(R), int(bool(descending)), X, D)
    return (*_shape(X, D, n, z), int(f))


def apply_chunked(n, rowptr, colidx, X, Dinv, r, nsw, R, descending=False):
    rp, ci = _pat(rowptr, colidx)
    z = np.zeros(max(4 * n, 1))
    _lib().oracle_apply_chunked(n, rp, ci, _c(X, np.float64).reshape(-1), _c(Dinv, np.float64).reshape(-1),
                                _c(r, np.float64), z, int(nsw), int(R), int(bool(descending)))
    return z[: 4 * n]


def apply_sync(n, rowptr, colidx, X, Dinv, r, nsw):
    rp, ci = _pat(rowptr, colidx)
    z = np.zeros(max(4 * n, 1))
    _lib().oracle_apply_sync(n, rp, ci, _c(X, np.float64).reshape(-1), _c(Dinv, np.float64).reshape(-1),
                             _c(r, np.float64), z, int(nsw))
    return z[: 4 * n]


def trisolve_exact(n, rowptr, colidx, X, Dinv, r):
    rp, ci = _pat(rowptr, colidx)
    z = np.zeros(max(4 * n, 1))
    _lib().oracle_trisolve_exact(n, rp, ci, _c(X, np.float64).reshape(-1), _c(Dinv, np.float64).reshape(-1),
                                 _c(r, np.float64), z)
    return z[: 4 * n]


def spmv(n, rowptr, colidx, A, x):
    rp, ci = _pat(rowptr, colidx)
    y = np.zeros(max(4 * n, 1))
    _lib().oracle_spmv(n, rp, ci, _c(A, np.float64).reshape(-1), _c(x, np.float64), y)
    return y[: 4 * n]


def fgmres(n, rowptr, colidx, A, b, X, Dinv, restart=30, maxit=2500, rtol=1e-2, apply_nsw=3, x0=None,
           history=False):
    """Restarted FGMRES(restart), right preconditioned by the sweep apply (apply_nsw sweeps;
    0 = none, PC_EXACT = exact triangular solves). Returns dict(x, iters, restarts, converged,
    rel_true_residual[, hist])."""
    rp, ci = _pat(rowptr, colidx)
    x = np.zeros(4 * n) if x0 is None else _c(x0, np.float64).copy()
    res = _FgmresResult()
    hist = np.zeros(maxit + 1) if history else None
    _lib().oracle_fgmres(n, rp, ci, _c(A, np.float64).reshape(-1), _c(b, np.float64), x, int(restart),
                         int(maxit), float(rtol), _c(X, np.float64).reshape(-1), _c(Dinv, np.float64).reshape(-1),
                         int(apply_nsw), C.cast(C.pointer(res), C.c_void_p),
                         hist.ctypes.data_as(C.c_void_p) if history else None)
    out = dict(x=x, iters=res.iters, restarts=res.restarts, converged=bool(res.converged),
               rel_true_residual=res.rel_true_residual)
    if history:
        out["hist"] = hist[: res.iters + 1]
    return out


def ilu_residual(n, rowptr, colidx, A, X) -> float:
    rp, ci = _pat(rowptr, colidx)
    return float(_lib().oracle_ilu_residual(n, rp, ci, _c(A, np.float64).reshape(-1), _c(X, np.float64).reshape(-1)))


def fixed_point_residual(n, rowptr, colidx, A, X) -> float:
    rp, ci = _pat(rowptr, colidx)
    return float(_lib().oracle_fixed_point_residual(n, rp, ci, _c(A, np.float64).reshape(-1),
                                                    _c(X, np.float64).reshape(-1)))


def jacobi_norms(n, rowptr, colidx, X, Dinv):
    rp, ci = _pat(rowptr, colidx)
    a = C.c_double(0); b = C.c_double(0)
    _lib().oracle_jacobi_norms(n, rp, ci, _c(X, np.float64).reshape(-1), _c(Dinv, np.float64).reshape(-1),
                               C.byref(a), C.byref(b))
    return a.value, b.value


def factor_error(n, rowptr, colidx, X, X0, Xilu):
    """(L error, U error): ||vec(L - L_ilu)||_inf / ||vec(L0 - L_ilu)||_inf and likewise for U, the
    factors in CSR block order (Section 6.2)."""
    rp, ci = _pat(rowptr, colidx)
    eL, eU = C.c_double(), C.c_double()
    _lib().oracle_factor_error(int(n), rp, ci, _c(X, np.float64).reshape(-1), _c(X0, np.float64).reshape(-1),
                               _c(Xilu, np.float64).reshape(-1), C.byref(eL), C.byref(eU))
    return eL.value, eU.value
