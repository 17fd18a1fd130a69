"""ctypes front end of the C FP64 oracle (test infrastructure only)."""

from __future__ import annotations

import ctypes
import os

import numpy as np

from ._build import LIB, SRC, build_oracle

PC_IDENTITY, PC_JACOBI, PC_CHEBYSHEV = 0, 1, 2
ST_CONVERGED, ST_ARG, ST_MAXIT, ST_BREAKDOWN = 0, 1, 2, 3

_lib = None
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build_oracle()
        L = ctypes.CDLL(LIB)
        L.oracle_spmv.argtypes = [ctypes.c_int, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.oracle_spmv.restype = None
        L.oracle_precond.argtypes = [ctypes.c_int, _i32p, _i32p, _f64p, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double, _f64p, _f64p]
        L.oracle_precond.restype = ctypes.c_int
        L.oracle_pcg.argtypes = [ctypes.c_int, _i32p, _i32p, _f64p, _f64p, _f64p, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, _f64p]
        L.oracle_pcg.restype = ctypes.c_int
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _csr_arrays(A):
    return (np.ascontiguousarray(A.row_ptr, dtype=np.int32),
            np.ascontiguousarray(A.col_idx, dtype=np.int32),
            np.ascontiguousarray(A.val, dtype=np.float64))


def spmv(A, x):
    rp, ci, v = _csr_arrays(A)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.n)
    lib().oracle_spmv(A.n, rp, ci, v, x, y)
    return y


def precond_apply(A, r, kind=PC_JACOBI, degree=4, lam_lo=0.0, lam_hi=0.0):
    rp, ci, v = _csr_arrays(A)
    r = np.ascontiguousarray(r, dtype=np.float64)
    z = np.empty(A.n)
    st = lib().oracle_precond(A.n, rp, ci, v, kind, degree, lam_lo, lam_hi, r, z)
    if st != 0:
        raise ValueError("oracle_precond: bad arguments")
    return z


def pcg(A, b, x0=None, tol=1e-10, maxit=5000, precond=PC_JACOBI, degree=4, lam_lo=0.0,
        lam_hi=0.0, history=False, threads=0):
    """FP64 PCG (Alg. 1).  Returns (x, info) with info keys iters, status,
    relres (updated), relres_true, bnorm and, if ``history``, delta, alpha, beta."""
    rp, ci, v = _csr_arrays(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    out = np.zeros(5)
    hist = [np.zeros(maxit + 1) for _ in range(3)] if history else [None, None, None]
    ptr = [h.ctypes.data_as(ctypes.c_void_p) if h is not None else None for h in hist]
    L = lib()
    if threads:
        L.oracle_set_threads(int(threads))
    L.oracle_pcg(A.n, rp, ci, v, b, x, float(tol), int(maxit), int(precond), int(degree),
                 float(lam_lo), float(lam_hi), ptr[0], ptr[1], ptr[2], out)
    it = int(out[0])
    info = dict(iters=it, status=int(out[1]), relres=out[2], relres_true=out[3], bnorm=out[4])
    if history:
        info["delta"] = hist[0][: it + 1]
        info["alpha"] = hist[1][:it]
        info["beta"] = hist[2][:it]
    return x, info


def num_threads() -> int:
    return int(lib().oracle_num_threads())
