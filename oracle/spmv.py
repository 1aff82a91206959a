"""Oracle SpMV in FP64 (C, via ctypes) and an exact rational brute force.

Test infrastructure only. ``spmv_csr`` calls the plain C loop in
spmv_oracle.c; ``spmv_dense_exact`` evaluates y = alpha*A*x + beta*y over the
dense matrix with Python fractions, for pinning the C loop on tiny inputs.
"""
from __future__ import annotations

import ctypes
import os
from fractions import Fraction

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.oracle_spmv_csr_f64.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_double,
                                            ctypes.c_double, P, ctypes.c_int]
        lib.oracle_spmv_csr_f64.restype = None
        lib.oracle_spmv_rows_f64.argtypes = [ctypes.c_int64, P, P, P, P, P, ctypes.c_double,
                                             ctypes.c_double, P, P, P]
        lib.oracle_spmv_rows_f64.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def spmv_csr(row_ptr, col, val, x, alpha=1.0, beta=0.0, y=None, n_threads=1) -> np.ndarray:
    """y = alpha * A x + beta * y in FP64 (FP32 inputs are promoted exactly)."""
    lib = _load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    n = rp.size - 1
    out = np.zeros(n, dtype=np.float64) if y is None else np.array(y, dtype=np.float64, copy=True)
    lib.oracle_spmv_csr_f64(n, _ptr(rp), _ptr(c), _ptr(v), _ptr(xx), float(alpha), float(beta),
                            _ptr(out), int(n_threads))
    return out


def spmv_rows(rows, row_ptr, col, val, x, alpha=1.0, beta=0.0, y=None):
    """Selected rows only: (y_ref[rows], D[rows]) with D_i = |alpha| sum_j |a_ij x_j| + |beta y_i|."""
    lib = _load()
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    yin = np.zeros(rp.size - 1) if y is None else np.ascontiguousarray(y, dtype=np.float64)
    out = np.zeros(rows.size)
    den = np.zeros(rows.size)
    lib.oracle_spmv_rows_f64(rows.size, _ptr(rows), _ptr(rp), _ptr(c), _ptr(v), _ptr(xx),
                             float(alpha), float(beta), _ptr(yin), _ptr(out), _ptr(den))
    return out, den


def row_denominator(row_ptr, col, val, x, alpha, beta, y_in) -> np.ndarray:
    """D_i = |alpha| * sum_j |a_ij x_j| + |beta| * |y_i| (the beta term only when beta != 0)."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    p = np.abs(np.asarray(val, np.float64) * np.asarray(x, np.float64)[np.asarray(col, np.int64)])
    n = rp.size - 1
    s = np.zeros(n)
    if p.size:
        r = np.repeat(np.arange(n), np.diff(rp))
        np.add.at(s, r, p)
    d = abs(alpha) * s
    if beta != 0.0:
        d = d + abs(beta) * np.abs(np.asarray(y_in, np.float64))
    return d


def spmv_dense_exact(n_rows, n_cols, row, col, val, x, alpha, beta, y_in):
    """Exact rational y = alpha*A*x + beta*y over the dense matrix; returns a list of Fractions."""
    A = [[Fraction(0)] * n_cols for _ in range(n_rows)]
    for r, c, v in zip(np.asarray(row).tolist(), np.asarray(col).tolist(), np.asarray(val, np.float64).tolist()):
        A[r][c] = Fraction(v)
    xs = [Fraction(v) for v in np.asarray(x, np.float64).tolist()]
    fa, fb = Fraction(alpha), Fraction(beta)
    out = []
    for i in range(n_rows):
        s = sum((A[i][j] * xs[j] for j in range(n_cols)), Fraction(0))
        yi = fa * s
        if beta != 0.0:
            yi += fb * Fraction(float(y_in[i]))
        out.append(yi)
    return out


def max_row_error(y, y_ref, denom) -> float:
    """max_i |y_i - y_ref_i| / D_i; rows with D_i = 0 must match exactly (else inf)."""
    y = np.asarray(y, np.float64)
    y_ref = np.asarray(y_ref, np.float64)
    denom = np.asarray(denom, np.float64)
    diff = np.abs(y - y_ref)
    zero = denom == 0
    if np.any(diff[zero] != 0) or np.any(np.isnan(y) != np.isnan(y_ref)):
        return float("inf")
    with np.errstate(invalid="ignore", divide="ignore"):
        r = np.where(zero, 0.0, diff / np.where(zero, 1.0, denom))
    return float(np.nanmax(r)) if r.size else 0.0
