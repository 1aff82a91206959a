"""Oracle: COO ingest, the sparse formats and the sparsity features, in plain NumPy.

Test infrastructure only. Nothing here is imported by the GPU library.

Definitions followed:
* CSR, ELL: the paper's background section on popular SpMV formats (CSR
  paragraph: data, column index and row index arrays; ELL paragraph: an
  m x max_nnz data matrix and a matching column index matrix).
* COO input: the paper's run-time overhead discussion notes that matrices
  arrive in COO, the SuiteSparse default.
* HYB (ELL part + COO tail) is not defined in the paper; its width follows the
  rule published with the format by Bell and Garland (SC'09, cited by the
  paper for COO/CSR/ELL).
* Features: the paper's table of sparsity features (n, nnz, average, variance,
  ELL ratio, median, mode, standard deviation) plus max row length,
  bandwidth, fill and the HYB tail fraction.

Readings where the paper is silent (listed in the design notes too): indices
are 0-based; entries are sorted by (row, col); duplicate coordinates are an
error; explicit zeros are stored entries; ELL is column-major with the row
count padded to a multiple of 64, padding slots hold column -1 and value +0.0,
and ELL is refused when its padded size exceeds 8 * nnz.
"""
from __future__ import annotations

import math

import numpy as np

OK = "OK"
INVALID_ARG = "INVALID_ARG"
OUT_OF_BOUNDS = "OUT_OF_BOUNDS"
DUPLICATE = "DUPLICATE"
NOT_APPLICABLE = "NOT_APPLICABLE"

ELL_PITCH_MULTIPLE = 64
ELL_FILL_CAP = 8  # padded ELL slots may be at most this many times nnz
HYB_MIN_ROWS = 4096  # Bell-Garland break-even row count
HYB_ROW_FRACTION = 3  # ... or a third of the rows, whichever is larger


class OracleError(Exception):
    def __init__(self, status: str, msg: str = ""):
        super().__init__(f"{status}: {msg}")
        self.status = status


def canonicalize(n_rows: int, n_cols: int, row, col, val):
    """COO ingest: bounds check, sort entries by (row, col), reject duplicates.

    Returns a dict with the canonical ``row``, ``col``, ``val`` arrays (int32,
    int32, input dtype), ``row_ptr`` (int64, n_rows + 1) and ``perm`` (the input
    position of each canonical entry).
    """
    if n_rows < 0 or n_cols < 0:
        raise OracleError(INVALID_ARG, "negative dimension")
    row = np.asarray(row, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    val = np.asarray(val)
    if not (row.shape == col.shape == val.shape) or row.ndim != 1:
        raise OracleError(INVALID_ARG, "row/col/val must be 1-D of equal length")
    if row.size and (row.min() < 0 or row.max() >= n_rows or col.min() < 0 or col.max() >= n_cols):
        raise OracleError(OUT_OF_BOUNDS, "index outside the matrix")
    perm = np.lexsort((col, row))  # stable; primary key row, secondary col
    r, c = row[perm], col[perm]
    if r.size > 1 and np.any((r[1:] == r[:-1]) & (c[1:] == c[:-1])):
        raise OracleError(DUPLICATE, "repeated (row, col)")
    lengths = np.bincount(r, minlength=n_rows) if n_rows else np.zeros(0, np.int64)
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(lengths, out=row_ptr[1:])
    return {
        "n_rows": int(n_rows),
        "n_cols": int(n_cols),
        "row": r.astype(np.int32),
        "col": c.astype(np.int32),
        "val": val[perm],
        "row_ptr": row_ptr,
        "perm": perm,
    }


def row_lengths(row_ptr) -> np.ndarray:
    return np.diff(np.asarray(row_ptr, dtype=np.int64))


def ell_pitch(n_rows: int) -> int:
    m = ELL_PITCH_MULTIPLE
    return (n_rows + m - 1) // m * m


def _ell_scatter(row_ptr, col, val, n_rows, width, pitch):
    """Column-major ELL arrays of the given width holding entries k < min(len_i, width)."""
    lengths = row_lengths(row_ptr)
    ell_col = np.full(width * pitch, -1, dtype=np.int32)
    ell_val = np.zeros(width * pitch, dtype=np.asarray(val).dtype)
    if col.size:
        r = np.repeat(np.arange(n_rows, dtype=np.int64), lengths)
        k = np.arange(col.size, dtype=np.int64) - row_ptr[r]
        keep = k < width
        slot = k[keep] * pitch + r[keep]
        ell_col[slot] = col[keep]
        ell_val[slot] = val[keep]
    return ell_col, ell_val


def to_ell(canon) -> dict:
    """ELL: width K = longest row; slot (i, k) at k * pitch + i."""
    n = canon["n_rows"]
    nnz = canon["col"].size
    lengths = row_lengths(canon["row_ptr"])
    K = int(lengths.max()) if n and nnz else 0
    pitch = ell_pitch(n)
    if nnz > 0 and pitch * K > ELL_FILL_CAP * nnz:
        raise OracleError(NOT_APPLICABLE, f"ELL would hold {pitch * K} slots for {nnz} entries")
    ell_col, ell_val = _ell_scatter(canon["row_ptr"], canon["col"], canon["val"], n, K, pitch)
    return {"K": K, "pitch": pitch, "ell_col": ell_col, "ell_val": ell_val}


def hyb_width(lengths, n_rows: int) -> int:
    """Bell-Garland HYB width: the largest k with at least T rows of length >= k,
    T = min(n_rows, max(4096, ceil(n_rows / 3)))."""
    if n_rows == 0:
        return 0
    T = min(n_rows, max(HYB_MIN_ROWS, -(-n_rows // HYB_ROW_FRACTION)))
    hist = np.bincount(np.asarray(lengths, dtype=np.int64))
    count_ge = np.cumsum(hist[::-1])[::-1]  # count_ge[k] = #{i : len_i >= k}
    ks = np.nonzero(count_ge >= T)[0]
    return int(ks.max())


def to_hyb(canon, k_override: int = -1) -> dict:
    """HYB: ELL part of width K_h plus the remaining entries as a COO tail in canonical order."""
    n = canon["n_rows"]
    rp = canon["row_ptr"]
    lengths = row_lengths(rp)
    K = hyb_width(lengths, n) if k_override < 0 else int(k_override)
    pitch = ell_pitch(n)
    ell_col, ell_val = _ell_scatter(rp, canon["col"], canon["val"], n, K, pitch)
    r = canon["row"].astype(np.int64)
    k = np.arange(r.size, dtype=np.int64) - rp[r] if r.size else np.zeros(0, np.int64)
    tail = k >= K
    return {
        "K": K,
        "pitch": pitch,
        "ell_col": ell_col,
        "ell_val": ell_val,
        "tail_row": canon["row"][tail],
        "tail_col": canon["col"][tail],
        "tail_val": canon["val"][tail],
    }


# ---- inverse maps, used by round-trip pins ---------------------------------

def csr_to_coo_rows(row_ptr) -> np.ndarray:
    rp = np.asarray(row_ptr, dtype=np.int64)
    return np.repeat(np.arange(rp.size - 1, dtype=np.int32), np.diff(rp))


def ell_to_coo(ell: dict, n_rows: int):
    """Stored (row, col, val) of an ELL or HYB-ELL part, in (row, col) order."""
    K, pitch = ell["K"], ell["pitch"]
    c = ell["ell_col"].reshape(K, pitch)[:, :n_rows]
    v = ell["ell_val"].reshape(K, pitch)[:, :n_rows]
    k_idx, r_idx = np.nonzero(c >= 0)
    order = np.lexsort((k_idx, r_idx))
    r_idx, k_idx = r_idx[order], k_idx[order]
    return r_idx.astype(np.int32), c[k_idx, r_idx].astype(np.int32), v[k_idx, r_idx]


def to_dense(n_rows, n_cols, row, col, val) -> np.ndarray:
    d = np.zeros((n_rows, n_cols), dtype=np.float64)
    d[np.asarray(row, np.int64), np.asarray(col, np.int64)] = np.asarray(val, np.float64)
    return d


# ---- sparsity features -------------------------------------------------------

FEATURE_NAMES = ("n", "nnz", "mean", "var", "std", "median", "mode", "ell_ratio",
                 "max", "bandwidth", "fill", "hyb_coo_frac")


def features(canon) -> np.ndarray:
    """The 12 features, in FP64, in FEATURE_NAMES order.

    mean = nnz / n; var = population variance of row lengths; std = sqrt(var);
    median = middle row length (mean of the two middle ones for even n);
    mode = most frequent row length, smallest on ties; ell_ratio = nnz / (n * max);
    bandwidth = max |i - j| over stored entries; fill = nnz / (n_rows * n_cols);
    hyb_coo_frac = entries left to the HYB tail at the Bell-Garland width / nnz.
    Quantities with an empty denominator are 0.
    """
    n = canon["n_rows"]
    n_cols = canon["n_cols"]
    lengths = row_lengths(canon["row_ptr"])
    nnz = int(lengths.sum())
    out = np.zeros(12, dtype=np.float64)
    out[0] = n
    out[1] = nnz
    if n == 0:
        return out
    mx = int(lengths.max())
    out[2] = nnz / n
    out[3] = float(np.var(lengths.astype(np.float64)))
    out[4] = math.sqrt(out[3])
    out[5] = float(np.median(lengths))
    out[6] = int(np.bincount(lengths).argmax())
    out[7] = nnz / (n * mx) if mx > 0 else 0.0
    out[8] = mx
    if nnz:
        out[9] = int(np.abs(canon["row"].astype(np.int64) - canon["col"].astype(np.int64)).max())
        Kh = hyb_width(lengths, n)
        out[11] = int(np.maximum(lengths - Kh, 0).sum()) / nnz
    out[10] = nnz / (n * n_cols) if n_cols else 0.0
    return out


# columns that enter the selector network as log2(1 + v); the rest stay raw
LOG_FEATURES = (0, 1, 2, 3, 4, 5, 6, 8, 9)


def transform_features(F) -> np.ndarray:
    """Selector input map: log2(1 + v) on counts and lengths, ratios unchanged."""
    T = np.array(F, dtype=np.float64, copy=True)
    idx = list(LOG_FEATURES)
    T[..., idx] = np.log2(1.0 + T[..., idx])
    return T
