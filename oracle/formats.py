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


# ---- SELL-C-sigma (sliced ELL) ------------------------------------------------
#
# The paper's SELL paragraph (Background, popular SpMV formats): rows are cut
# into slices of a constant number of rows, each slice is an ELL block as wide
# as its longest row, and a slice index array points at each slice's start.
# Readings where the paper leaves the layout open (listed in the design notes):
#   * slice height C = 64 rows (one wavefront);
#   * a slice's width is its longest row rounded up to a whole number of groups
#     of G = 4 slots, and slot k of the row at position l of slice s sits at
#     slice_ptr[s] + (k // G) * C * G + l * G + k % G (each row's slots come in
#     runs of four, the runs of the slice's rows one after another);
#   * sigma: rows may be reordered inside windows of sigma consecutive rows by
#     descending length (stable), as in SELL-C-sigma (Kreutzer et al., SIAM J.
#     Sci. Comput. 2014); sigma = 1 keeps the natural order, which is the
#     paper's SELL. perm[p] is the row stored at position p;
#   * padding slots hold column -1 and value +0.0, also the positions past the
#     last row in the last slice; the slice pointers count slots (int64);
#   * refused (NOT_APPLICABLE) when the slots exceed 8 * nnz, as for ELL, unless
#     the layout is small (at most SMALL_LAYOUT_SLOTS slots);
#   * the default sigma is the one of {1, 16384} whose layout stores fewer bytes
#     (slots * (4 + v), plus 4 bytes per row for perm when sigma > 1), ties to 1.

SELL_SLICE = 64
SMALL_LAYOUT_SLOTS = 65536  # SELL slots / BELL values that are never refused
SELL_GROUP = 4
SELL_SIGMA_WIDE = 16384


def sell_order(lengths, sigma: int) -> np.ndarray:
    """perm[p] = row at position p: descending length inside each window of sigma rows (stable)."""
    lengths = np.asarray(lengths, np.int64)
    n = lengths.size
    if sigma <= 1:
        return np.arange(n, dtype=np.int32)
    window = np.arange(n, dtype=np.int64) // sigma
    # lexsort: last key primary -> window, then longer rows first, then row index
    perm = np.lexsort((np.arange(n), -lengths, window))
    return perm.astype(np.int32)


def sell_slice_widths(lengths, perm, C=SELL_SLICE, G=SELL_GROUP) -> np.ndarray:
    """Each slice's width: its longest row rounded up to a multiple of G."""
    lengths = np.asarray(lengths, np.int64)
    n = lengths.size
    n_slices = -(-n // C)
    w = np.zeros(n_slices, np.int64)
    for s in range(n_slices):
        rows = perm[s * C:(s + 1) * C]
        m = int(lengths[rows].max()) if rows.size else 0
        w[s] = -(-m // G) * G
    return w


def sell_sigma_rule(lengths, value_bytes: int) -> int:
    """Default sigma: the candidate (1 or SELL_SIGMA_WIDE) whose layout stores fewer bytes."""
    lengths = np.asarray(lengths, np.int64)
    best, best_bytes = 1, None
    for sigma in (1, SELL_SIGMA_WIDE):
        w = sell_slice_widths(lengths, sell_order(lengths, sigma))
        b = int(w.sum()) * SELL_SLICE * (4 + value_bytes) + (4 * lengths.size if sigma > 1 else 0)
        if best_bytes is None or b < best_bytes:
            best, best_bytes = sigma, b
    return best


def to_sell(canon, sigma: int = -1, C: int = SELL_SLICE, G: int = SELL_GROUP) -> dict:
    """SELL-C-sigma layout of the canonical matrix (see the block comment above)."""
    n = canon["n_rows"]
    nnz = canon["col"].size
    rp = np.asarray(canon["row_ptr"], np.int64)
    lengths = row_lengths(rp)
    vb = np.asarray(canon["val"]).dtype.itemsize
    if sigma < 0:
        sigma = sell_sigma_rule(lengths, vb) if n else 1
    perm = sell_order(lengths, sigma)
    widths = sell_slice_widths(lengths, perm, C, G)
    slice_ptr = np.zeros(widths.size + 1, np.int64)
    np.cumsum(widths * C, out=slice_ptr[1:])
    slots = int(slice_ptr[-1])
    if nnz > 0 and slots > max(ELL_FILL_CAP * nnz, SMALL_LAYOUT_SLOTS):
        raise OracleError(NOT_APPLICABLE, f"SELL would hold {slots} slots for {nnz} entries")
    col = np.full(slots, -1, np.int32)
    val = np.zeros(slots, dtype=np.asarray(canon["val"]).dtype)
    for p in range(n):
        r = int(perm[p])
        s, l = divmod(p, C)
        k = np.arange(lengths[r], dtype=np.int64)
        slot = slice_ptr[s] + (k // G) * C * G + l * G + k % G
        col[slot] = canon["col"][rp[r]:rp[r + 1]]
        val[slot] = canon["val"][rp[r]:rp[r + 1]]
    return {"C": C, "G": G, "sigma": int(sigma), "n_slices": int(widths.size),
            "slice_ptr": slice_ptr, "perm": perm, "col": col, "val": val}


# ---- BELL (blocked ELL) ---------------------------------------------------------
#
# The paper's BELL paragraph: the ELL format over dense blocks, a data matrix of
# blocks and a column index matrix of block indices, default block 2 x 2.
# Readings (listed in the design notes):
#   * square b x b blocks, b in {2, 4, 8}; block row i holds rows [b i, b i + b),
#     block column j columns [b j, b j + b); a block is stored when it holds at
#     least one entry; absent entries inside a stored block are +0.0 (so a
#     non-finite x value meeting such a zero gives NaN, as in any blocked format);
#   * block rows are ELL rows: width K_b = most stored blocks in one block row,
#     the blocks of a block row in increasing block column, pitch = block rows
#     rounded up to 64; slot (i, k) sits at k * pitch + i: bcol holds the block
#     column (-1 for padding), bval holds the block's b * b values at
#     (k * pitch + i) * b * b, row-major inside the block (zeros for padding);
#   * refused (NOT_APPLICABLE) when the stored values (pitch * K_b * b^2) exceed
#     8 * nnz, unless they are at most SMALL_LAYOUT_SLOTS;
#   * the default b is the one of 2, 4, 8 within the cap whose layout stores the
#     fewest bytes (pitch * K_b * (4 + b^2 v)), ties to the smaller block (2 when
#     none is within the cap).

BELL_SIZES = (2, 4, 8)


def bell_block_counts(canon, b: int) -> np.ndarray:
    """Stored blocks per block row for b x b blocks."""
    n = canon["n_rows"]
    nbr = -(-n // b)
    r = np.asarray(canon["row"], np.int64) // b
    c = np.asarray(canon["col"], np.int64) // b
    keys = np.unique(r * (int(canon["n_cols"]) // b + 1) + c) if r.size else np.zeros(0, np.int64)
    br = keys // (int(canon["n_cols"]) // b + 1)
    return np.bincount(br, minlength=nbr).astype(np.int64) if nbr else np.zeros(0, np.int64)


def bell_size_rule(canon, value_bytes: int) -> int:
    """Default block edge: of the sizes within the fill cap, the one storing the fewest
    bytes, ties to the smaller; 2 (the paper's default) when none is within the cap."""
    nnz = canon["col"].size
    best, best_bytes = BELL_SIZES[0], None
    for b in BELL_SIZES:
        cnt = bell_block_counts(canon, b)
        K = int(cnt.max()) if cnt.size and nnz else 0
        pitch = ell_pitch(cnt.size)
        if nnz > 0 and pitch * K * b * b > max(ELL_FILL_CAP * nnz, SMALL_LAYOUT_SLOTS):
            continue
        by = pitch * K * (4 + b * b * value_bytes)
        if best_bytes is None or by < best_bytes:
            best, best_bytes = b, by
    return best


def to_bell(canon, b: int = -1) -> dict:
    """BELL layout with b x b blocks (see the block comment above)."""
    n, n_cols = canon["n_rows"], canon["n_cols"]
    nnz = canon["col"].size
    vdt = np.asarray(canon["val"]).dtype
    if b < 0:
        b = bell_size_rule(canon, vdt.itemsize)
    if b not in BELL_SIZES:
        raise OracleError(INVALID_ARG, f"block size {b}")
    cnt = bell_block_counts(canon, b)
    nbr = cnt.size
    K = int(cnt.max()) if nbr and nnz else 0
    pitch = ell_pitch(nbr)
    if nnz > 0 and pitch * K * b * b > max(ELL_FILL_CAP * nnz, SMALL_LAYOUT_SLOTS):
        raise OracleError(NOT_APPLICABLE, f"BELL would hold {pitch * K * b * b} values for {nnz} entries")
    bcol = np.full(K * pitch, -1, np.int32)
    bval = np.zeros(K * pitch * b * b, dtype=vdt)
    # blocks of each block row in increasing block column: slot k = rank of the block
    slot_of = {}
    next_k = np.zeros(nbr, np.int64)
    rows = np.asarray(canon["row"], np.int64)
    cols = np.asarray(canon["col"], np.int64)
    blocks = sorted(set(zip((rows // b).tolist(), (cols // b).tolist())))
    for br, bc in blocks:
        k = int(next_k[br])
        next_k[br] += 1
        slot_of[(br, bc)] = k
        bcol[k * pitch + br] = bc
    for e in range(nnz):
        r, c = int(rows[e]), int(cols[e])
        k = slot_of[(r // b, c // b)]
        bval[(k * pitch + r // b) * b * b + (r % b) * b + (c % b)] = canon["val"][e]
    return {"b": b, "K": K, "pitch": pitch, "n_block_rows": nbr, "bcol": bcol, "bval": bval}


def sell_to_coo(sell: dict, n_rows: int):
    """Stored (row, col, val) of a SELL layout, in (row, col) order."""
    C, G = sell["C"], sell["G"]
    rows, cols, vals = [], [], []
    for s in range(sell["n_slices"]):
        s0, s1 = int(sell["slice_ptr"][s]), int(sell["slice_ptr"][s + 1])
        width = (s1 - s0) // C
        for l in range(C):
            p = s * C + l
            if p >= n_rows:
                continue
            for k in range(width):
                slot = s0 + (k // G) * C * G + l * G + k % G
                if sell["col"][slot] >= 0:
                    rows.append(int(sell["perm"][p]))
                    cols.append(int(sell["col"][slot]))
                    vals.append(sell["val"][slot])
    order = np.lexsort((np.array(cols, np.int64), np.array(rows, np.int64))) if rows else []
    return (np.array(rows, np.int32)[order], np.array(cols, np.int32)[order],
            np.array(vals, dtype=np.asarray(sell["val"]).dtype)[order])


def bell_to_dense(bell: dict, n_rows: int, n_cols: int) -> np.ndarray:
    """Dense matrix a BELL layout stores (stored zeros and absent entries alike 0)."""
    b, K, pitch = bell["b"], bell["K"], bell["pitch"]
    d = np.zeros((bell["n_block_rows"] * b, (n_cols // b + 1) * b))
    for k in range(K):
        for i in range(bell["n_block_rows"]):
            bc = int(bell["bcol"][k * pitch + i])
            if bc < 0:
                continue
            blk = bell["bval"][(k * pitch + i) * b * b:(k * pitch + i + 1) * b * b].reshape(b, b)
            d[i * b:(i + 1) * b, bc * b:(bc + 1) * b] = blk
    return d[:n_rows, :n_cols]


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
