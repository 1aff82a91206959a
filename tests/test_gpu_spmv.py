"""GPU SpMV parity: every format, every compiled variant, FP32 and FP64, against the oracle.

The bar is the per-row error |y - y_ref| / (|alpha| sum_j |a_ij x_j| + |beta y_i|):
at most 1e-5 for FP32 and 1e-12 for FP64, with exact equality where the
denominator is 0. Integer-valued problems must match bit for bit.
"""
import math

import numpy as np
import pytest

import _cases as C
import synth
from oracle import formats as OF
from oracle import spmv as OS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2302_05662_amd as S  # noqa: E402

DTYPES = [np.float32, np.float64]
FORMATS = [S.SPMV_FMT_CSR, S.SPMV_FMT_COO, S.SPMV_FMT_ELL, S.SPMV_FMT_HYB, S.SPMV_FMT_SELL,
           S.SPMV_FMT_BELL]


def _create(name, dtype):
    m = C.matrix(name)
    r, c, v = C.shuffled_input(name, dtype)
    return S.spmv_create(m.n_rows, m.n_cols, r, c, v)


def _set_variant(h, fmt, var):
    """Set a variant; False when it does not apply to this matrix (its reordered copy
    cannot be built, e.g. column-split COO on a matrix with one column panel)."""
    try:
        S.spmv_set_variant(h, fmt, var)
        return True
    except S.SpmvError as e:
        if e.status != "NOT_APPLICABLE":
            raise
        return False


def _formats_for(h, name, dtype):
    """Every format the oracle says applies, converted on h (SELL and BELL by their rules)."""
    out = [S.SPMV_FMT_CSR, S.SPMV_FMT_COO]
    ref = C.canonical(name, dtype)
    for fmt, build in ((S.SPMV_FMT_ELL, OF.to_ell), (S.SPMV_FMT_HYB, OF.to_hyb),
                       (S.SPMV_FMT_SELL, OF.to_sell), (S.SPMV_FMT_BELL, OF.to_bell)):
        try:
            build(ref)
        except OF.OracleError as e:
            assert e.status == OF.NOT_APPLICABLE
            with pytest.raises(S.SpmvError) as got:
                S.spmv_convert(h, fmt)
            assert got.value.status == "NOT_APPLICABLE", (name, S.FORMAT_NAMES[fmt])
            continue
        S.spmv_convert(h, fmt)
        out.append(fmt)
    return out


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("name", list(C.CASES))
def test_every_variant_matches_oracle(name, dtype):
    print(f"[spmv] {name} {dtype.__name__}", flush=True)
    m = C.matrix(name)
    h = _create(name, dtype)
    x, y0 = C.vectors(name, dtype)
    xd = torch.from_numpy(x).cuda()
    runs = []
    for fmt in _formats_for(h, name, dtype):
        for var in range(S.spmv_variant_count(fmt, h.dtype_code)):
            if not _set_variant(h, fmt, var):
                continue
            for a, b in C.ALPHA_BETA:
                yd = torch.from_numpy(y0.copy()).cuda()
                S.spmv_run(h, fmt, a, xd, b, yd)
                runs.append((fmt, var, a, b, yd))
    torch.cuda.synchronize()
    tol = C.TOL[dtype]
    for fmt, var, a, b, yd in runs:
        y_ref, den = C.reference(name, dtype, a, b)
        err = OS.max_row_error(yd.cpu().numpy(), y_ref, den)
        assert err <= tol, (S.FORMAT_NAMES[fmt], S.spmv_variant_describe(fmt, h.dtype_code, var), a, b, err)
    assert m.n_rows == 0 or runs


SELL_BELL_CASES = ["random", "powerlaw", "banded", "blockdiag", "stencil", "wide", "tall",
                   "one_long_row", "last_row_only", "single", "empty", "lap64"]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("name", SELL_BELL_CASES)
def test_sell_and_bell_layouts_every_variant(name, dtype):
    """SELL at sigma 1, 128 and 16384 and BELL at 2, 4 and 8: every variant, every (alpha, beta)."""
    print(f"[spmv sell/bell] {name} {dtype.__name__}", flush=True)
    m = C.matrix(name)
    h = _create(name, dtype)
    ref = C.canonical(name, dtype)
    x, y0 = C.vectors(name, dtype)
    xd = torch.from_numpy(x).cuda()
    tol = C.TOL[dtype]
    layouts = [(S.SPMV_FMT_SELL, p, OF.to_sell) for p in (1, 128, 16384)] + \
              [(S.SPMV_FMT_BELL, p, OF.to_bell) for p in (2, 4, 8)]
    ran = built = 0
    for fmt, param, build in layouts:
        try:
            build(ref, param)
        except OF.OracleError as e:
            assert e.status == OF.NOT_APPLICABLE
            with pytest.raises(S.SpmvError) as got:
                S.spmv_convert(h, fmt, param)
            assert got.value.status == "NOT_APPLICABLE"
            continue
        S.spmv_convert(h, fmt, param)
        built += 1
        for var in range(S.spmv_variant_count(fmt, h.dtype_code)):
            if not _set_variant(h, fmt, var):
                d = S.spmv_variant_describe(fmt, h.dtype_code, var)
                assert fmt == S.SPMV_FMT_BELL and d["lanes"] > param  # more rows than the block
                continue
            for a, b in C.ALPHA_BETA:
                yd = torch.from_numpy(y0.copy()).cuda()
                S.spmv_run(h, fmt, a, xd, b, yd)
                y_ref, den = C.reference(name, dtype, a, b)
                err = OS.max_row_error(yd.cpu().numpy(), y_ref, den)
                assert err <= tol, (S.FORMAT_NAMES[fmt], param, var, a, b, err)
                ran += 1
    assert ran > 0 or built == 0 or m.nnz == 0 or m.n_rows == 0


def test_laplacian_integer_closed_form_bit_exact():
    """x = i^2 + j^2 on the 64 x 64 grid: A x = -4 + sum of x over missing neighbours."""
    g = 64
    m = C.matrix("lap64")
    h = _create("lap64", np.float32)
    i, j = np.divmod(np.arange(g * g), g)
    x = (i * i + j * j).astype(np.float32)
    want = []
    for a, b in zip(i.tolist(), j.tolist()):
        s = -4
        for p, q in ((a - 1, b), (a + 1, b), (a, b - 1), (a, b + 1)):
            if not (0 <= p < g and 0 <= q < g):
                s += p * p + q * q
        want.append(s)
    want = np.array(want, np.float32)
    xd = torch.from_numpy(x).cuda()
    for fmt in _formats_for(h, "lap64", np.float32):
        for var in range(S.spmv_variant_count(fmt, S.SPMV_F32)):
            if not _set_variant(h, fmt, var):
                continue
            yd = torch.empty(m.n_rows, device="cuda")
            S.spmv_run(h, fmt, 1.0, xd, 0.0, yd)
            assert np.array_equal(yd.cpu().numpy(), want), (S.FORMAT_NAMES[fmt], var)


@pytest.mark.parametrize("dtype", DTYPES)
def test_beta_zero_ignores_nan_and_runs_are_deterministic(dtype):
    name = "powerlaw"
    m = C.matrix(name)
    h = _create(name, dtype)
    x, _ = C.vectors(name, dtype)
    xd = torch.from_numpy(x).cuda()
    y_ref, den = C.reference(name, dtype, 1.0, 0.0)
    for fmt in _formats_for(h, name, dtype):
        for var in range(S.spmv_variant_count(fmt, h.dtype_code)):
            if not _set_variant(h, fmt, var):
                continue
            y1 = torch.full((m.n_rows,), float("nan"), dtype=xd.dtype, device="cuda")
            y2 = torch.full((m.n_rows,), float("inf"), dtype=xd.dtype, device="cuda")
            S.spmv_run(h, fmt, 1.0, xd, 0.0, y1)
            S.spmv_run(h, fmt, 1.0, xd, 0.0, y2)
            a, b = y1.cpu().numpy(), y2.cpu().numpy()
            # the sorted-block COO kernel (also the tail of the HYB variants with
            # pipelined = 1) adds with LDS atomics in no fixed order
            d = S.spmv_variant_describe(fmt, h.dtype_code, var)
            if d["kernel"] != "coo_sorted" and not (d["kernel"] == "hyb" and d["pipelined"] == 1):
                assert a.tobytes() == b.tobytes()
            assert OS.max_row_error(a, y_ref, den) <= C.TOL[dtype]


def _sample_rows(row_ptr, n, seed, k=3000):
    lengths = np.diff(row_ptr)
    rng = np.random.default_rng(seed)
    pick = rng.choice(n, min(k, n), replace=False)
    longest = np.argsort(lengths)[-50:]
    return np.unique(np.concatenate([pick, longest, [0, n - 1]]))


@pytest.mark.parametrize("which", ["powerlaw_2M_f32", "random_f64"])
def test_full_size_sampled_rows(which):
    """Full-size matrices, all variants, checked on sampled rows (incl. the longest)."""
    if which == "powerlaw_2M_f32":
        m, dtype = synth.config3_matrix(), np.float32
    else:
        m, dtype = synth.config2_matrix(2009), np.float64
    print(f"[spmv full] {m.name} nnz={m.nnz} {dtype.__name__}", flush=True)
    v = m.values(dtype)
    x = m.x(dtype)
    y0 = synth.uniform_vector(m.n_rows, dtype, [m.seed, 4])
    h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, v)
    row_ptr = np.zeros(m.n_rows + 1, np.int64)
    np.cumsum(np.bincount(m.row, minlength=m.n_rows), out=row_ptr[1:])
    rows = _sample_rows(row_ptr, m.n_rows, 7)
    a, b = 1.5, -0.5
    y_ref, den = OS.spmv_rows(rows, row_ptr, m.col, v, x, a, b, y0)
    xd = torch.from_numpy(x).cuda()
    fmts = [S.SPMV_FMT_CSR, S.SPMV_FMT_COO, S.SPMV_FMT_HYB]
    try:
        S.spmv_convert(h, S.SPMV_FMT_ELL)
        fmts.append(S.SPMV_FMT_ELL)
    except S.SpmvError as e:
        assert e.status == "NOT_APPLICABLE"
    S.spmv_convert(h, S.SPMV_FMT_HYB)
    rows_t = torch.from_numpy(rows).cuda()
    for fmt in fmts:
        for var in range(S.spmv_variant_count(fmt, h.dtype_code)):
            if not _set_variant(h, fmt, var):
                continue
            yd = torch.from_numpy(y0).cuda()
            S.spmv_run(h, fmt, a, xd, b, yd)
            got = yd[rows_t].cpu().numpy()
            err = OS.max_row_error(got, y_ref, den)
            assert err <= C.TOL[dtype], (S.FORMAT_NAMES[fmt], var, err)
            assert math.isfinite(err)


@pytest.mark.parametrize("dtype", DTYPES)
def test_panel_variants_with_unaligned_x(dtype):
    """The streaming COO kernels give the same bits for x at any 4-byte alignment."""
    name = "wide"
    m = C.matrix(name)
    print(f"[spmv panel unaligned] {name} {dtype.__name__}", flush=True)
    h = _create(name, dtype)
    x, y0 = C.vectors(name, dtype)
    xd = torch.from_numpy(x).cuda()
    buf = torch.zeros(m.n_cols + 1, dtype=xd.dtype, device="cuda")
    buf[1:] = xd
    xu = buf[1:]
    assert xu.data_ptr() % 16 != 0
    a, b = C.ALPHA_BETA[1]
    y_ref, den = C.reference(name, dtype, a, b)
    panel = [v for v in range(S.spmv_variant_count(S.SPMV_FMT_COO, h.dtype_code))
             if S.spmv_variant_describe(S.SPMV_FMT_COO, h.dtype_code, v)["kernel"] == "coo_panel"]
    assert panel
    for var in panel:
        S.spmv_set_variant(h, S.SPMV_FMT_COO, var)
        ya = torch.from_numpy(y0.copy()).cuda()
        yu = torch.from_numpy(y0.copy()).cuda()
        S.spmv_run(h, S.SPMV_FMT_COO, a, xd, b, ya)
        S.spmv_run(h, S.SPMV_FMT_COO, a, xu, b, yu)
        ga, gu = ya.cpu().numpy(), yu.cpu().numpy()
        assert ga.tobytes() == gu.tobytes(), var
        assert OS.max_row_error(ga, y_ref, den) <= C.TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_column_tiles_with_unaligned_y(dtype):
    """The column-tile variants add the second half's row sums into y with 16-byte
    accesses when y allows them and one row at a time otherwise: y at an offset of one
    value gives a result within the bound, and rows past y's end stay untouched."""
    name = "random"
    m = C.matrix(name)
    print(f"[spmv tiles unaligned y] {name} {dtype.__name__}", flush=True)
    h = _create(name, dtype)
    x, y0 = C.vectors(name, dtype)
    xd = torch.from_numpy(x).cuda()
    a, b = C.ALPHA_BETA[1]
    y_ref, den = C.reference(name, dtype, a, b)
    tiles = [v for v in range(S.spmv_variant_count(S.SPMV_FMT_COO, h.dtype_code))
             if S.spmv_variant_describe(S.SPMV_FMT_COO, h.dtype_code, v)["ksplit"] > 1]
    assert tiles
    for var in tiles:
        S.spmv_set_variant(h, S.SPMV_FMT_COO, var)
        buf = torch.full((m.n_rows + 2,), 7.0, dtype=xd.dtype, device="cuda")
        buf[1:m.n_rows + 1] = torch.from_numpy(y0.copy()).cuda()
        yu = buf[1:m.n_rows + 1]
        assert yu.data_ptr() % 16 != 0
        S.spmv_run(h, S.SPMV_FMT_COO, a, xd, b, yu)
        g = buf.cpu().numpy()
        assert g[0] == 7.0 and g[-1] == 7.0, var
        assert OS.max_row_error(g[1:-1], y_ref, den) <= C.TOL[dtype], var


def test_four_column_tiles_refused_past_the_lds_rows():
    """Four column tiles need blocks of 4 n / 256 rows, at most 16384 (the FP64 row sums of a
    block fill 128 KB of LDS): a 1.1M-row matrix is refused four tiles (NOT_APPLICABLE) and
    runs in two, within the bound of the oracle."""
    n_rows, n_cols = 1_100_000, 4000
    rng = np.random.default_rng(44)
    row = np.arange(n_rows, dtype=np.int64)
    col = rng.integers(0, n_cols, n_rows)
    m = synth.from_coords("tall_single", n_rows, n_cols, row, col, 45)
    v = m.values(np.float32)
    print(f"[spmv tiles limit] {n_rows} x {n_cols}", flush=True)
    h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, v)
    x = synth.uniform_vector(n_cols, np.float32, [44, 3])
    xd = torch.from_numpy(x).cuda()
    c = OF.canonicalize(n_rows, n_cols, m.row, m.col, v)
    y_ref = OS.spmv_csr(c["row_ptr"], c["col"], c["val"], x, np.float32(1.0), np.float32(0.0), None)
    den = OS.row_denominator(c["row_ptr"], c["col"], c["val"], x, np.float32(1.0), np.float32(0.0), None)
    by_tiles = {}
    for i in range(S.spmv_variant_count(S.SPMV_FMT_COO, h.dtype_code)):
        d = S.spmv_variant_describe(S.SPMV_FMT_COO, h.dtype_code, i)
        if d["kernel"] == "coo_sorted" and d["ksplit"] > 1:
            by_tiles.setdefault(d["ksplit"], []).append(i)
    assert sorted(by_tiles) == [2, 4]
    for var in by_tiles[4]:
        with pytest.raises(S.SpmvError) as e:
            S.spmv_set_variant(h, S.SPMV_FMT_COO, var)
        assert e.value.status == "NOT_APPLICABLE"
    for var in by_tiles[2]:
        S.spmv_set_variant(h, S.SPMV_FMT_COO, var)
        yd = torch.zeros(n_rows, dtype=torch.float32, device="cuda")
        S.spmv_run(h, S.SPMV_FMT_COO, 1.0, xd, 0.0, yd)
        assert OS.max_row_error(yd.cpu().numpy(), y_ref, den) <= C.TOL[np.float32], var


def test_reordered_coo_layouts_at_their_column_limits():
    """Streaming COO packs columns in 23 bits and refuses wider matrices; sorted-block COO
    packs the row in the bits the column leaves free and still runs."""
    n_rows, n_cols = 3000, (1 << 23) + 5
    rng = np.random.default_rng(21)
    rows = np.repeat(np.arange(n_rows), 3)
    cols = np.concatenate([np.sort(rng.choice(n_cols, 3, replace=False)) for _ in range(n_rows)])
    cols[-1] = n_cols - 1  # the last column is used
    m = synth.from_coords("wide_cols", n_rows, n_cols, rows, cols, 22)
    print(f"[spmv wide cols] n_cols={n_cols}", flush=True)
    v = m.values(np.float32)
    h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, v)
    kinds = {i: S.spmv_variant_describe(S.SPMV_FMT_COO, S.SPMV_F32, i)["kernel"]
             for i in range(S.spmv_variant_count(S.SPMV_FMT_COO, S.SPMV_F32))}
    x = synth.uniform_vector(n_cols, np.float32, [22, 3])
    xd = torch.from_numpy(x).cuda()
    row_ptr = np.zeros(n_rows + 1, np.int64)
    np.cumsum(np.bincount(m.row, minlength=n_rows), out=row_ptr[1:])
    c = OF.canonicalize(n_rows, n_cols, m.row, m.col, v)
    y_ref = OS.spmv_csr(c["row_ptr"], c["col"], c["val"], x, np.float32(1.0), np.float32(0.0), None)
    den = OS.row_denominator(c["row_ptr"], c["col"], c["val"], x, np.float32(1.0), np.float32(0.0), None)
    for i, k in kinds.items():
        if k == "coo_panel":
            with pytest.raises(S.SpmvError) as e:
                S.spmv_set_variant(h, S.SPMV_FMT_COO, i)
            assert e.value.status == "NOT_APPLICABLE"
        elif k == "coo_sorted":
            S.spmv_set_variant(h, S.SPMV_FMT_COO, i)
            yd = torch.zeros(n_rows, dtype=torch.float32, device="cuda")
            S.spmv_run(h, S.SPMV_FMT_COO, 1.0, xd, 0.0, yd)
            assert OS.max_row_error(yd.cpu().numpy(), y_ref, den) <= C.TOL[np.float32]
    # tuning skips the variants that do not apply and keeps a runnable one
    yd = torch.zeros(n_rows, dtype=torch.float32, device="cuda")
    var, _ = S.spmv_tune(h, S.SPMV_FMT_COO, xd, yd, reps=2, flush=False)
    assert kinds[var] != "coo_panel"


@pytest.mark.parametrize("dtype", DTYPES)
def test_sorted_block_rows_beside_wide_columns(dtype):
    """Columns too wide to leave the block's rows any room in the packed index: the
    sorted-block layout keeps the row inside the block in 16 bits beside the column."""
    n_rows, n_cols = 20011, (1 << 26) + 3
    rng = np.random.default_rng(31)
    lengths = rng.integers(0, 9, n_rows)
    lengths[[0, 777, n_rows - 1]] = [0, 0, 6]  # empty rows and a full last row
    rows = np.repeat(np.arange(n_rows), lengths)
    cols = np.concatenate([np.sort(rng.choice(n_cols, k, replace=False)) for k in lengths])
    cols[-1] = n_cols - 1
    m = synth.from_coords("wide_rows16", n_rows, n_cols, rows, cols, 32)
    print(f"[spmv rows16] n_cols={n_cols} nnz={m.nnz} {dtype.__name__}", flush=True)
    v = m.values(dtype)
    x = synth.uniform_vector(n_cols, dtype, [32, 3])
    y0 = synth.uniform_vector(n_rows, dtype, [32, 4])
    a, b = 0.75, -1.25
    c = OF.canonicalize(n_rows, n_cols, m.row, m.col, v)
    y_ref = OS.spmv_csr(c["row_ptr"], c["col"], c["val"], x, dtype(a), dtype(b), y0)
    den = OS.row_denominator(c["row_ptr"], c["col"], c["val"], x, dtype(a), dtype(b), y0)
    h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, v)
    xd = torch.from_numpy(x).cuda()
    sorted_vars = [i for i in range(S.spmv_variant_count(S.SPMV_FMT_COO, h.dtype_code))
                   if S.spmv_variant_describe(S.SPMV_FMT_COO, h.dtype_code, i)["kernel"] == "coo_sorted"]
    assert sorted_vars
    for var in sorted_vars:
        S.spmv_set_variant(h, S.SPMV_FMT_COO, var)
        yd = torch.from_numpy(y0.copy()).cuda()
        S.spmv_run(h, S.SPMV_FMT_COO, a, xd, b, yd)
        err = OS.max_row_error(yd.cpu().numpy(), y_ref, den)
        assert err <= C.TOL[dtype], (var, err)
    del xd


@pytest.mark.parametrize("dtype", DTYPES)
def test_sorted_blocks_with_long_rows_and_empty_runs(dtype):
    """Sorted-block COO with a few rows of 9K-20K entries (thousands of local atomic adds
    to one accumulator), scattered short rows and a run of 30K empty rows."""
    n_rows, n_cols = 100_003, 40_009
    rng = np.random.default_rng(51)
    lengths = np.zeros(n_rows, np.int64)
    lengths[rng.choice(n_rows, 3000, replace=False)] = rng.integers(1, 6, 3000)
    lengths[[7, 50_000, 50_001, n_rows - 1]] = [20_000, 15_000, 9, 12_000]
    lengths[60_000:90_000] = 0
    rows = np.repeat(np.arange(n_rows), lengths)
    cols = np.concatenate([np.sort(rng.choice(n_cols, k, replace=False)) for k in lengths])
    m = synth.from_coords("long_rows_empty_runs", n_rows, n_cols, rows, cols, 52)
    print(f"[spmv long rows] nnz={m.nnz} {dtype.__name__}", flush=True)
    v = m.values(dtype)
    x = synth.uniform_vector(n_cols, dtype, [52, 3])
    y0 = synth.uniform_vector(n_rows, dtype, [52, 4])
    a, b = -1.5, 0.5
    c = OF.canonicalize(n_rows, n_cols, m.row, m.col, v)
    y_ref = OS.spmv_csr(c["row_ptr"], c["col"], c["val"], x, dtype(a), dtype(b), y0)
    den = OS.row_denominator(c["row_ptr"], c["col"], c["val"], x, dtype(a), dtype(b), y0)
    h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, v)
    xd = torch.from_numpy(x).cuda()
    sorted_vars = [i for i in range(S.spmv_variant_count(S.SPMV_FMT_COO, h.dtype_code))
                   if S.spmv_variant_describe(S.SPMV_FMT_COO, h.dtype_code, i)["kernel"] == "coo_sorted"]
    for var in sorted_vars:
        S.spmv_set_variant(h, S.SPMV_FMT_COO, var)
        yd = torch.from_numpy(y0.copy()).cuda()
        S.spmv_run(h, S.SPMV_FMT_COO, a, xd, b, yd)
        err = OS.max_row_error(yd.cpu().numpy(), y_ref, den)
        assert err <= C.TOL[dtype], (var, err)


@pytest.mark.parametrize("dtype", DTYPES)
def test_csr_stream_rows_at_the_stage_size(dtype):
    """CSR stream row blocks: rows of 2043-2050 entries starting at every alignment (some fit
    the 2048-entry stage with their 4-aligned start, some get a workgroup of their own),
    runs of 1-entry rows longer than 256 rows (blocks capped at 256 rows), empty rows."""
    lengths = []
    for extra in range(4):  # shift the alignment of what follows
        lengths += [extra + 1] + [2043 + extra, 2044 + extra, 2045 + extra, 2046 + extra, 2047, 2048,
                                  2049, 2050, 0, 3]
    lengths += [1] * 700 + [0] * 300 + [5] * 600
    lengths = np.array(lengths, np.int64)
    n_rows, n_cols = len(lengths), 5003
    rng = np.random.default_rng(61)
    rows = np.repeat(np.arange(n_rows), lengths)
    cols = np.concatenate([np.sort(rng.choice(n_cols, k, replace=False)) for k in lengths])
    m = synth.from_coords("stage_edges", n_rows, n_cols, rows, cols, 62)
    print(f"[spmv csr stream edges] rows={n_rows} nnz={m.nnz} {dtype.__name__}", flush=True)
    v = m.values(dtype)
    x = synth.uniform_vector(n_cols, dtype, [62, 3])
    y0 = synth.uniform_vector(n_rows, dtype, [62, 4])
    a, b = 1.25, -0.75
    c = OF.canonicalize(n_rows, n_cols, m.row, m.col, v)
    y_ref = OS.spmv_csr(c["row_ptr"], c["col"], c["val"], x, dtype(a), dtype(b), y0)
    den = OS.row_denominator(c["row_ptr"], c["col"], c["val"], x, dtype(a), dtype(b), y0)
    h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, v)
    xd = torch.from_numpy(x).cuda()
    stream = [i for i in range(S.spmv_variant_count(S.SPMV_FMT_CSR, h.dtype_code))
              if S.spmv_variant_describe(S.SPMV_FMT_CSR, h.dtype_code, i)["kernel"] == "csr_stream"]
    assert len(stream) == 2
    for var in stream:
        S.spmv_set_variant(h, S.SPMV_FMT_CSR, var)
        for rep in range(2):  # deterministic: the same bits twice
            yd = torch.from_numpy(y0.copy()).cuda()
            S.spmv_run(h, S.SPMV_FMT_CSR, a, xd, b, yd)
            got = yd.cpu().numpy()
            if rep == 0:
                first = got.tobytes()
            assert got.tobytes() == first
        assert OS.max_row_error(got, y_ref, den) <= C.TOL[dtype], var


@pytest.mark.parametrize("dtype", DTYPES)
def test_hyb_sorted_tail_follows_a_new_split(dtype):
    """HYB variants that add the tail with the sorted-block kernel: right for several ELL
    widths, and a new spmv_convert of HYB (another width, so another tail) keeps the chosen
    variant runnable and right."""
    m = synth.power_law(20000, 71, cap=5000, value_dist="uniform")
    print(f"[spmv hyb sorted tail] nnz={m.nnz} {dtype.__name__}", flush=True)
    v = m.values(dtype)
    x = synth.uniform_vector(m.n_cols, dtype, [71, 3])
    y0 = synth.uniform_vector(m.n_rows, dtype, [71, 4])
    a, b = 1.5, -0.5
    c = OF.canonicalize(m.n_rows, m.n_cols, m.row, m.col, v)
    y_ref = OS.spmv_csr(c["row_ptr"], c["col"], c["val"], x, dtype(a), dtype(b), y0)
    den = OS.row_denominator(c["row_ptr"], c["col"], c["val"], x, dtype(a), dtype(b), y0)
    h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, v)
    xd = torch.from_numpy(x).cuda()
    tails = [i for i in range(S.spmv_variant_count(S.SPMV_FMT_HYB, h.dtype_code))
             if S.spmv_variant_describe(S.SPMV_FMT_HYB, h.dtype_code, i)["pipelined"] == 1]
    assert tails
    with pytest.raises(S.SpmvError) as e:  # the tail's copy needs a HYB split first
        S.spmv_set_variant(h, S.SPMV_FMT_HYB, tails[0])
    assert e.value.status == "NOT_CONVERTED"
    for k in (0, 1, 3, 8):
        S.spmv_convert(h, S.SPMV_FMT_HYB, k)
        for var in tails:
            S.spmv_set_variant(h, S.SPMV_FMT_HYB, var)
            yd = torch.from_numpy(y0.copy()).cuda()
            S.spmv_run(h, S.SPMV_FMT_HYB, a, xd, b, yd)
            assert OS.max_row_error(yd.cpu().numpy(), y_ref, den) <= C.TOL[dtype], (k, var)
    S.spmv_convert(h, S.SPMV_FMT_HYB, 2)  # the last variant stays set
    yd = torch.from_numpy(y0.copy()).cuda()
    S.spmv_run(h, S.SPMV_FMT_HYB, a, xd, b, yd)
    assert OS.max_row_error(yd.cpu().numpy(), y_ref, den) <= C.TOL[dtype]
