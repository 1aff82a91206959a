"""Pins for the oracle's ingest, format layouts and sparsity features (CPU only).

Each check fixes the oracle to something other than itself: Python's tuple
sort and counting, dense reconstruction, hand-derived layouts, closed forms of
structured matrices, and the feature values the paper prints for its own
matrices (tests/golden/paper_matrix_features.csv).
"""
import collections
import csv
import itertools
import math
import os

import numpy as np
import pytest

import synth
from oracle import formats as F

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _canon_of(m, dtype=np.float64, seed=0):
    r, c, perm = synth.shuffled(m, seed)
    v = m.values(dtype)[perm]
    return F.canonicalize(m.n_rows, m.n_cols, r, c, v)


# ---- ingest --------------------------------------------------------------------

def test_canonicalize_rejects_bad_input():
    with pytest.raises(F.OracleError) as e:
        F.canonicalize(3, 3, [0, 3], [0, 0], [1.0, 2.0])
    assert e.value.status == F.OUT_OF_BOUNDS
    with pytest.raises(F.OracleError) as e:
        F.canonicalize(3, 3, [0, 1], [0, -1], [1.0, 2.0])
    assert e.value.status == F.OUT_OF_BOUNDS
    with pytest.raises(F.OracleError) as e:
        F.canonicalize(3, 3, [1, 0, 1], [2, 0, 2], [1.0, 2.0, 3.0])
    assert e.value.status == F.DUPLICATE
    with pytest.raises(F.OracleError) as e:
        F.canonicalize(-1, 3, [], [], [])
    assert e.value.status == F.INVALID_ARG


def test_canonical_order_matches_tuple_sort():
    rng = np.random.default_rng(5)
    n_rows, n_cols, nnz = 37, 23, 300
    flat = rng.choice(n_rows * n_cols, nnz, replace=False)
    row, col = np.divmod(flat, n_cols)
    val = rng.standard_normal(nnz)
    c = F.canonicalize(n_rows, n_cols, row, col, val)
    expect = sorted(zip(row.tolist(), col.tolist(), val.tolist()))
    assert list(zip(c["row"].tolist(), c["col"].tolist(), c["val"].tolist())) == expect
    counts = collections.Counter(row.tolist())
    rp = [0]
    for i in range(n_rows):
        rp.append(rp[-1] + counts.get(i, 0))
    assert c["row_ptr"].tolist() == rp
    assert np.array_equal(c["val"], val[c["perm"]])


def test_explicit_zeros_are_stored_entries():
    c = F.canonicalize(2, 2, [1, 0], [0, 1], [0.0, 5.0])
    assert c["row_ptr"].tolist() == [0, 1, 2]
    assert c["val"].tolist() == [5.0, 0.0]


def test_empty_matrices():
    c = F.canonicalize(0, 0, [], [], np.zeros(0))
    assert c["row_ptr"].tolist() == [0]
    c = F.canonicalize(5, 7, [], [], np.zeros(0))
    assert c["row_ptr"].tolist() == [0] * 6
    e = F.to_ell(c)
    assert e["K"] == 0 and e["pitch"] == 64 and e["ell_col"].size == 0
    h = F.to_hyb(c)
    assert h["K"] == 0 and h["tail_row"].size == 0
    f = F.features(c)
    assert f.tolist() == [5, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0]


# ---- layouts ---------------------------------------------------------------------

def test_hand_written_ell_layout():
    # 3 x 4: row 0 holds (0,1)=a, (0,3)=b; row 1 empty; row 2 holds (2,0)=c.
    a, b, cc = 1.5, -2.0, 3.25
    canon = F.canonicalize(3, 4, [2, 0, 0], [0, 3, 1], [cc, b, a])
    assert canon["row_ptr"].tolist() == [0, 2, 2, 3]
    assert canon["col"].tolist() == [1, 3, 0]
    h = F.to_hyb(canon, k_override=2)  # the ELL part at full width is the plain ELL layout
    assert h["pitch"] == 64 and h["K"] == 2
    want_col = np.full(128, -1, np.int32)
    want_val = np.zeros(128)
    want_col[0], want_val[0] = 1, a          # slot (row 0, k 0)
    want_col[64], want_val[64] = 3, b        # slot (row 0, k 1)
    want_col[2], want_val[2] = 0, cc         # slot (row 2, k 0)
    assert np.array_equal(h["ell_col"], want_col)
    assert np.array_equal(h["ell_val"], want_val)
    assert h["tail_row"].size == 0
    h1 = F.to_hyb(canon, k_override=1)
    assert h1["tail_row"].tolist() == [0] and h1["tail_col"].tolist() == [3]
    assert h1["tail_val"].tolist() == [b]
    # ELL proper is refused: 64 * 2 padded slots > 8 * 3 entries
    with pytest.raises(F.OracleError) as e:
        F.to_ell(canon)
    assert e.value.status == F.NOT_APPLICABLE


@pytest.mark.parametrize("n_rows,n_cols", [(3, 3)])
def test_every_3x3_pattern_reconstructs(n_rows, n_cols):
    rng = np.random.default_rng(7)
    cells = list(itertools.product(range(n_rows), range(n_cols)))
    for mask in range(1 << len(cells)):
        on = [cells[i] for i in range(len(cells)) if mask >> i & 1]
        rng.shuffle(on)
        row = np.array([p[0] for p in on], np.int64)
        col = np.array([p[1] for p in on], np.int64)
        val = rng.standard_normal(len(on))
        dense = np.zeros((n_rows, n_cols))
        dense[row, col] = val
        canon = F.canonicalize(n_rows, n_cols, row, col, val)
        csr_rows = F.csr_to_coo_rows(canon["row_ptr"])
        assert np.array_equal(F.to_dense(n_rows, n_cols, csr_rows, canon["col"], canon["val"]), dense)
        assert np.array_equal(canon["row"], csr_rows)
        lengths = F.row_lengths(canon["row_ptr"])
        for k in range(0, 4):
            h = F.to_hyb(canon, k_override=k)
            er, ec, ev = F.ell_to_coo(h, n_rows)
            assert np.all(np.bincount(er, minlength=n_rows) == np.minimum(lengths, k))
            d = F.to_dense(n_rows, n_cols, er, ec, ev) + F.to_dense(
                n_rows, n_cols, h["tail_row"], h["tail_col"], h["tail_val"])
            assert np.array_equal(d, dense)
            # padding slots: column -1 and value +0.0
            pad = h["ell_col"] < 0
            assert np.all(h["ell_val"][pad] == 0) and not np.any(np.signbit(h["ell_val"][pad]))


@pytest.mark.parametrize("gen", [
    lambda: synth.poisson_random(300, 8.0, 11),
    lambda: synth.banded(257, 5),
    lambda: synth.laplacian2d(20),
    lambda: synth.power_law(500, 12, cap=300),
])
def test_round_trips(gen):
    m = gen()
    canon = _canon_of(m, np.float32, seed=3)
    # COO -> CSR -> COO
    assert np.array_equal(F.csr_to_coo_rows(canon["row_ptr"]), m.row)
    assert np.array_equal(canon["col"], m.col)
    assert np.array_equal(canon["val"], m.values(np.float32))
    # CSR -> HYB -> COO at the rule's width
    h = F.to_hyb(canon)
    er, ec, ev = F.ell_to_coo(h, m.n_rows)
    r = np.concatenate([er, h["tail_row"]])
    c = np.concatenate([ec, h["tail_col"]])
    v = np.concatenate([ev, h["tail_val"]])
    o = np.lexsort((c, r))
    assert np.array_equal(r[o], m.row) and np.array_equal(c[o], m.col)
    assert np.array_equal(v[o], m.values(np.float32))
    # CSR -> ELL -> COO where ELL is allowed
    try:
        e = F.to_ell(canon)
    except F.OracleError as err:
        assert err.status == F.NOT_APPLICABLE
        assert m.family == "powerlaw"
        return
    er, ec, ev = F.ell_to_coo(e, m.n_rows)
    assert np.array_equal(er, m.row) and np.array_equal(ec, m.col)
    assert np.array_equal(ev, m.values(np.float32))
    assert e["ell_col"].size == e["pitch"] * e["K"]


def test_laplacian_layout_counts():
    m = synth.config1_matrix()
    canon = _canon_of(m)
    lengths = F.row_lengths(canon["row_ptr"])
    assert dict(collections.Counter(lengths.tolist())) == {3: 4, 4: 248, 5: 3844}
    e = F.to_ell(canon)
    assert e["K"] == 5 and e["pitch"] == 4096
    assert int((e["ell_col"] < 0).sum()) == 5 * 4096 - 20224 == 256
    h = F.to_hyb(canon)
    # T = 4096 rows; every row has >= 3 entries but only 4092 have >= 4
    assert h["K"] == 3 and h["tail_row"].size == 248 * 1 + 3844 * 2 == 7936


def test_ell_fill_cap():
    pl = synth.power_law(4096, 5, cap=4000)
    with pytest.raises(F.OracleError) as e:
        F.to_ell(_canon_of(pl))
    assert e.value.status == F.NOT_APPLICABLE
    F.to_ell(_canon_of(synth.poisson_random(4096, 8.0, 5)))  # allowed


def _lengths_canon(lengths, n_cols=None):
    lengths = np.asarray(lengths, np.int64)
    n = lengths.size
    n_cols = n_cols or max(1, int(lengths.max(initial=0)))
    row = np.repeat(np.arange(n), lengths)
    starts = np.concatenate([[0], np.cumsum(lengths)])
    col = np.arange(row.size) - starts[row]
    return F.canonicalize(n, n_cols, row, col, np.ones(row.size))


@pytest.mark.parametrize("lengths,want", [
    ([2] * 5000 + [10] * 4000, 2),            # T = 4096: only 4000 rows reach 3
    ([10] * 4096 + [1] * 4904, 10),           # exactly T rows reach 10
    ([5] * 9999 + [1] * 20001, 1),            # T = ceil(30000/3) = 10000 > 9999
    ([5] * 10000 + [1] * 20000, 5),           # T = 10000 rows reach 5
    ([3, 7, 4, 9, 5, 6], 3),                  # small n: T = n, width = shortest row
    ([0, 4, 4], 0),
])
def test_hyb_width_rule(lengths, want):
    canon = _lengths_canon(lengths)
    assert F.hyb_width(F.row_lengths(canon["row_ptr"]), canon["n_rows"]) == want
    h = F.to_hyb(canon)
    assert h["K"] == want
    assert h["tail_row"].size == int(np.maximum(np.asarray(lengths) - want, 0).sum())


# ---- features ----------------------------------------------------------------------

def test_features_laplacian_closed_form():
    f = F.features(_canon_of(synth.config1_matrix()))
    # lengths {3: 4, 4: 248, 5: 3844}; E[l] = 20224/4096, E[l^2] = 100104/4096
    want = {
        "n": 4096, "nnz": 20224, "mean": 4.9375, "var": 100104 / 4096 - 4.9375 ** 2,
        "median": 5, "mode": 5, "ell_ratio": 20224 / (4096 * 5), "max": 5, "bandwidth": 64,
        "fill": 20224 / 4096 ** 2, "hyb_coo_frac": 7936 / 20224,
    }
    for k, v in want.items():
        assert f[F.FEATURE_NAMES.index(k)] == pytest.approx(v, rel=1e-15, abs=0), k
    assert want["var"] == 0.060546875
    assert f[4] == pytest.approx(math.sqrt(0.060546875), rel=1e-15)


def test_features_structured_families():
    bd = F.features(_canon_of(synth.block_diagonal(8 * 700)))
    assert bd[3] == 0 and bd[5] == 8 and bd[6] == 8 and bd[7] == 1 and bd[8] == 8 and bd[9] == 7
    assert bd[11] == 0
    n, b = 1000, 6
    fb = F.features(_canon_of(synth.banded(n, b)))
    assert fb[1] == n * (2 * b + 1) - b * (b + 1) and fb[9] == b and fb[8] == 2 * b + 1
    assert fb[6] == 2 * b + 1
    g = 9
    st = _canon_of(synth.stencil3d(g))
    cnt = collections.Counter(F.row_lengths(st["row_ptr"]).tolist())
    assert cnt == {7: (g - 2) ** 3, 6: 6 * (g - 2) ** 2, 5: 12 * (g - 2), 4: 8}
    assert F.features(st)[9] == g * g


def test_median_and_mode_conventions():
    c = _lengths_canon([1, 2, 3, 4])
    f = F.features(c)
    assert f[5] == 2.5
    c = _lengths_canon([3, 1, 1, 2, 2])
    f = F.features(c)
    assert f[6] == 1 and f[5] == 2
    c = _lengths_canon([0, 0, 7])
    f = F.features(c)
    assert f[5] == 0 and f[6] == 0 and f[7] == pytest.approx(7 / 21)


def _paper_rows():
    path = os.path.join(GOLDEN, "paper_matrix_features.csv")
    with open(path) as fh:
        rows = list(csv.DictReader(l for l in fh if not l.startswith("#")))
    return [{k: (v if k == "name" else float(v)) for k, v in r.items()} for r in rows]


def test_paper_printed_features_agree_with_definitions():
    """The paper's printed table fixes mean = nnz/n, std^2 = var and ELL_ratio = nnz/(n*max).

    For every row whose printed values are self-consistent, a matrix with the
    same n, nnz and longest row (max = Avg / ELL_ratio, an integer) is built
    and the oracle must reproduce the printed Avg and ELL_ratio.
    """
    rows = _paper_rows()
    checked = 0
    for r in rows:
        if r["var"] > 0:
            assert r["sd"] ** 2 == pytest.approx(r["var"], rel=1e-5), r["name"]
        if r["ell_ratio"] <= 0 or abs(r["avg"] - r["nnz"] / r["n"]) > 1e-6 * r["avg"]:
            continue  # garbled rows (Avg printed as 0, negative ratio, Avg off nnz/n)
        mx = r["avg"] / r["ell_ratio"]
        if abs(mx - round(mx)) > 1e-3:
            continue
        mx = int(round(mx))
        n, nnz = int(r["n"]), int(r["nnz"])
        rest, k = divmod(nnz - mx, n - 1)
        lengths = np.full(n - 1, rest, np.int64)
        lengths[:k] += 1
        lengths = np.concatenate([[mx], lengths])
        assert lengths.max() == mx and lengths.sum() == nnz
        f = F.features(_lengths_canon(lengths, n_cols=mx))
        assert f[2] == pytest.approx(r["avg"], rel=1e-6), r["name"]
        assert f[7] == pytest.approx(r["ell_ratio"], rel=2e-5), r["name"]
        checked += 1
    assert checked == 24  # 6 of the 30 printed rows are garbled or rounded too coarsely


def test_transform_features():
    # The selector input takes log2(1 + v) of the count and length features, the
    # 1-based feature columns 1-7 (n, nnz, mean, var, std, median, mode), 9 (max)
    # and 10 (bandwidth); columns 8 (ELL ratio), 11 (fill) and 12 (HYB tail
    # fraction) are ratios and stay raw. The list is written out here, not read
    # from the oracle.
    log_cols_1based = [1, 2, 3, 4, 5, 6, 7, 9, 10]
    f = np.array([7.0, 31.0, 3.0, 15.0, 0.5, 1.0, 63.0, 0.25, 255.0, 1023.0, 0.125, 0.75])
    t = F.transform_features(f)
    for i in range(12):
        want = math.log2(1 + f[i]) if (i + 1) in log_cols_1based else f[i]
        assert t[i] == pytest.approx(want, rel=1e-15), i + 1
    assert t.tolist() == [3.0, 5.0, 2.0, 4.0, math.log2(1.5), 1.0, 6.0, 0.25, 8.0, 10.0, 0.125, 0.75]
    # batched rows are transformed column by column in the same way
    assert np.array_equal(F.transform_features(np.stack([f, f]))[1], t)
