"""Pins for the oracle's SELL-C-sigma and BELL layouts (CPU only).

The paper's background section describes SELL (slices of a fixed number of
rows, each an ELL block as wide as its longest row, with slice pointers) and
BELL (ELL over dense blocks, default 2 x 2). These tests fix the oracle's
layouts to hand-written arrays, to dense reconstructions written here from the
layout definitions, and to closed forms of structured matrices.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import formats as F


def _canon(n_rows, n_cols, row, col, val):
    return F.canonicalize(n_rows, n_cols, np.asarray(row), np.asarray(col), np.asarray(val, np.float64))


def _sell_dense(sell, n_rows, n_cols, C, G):
    """Dense matrix read back from a SELL layout by its definition: slot k of the row at
    position l of slice s is slice_ptr[s] + (k // G) * C * G + l * G + k % G."""
    d = np.zeros((n_rows, n_cols))
    seen = 0
    for s in range(len(sell["slice_ptr"]) - 1):
        width = (sell["slice_ptr"][s + 1] - sell["slice_ptr"][s]) // C
        for l in range(C):
            for k in range(width):
                slot = sell["slice_ptr"][s] + (k // G) * C * G + l * G + k % G
                c = sell["col"][slot]
                if c < 0:
                    assert sell["val"][slot] == 0 and not np.signbit(sell["val"][slot])
                    continue
                p = s * C + l
                assert p < n_rows
                d[sell["perm"][p], c] = sell["val"][slot]
                seen += 1
    return d, seen


def _bell_dense(bell, n_rows, n_cols):
    b, K, pitch = bell["b"], bell["K"], bell["pitch"]
    d = np.zeros((pitch * b, (n_cols + b) // b * b + b))
    for k in range(K):
        for i in range(pitch):
            bc = bell["bcol"][k * pitch + i]
            base = (k * pitch + i) * b * b
            if bc < 0:
                assert not bell["bval"][base:base + b * b].any()
                continue
            for r in range(b):
                for c in range(b):
                    d[i * b + r, bc * b + c] = bell["bval"][base + r * b + c]
    assert not d[n_rows:].any() and not d[:, n_cols:].any()  # nothing outside the matrix
    return d[:n_rows, :n_cols]


# ---- SELL ------------------------------------------------------------------------

def test_hand_written_sell_layout():
    # 5 x 6, slice height 2, groups of 2 slots:
    # row 0: (0,1)=1 (0,4)=2 (0,5)=3; row 1: (1,0)=4; row 2: none;
    # row 3: (3,2)=5 (3,3)=6; row 4: (4,5)=7
    canon = _canon(5, 6, [0, 0, 0, 1, 3, 3, 4], [1, 4, 5, 0, 2, 3, 5], [1, 2, 3, 4, 5, 6, 7])
    s = F.to_sell(canon, sigma=1, C=2, G=2)
    # slice 0 (rows 0, 1): longest 3 -> width 4; slice 1 (rows 2, 3): 2; slice 2 (row 4): 1 -> 2
    assert s["slice_ptr"].tolist() == [0, 8, 12, 16]
    # slice 0, group 0: row 0 k0 k1, row 1 k0 k1; group 1: row 0 k2 k3, row 1 k2 k3
    assert s["col"].tolist() == [1, 4, 0, -1, 5, -1, -1, -1,
                                 -1, -1, 2, 3,
                                 5, -1, -1, -1]
    assert s["val"].tolist() == [1, 2, 4, 0, 3, 0, 0, 0, 0, 0, 5, 6, 7, 0, 0, 0]
    assert s["perm"].tolist() == [0, 1, 2, 3, 4]
    # sigma = 4: rows 0-3 by descending length (0: 3, 3: 2, 1: 1, 2: 0), row 4 alone
    t = F.to_sell(canon, sigma=4, C=2, G=2)
    assert t["perm"].tolist() == [0, 3, 1, 2, 4]
    # slice 0 holds rows 0 and 3 (width 4), slice 1 rows 1 and 2 (longest 1: width 2),
    # slice 2 row 4 and one padding position (width 2)
    assert t["slice_ptr"].tolist() == [0, 8, 12, 16]
    assert t["col"].tolist() == [1, 4, 2, 3, 5, -1, -1, -1,
                                 0, -1, -1, -1,
                                 5, -1, -1, -1]
    assert t["val"].tolist() == [1, 2, 5, 6, 3, 0, 0, 0, 4, 0, 0, 0, 7, 0, 0, 0]


def test_sell_order_is_a_stable_descending_sort_per_window():
    lengths = [1, 3, 2, 3, 0, 5]
    assert F.sell_order(lengths, 1).tolist() == [0, 1, 2, 3, 4, 5]
    assert F.sell_order(lengths, 4).tolist() == [1, 3, 2, 0, 5, 4]
    assert F.sell_order(lengths, 2).tolist() == [1, 0, 3, 2, 5, 4]


@pytest.mark.parametrize("C,G,sigma", [(2, 2, 1), (2, 2, 2), (2, 1, 1), (64, 4, 1), (64, 4, 16384)])
def test_every_3x3_pattern_through_sell(C, G, sigma):
    rng = np.random.default_rng(17)
    cells = list(itertools.product(range(3), range(3)))
    for mask in range(1 << 9):
        on = [cells[i] for i in range(9) if mask >> i & 1]
        row = np.array([p[0] for p in on], np.int64)
        col = np.array([p[1] for p in on], np.int64)
        val = rng.standard_normal(len(on))
        dense = np.zeros((3, 3))
        dense[row, col] = val
        s = F.to_sell(_canon(3, 3, row, col, val), sigma=sigma, C=C, G=G)
        got, seen = _sell_dense(s, 3, 3, C, G)
        assert np.array_equal(got, dense) and seen == len(on)
        assert sorted(s["perm"].tolist()) == [0, 1, 2]
        assert s["slice_ptr"][-1] == s["col"].size == s["val"].size
        assert all((s["slice_ptr"][i + 1] - s["slice_ptr"][i]) % (C * G) == 0
                   for i in range(len(s["slice_ptr"]) - 1))


@pytest.mark.parametrize("sigma", [1, 128, 16384])
def test_sell_default_shape_reconstructs(sigma):
    m = synth.poisson_random(1000, 9.0, 23)
    c = F.canonicalize(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float64))
    s = F.to_sell(c, sigma=sigma)
    got, seen = _sell_dense(s, m.n_rows, m.n_cols, 64, 4)
    assert seen == m.nnz
    assert np.array_equal(got, F.to_dense(m.n_rows, m.n_cols, c["row"], c["col"], c["val"]))


def test_sell_laplacian_closed_forms():
    m = synth.config1_matrix()
    canon = F.canonicalize(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float32))
    # natural order: a slice is one grid row; the first and last hold rows of 3 and 4
    # entries (width 4), the 62 others rows of 5 (width 8): 64*4 + 62*64*8 + 64*4
    s = F.to_sell(canon, sigma=1)
    assert s["n_slices"] == 64 and s["slice_ptr"][-1] == 32256
    assert int((s["col"] >= 0).sum()) == 20224
    # sorted in one window: 3844 rows of 5 fill 60 slices and 4 rows of the 61st (width
    # 8), the 248 rows of 4 and 4 rows of 3 leave three slices of width 4
    t = F.to_sell(canon, sigma=16384)
    assert t["slice_ptr"][-1] == 61 * 64 * 8 + 3 * 64 * 4 == 32000
    # bytes: 32256 * 8 = 258048 natural against 32000 * 8 + 4 * 4096 = 272384 sorted
    assert F.sell_sigma_rule(F.row_lengths(canon["row_ptr"]), 4) == 1
    assert F.to_sell(canon)["sigma"] == 1


def test_sell_sigma_rule_sorts_alternating_rows():
    # rows alternate 1 and 61 entries: natural slices all have width 64, sorted slices
    # half 64 and half 4, so sorting halves the slots and pays for the permutation
    n = 32768
    lengths = np.where(np.arange(n) % 2 == 0, 1, 61)
    rows = np.repeat(np.arange(n), lengths)
    cols = np.concatenate([np.arange(L) for L in lengths])
    canon = F.canonicalize(n, 64, rows, cols, np.ones(rows.size, np.float32))
    assert F.to_sell(canon, sigma=1)["slice_ptr"][-1] == n * 64
    t = F.to_sell(canon, sigma=16384)
    assert t["slice_ptr"][-1] == (n // 2) * 64 + (n // 2) * 4
    assert F.sell_sigma_rule(lengths, 4) == 16384 and F.to_sell(canon)["sigma"] == 16384
    # every window of 16384 rows starts with its 8192 long rows, in row order
    assert t["perm"][:3].tolist() == [1, 3, 5] and t["perm"][8192] == 0
    assert t["perm"][16384:16387].tolist() == [16385, 16387, 16389]


def test_sell_fill_cap_and_round_trip():
    pl = synth.power_law(4096, 5, cap=4000)
    canon = F.canonicalize(pl.n_rows, pl.n_cols, pl.row, pl.col, pl.values(np.float32))
    with pytest.raises(F.OracleError) as e:
        F.to_sell(canon, sigma=1)
    assert e.value.status == F.NOT_APPLICABLE
    for m in (synth.poisson_random(300, 8.0, 11), synth.banded(257, 5), synth.stencil3d(9, 3)):
        c = F.canonicalize(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float32))
        for sigma in (1, 128):
            r, cc, v = F.sell_to_coo(F.to_sell(c, sigma=sigma), m.n_rows)
            assert np.array_equal(r, m.row) and np.array_equal(cc, m.col)
            assert np.array_equal(v, m.values(np.float32))


# ---- BELL ------------------------------------------------------------------------

def test_hand_written_bell_layout():
    # 3 x 5 with 2 x 2 blocks: (0,0)=1 (0,3)=2 (1,1)=3 (2,4)=4
    # block row 0 (rows 0-1): block columns 0 {(0,0),(1,1)} and 1 {(0,3)}; block row 1
    # (row 2): block column 2 {(2,4)}. K = 2, pitch 64.
    canon = _canon(3, 5, [0, 0, 1, 2], [0, 3, 1, 4], [1, 2, 3, 4])
    b = F.to_bell(canon, 2)
    assert (b["b"], b["K"], b["pitch"], b["n_block_rows"]) == (2, 2, 64, 2)
    want_col = np.full(128, -1, np.int32)
    want_col[0], want_col[64], want_col[1] = 0, 1, 2
    assert np.array_equal(b["bcol"], want_col)
    want_val = np.zeros(128 * 4)
    want_val[0:4] = [1, 0, 0, 3]            # slot (0, 0): rows 0-1 x cols 0-1
    want_val[64 * 4:64 * 4 + 4] = [0, 2, 0, 0]  # slot (0, 1): rows 0-1 x cols 2-3
    want_val[4:8] = [4, 0, 0, 0]            # slot (1, 0): rows 2-3 x cols 4-5
    assert np.array_equal(b["bval"], want_val)


def test_every_3x3_pattern_through_bell():
    rng = np.random.default_rng(19)
    cells = list(itertools.product(range(3), range(3)))
    for mask in range(1 << 9):
        on = [cells[i] for i in range(9) if mask >> i & 1]
        row = np.array([p[0] for p in on], np.int64)
        col = np.array([p[1] for p in on], np.int64)
        val = rng.standard_normal(len(on))
        dense = np.zeros((3, 3))
        dense[row, col] = val
        for bs in (2, 4):
            bl = F.to_bell(_canon(3, 3, row, col, val), bs)
            assert np.array_equal(_bell_dense(bl, 3, 3), dense)
            blocks = {(r // bs, c // bs) for r, c in on}
            assert int((bl["bcol"] >= 0).sum()) == len(blocks)


def test_bell_laplacian_closed_forms():
    m = synth.config1_matrix()
    canon = F.canonicalize(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float32))
    # a block row of b consecutive rows of one grid row meets its own diagonal block, the
    # blocks left and right (not at the grid edge) and the blocks above and below (not in
    # the first or last grid row): 5 at most
    cnt8 = F.bell_block_counts(canon, 8)
    assert cnt8.max() == 5 and cnt8.sum() == 512 + 2 * 63 * 8 + 2 * 64 * 7
    # 8 x 8 blocks store 512 * 5 * 64 = 163840 values > 8 * 20224: refused
    with pytest.raises(F.OracleError) as e:
        F.to_bell(canon, 8)
    assert e.value.status == F.NOT_APPLICABLE
    for b, want in ((2, 2048 + 2 * 63 * 32 + 2 * 64 * 31), (4, 1024 + 2 * 63 * 16 + 2 * 64 * 15)):
        bl = F.to_bell(canon, b)
        assert bl["K"] == 5 and bl["pitch"] == 4096 // b
        assert int((bl["bcol"] >= 0).sum()) == want
        assert np.array_equal(_bell_dense(bl, 4096, 4096),
                              F.to_dense(4096, 4096, canon["row"], canon["col"], canon["val"]))
    # bytes 2048*5*(4+16) < 1024*5*(4+64) < 512*5*(4+256): the rule takes 2 x 2
    assert F.bell_size_rule(canon, 4) == 2 and F.to_bell(canon)["b"] == 2


def test_bell_block_diagonal_closed_forms():
    m = synth.block_diagonal(8 * 512, 8, 4)
    canon = F.canonicalize(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float32))
    b8 = F.to_bell(canon, 8)
    assert b8["K"] == 1 and (b8["bcol"] == np.arange(512)).all()
    assert np.array_equal(b8["bval"], m.values(np.float32))  # the dense blocks, in order
    assert F.to_bell(canon, 2)["K"] == 4 and F.to_bell(canon, 4)["K"] == 2
    # bytes per row: 2x2 (4 blocks of 2 rows) 40, 4x4 34, 8x8 32.5
    assert F.bell_size_rule(canon, 4) == 8 and F.to_bell(canon)["b"] == 8


def test_bell_fill_cap_and_round_trip():
    m = synth.poisson_random(2000, 8.0, 21)
    c = F.canonicalize(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float32))
    with pytest.raises(F.OracleError) as e:  # one entry per 8 x 8 block: 64 values each
        F.to_bell(c, 8)
    assert e.value.status == F.NOT_APPLICABLE
    # 2 x 2 blocks hold about one entry each: 4 values per entry, within the cap
    assert F.bell_size_rule(c, 4) == 2 and F.to_bell(c)["b"] == 2
    for mm in (synth.banded(257, 5), synth.stencil3d(9, 3), synth.laplacian2d(21)):
        cc = F.canonicalize(mm.n_rows, mm.n_cols, mm.row, mm.col, mm.values(np.float32))
        for b in (2, 4):
            d = _bell_dense(F.to_bell(cc, b), mm.n_rows, mm.n_cols)
            assert np.array_equal(d, F.to_dense(mm.n_rows, mm.n_cols, cc["row"], cc["col"], cc["val"]))
