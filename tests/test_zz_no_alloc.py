"""spmv_features_noalloc (temporaries in the library's fixed device array)
against spmv_features on the same handles: bit-equal features, also on a
second, smaller matrix right after a larger one (the array keeps the last
call's contents), at the longest accepted row, and the refusal beyond it."""
import numpy as np
import pytest

import _cases as C
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2302_05662_amd as S  # noqa: E402


def _handle(name):
    m = C.matrix(name)
    r, c, v = C.shuffled_input(name, np.float32)
    return S.spmv_create(m.n_rows, m.n_cols, r, c, v)


def _one_row(n_cols, seed):
    rng = np.random.default_rng(seed)
    col = np.arange(n_cols, dtype=np.int32)
    row = np.zeros(n_cols, dtype=np.int32)
    # two more rows, short, so the histogram has several bins
    row = np.concatenate([row, np.array([1, 2, 2], dtype=np.int32)])
    col = np.concatenate([col, np.array([5, 0, 7], dtype=np.int32)])
    val = rng.uniform(-1, 1, row.size).astype(np.float32)
    return S.spmv_create(3, n_cols, row, col, val)


def test_noalloc_features_equal_allocating_call_twice_in_a_row():
    big, small = _handle("powerlaw"), _handle("banded")
    assert C.matrix("banded").nnz < C.matrix("powerlaw").nnz
    for h in (big, small, big, small):
        got = S.spmv_features_noalloc(h)
        want = S.spmv_features(h)
        np.testing.assert_array_equal(got, want)
    # the allocation-free call first on a fresh handle, then the reference
    h = _handle("one_long_row")
    got = S.spmv_features_noalloc(h)
    np.testing.assert_array_equal(got, S.spmv_features(h))


@pytest.mark.parametrize("name", ["lap64", "stencil", "empty", "zero", "single", "very_wide"])
def test_noalloc_features_cases(name):
    h = _handle(name)
    np.testing.assert_array_equal(S.spmv_features_noalloc(h), S.spmv_features(h))


def test_noalloc_longest_accepted_row_and_refusal():
    n = S.SPMV_FEATURES_NOALLOC_MAX_LEN
    h = _one_row(n, 7)
    got = S.spmv_features_noalloc(h)
    np.testing.assert_array_equal(got, S.spmv_features(h))
    assert got[8] == n
    h2 = _one_row(n + 1, 8)
    with pytest.raises(S.SpmvError, match="allocation-free"):
        S.spmv_features_noalloc(h2)
    # the refused call left nothing behind: the next one is still right
    h3 = _handle("random")
    np.testing.assert_array_equal(S.spmv_features_noalloc(h3), S.spmv_features(h3))
