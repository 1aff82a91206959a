"""GPU sparsity features against the oracle's.

Integer-valued features (n, nnz, median, mode, max, bandwidth) must be equal
after rounding to FP32; the moments and ratios within 1e-6 relative.
"""
import numpy as np
import pytest

import _cases as C
import synth
from oracle import formats as OF

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2302_05662_amd as S  # noqa: E402

EXACT = [0, 1, 5, 6, 8, 9]
RATIOS = [2, 3, 4, 7, 10, 11]


def _compare(got, want, label):
    want32 = want.astype(np.float32)
    for i in EXACT:
        assert got[i] == want32[i], (label, OF.FEATURE_NAMES[i], got[i], want[i])
    for i in RATIOS:
        assert abs(float(got[i]) - want[i]) <= 1e-6 * abs(want[i]) + 1e-30, (
            label, OF.FEATURE_NAMES[i], got[i], want[i])


@pytest.mark.parametrize("name", list(C.CASES))
def test_features_match_oracle(name):
    m = C.matrix(name)
    r, c, v = C.shuffled_input(name, np.float32)
    h = S.spmv_create(m.n_rows, m.n_cols, r, c, v)
    _compare(S.spmv_features(h), OF.features(C.canonical(name, np.float32)), name)


def test_features_full_size_power_law():
    m = synth.config3_matrix()
    v = m.values(np.float32)
    h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, v)
    _compare(S.spmv_features(h), OF.features(OF.canonicalize(m.n_rows, m.n_cols, m.row, m.col, v)),
             m.name)


def test_hyb_width_from_features_agrees_with_conversion():
    m = C.matrix("powerlaw")
    r, c, v = C.shuffled_input("powerlaw", np.float32)
    h = S.spmv_create(m.n_rows, m.n_cols, r, c, v)
    f = S.spmv_features(h)
    S.spmv_convert(h, S.SPMV_FMT_HYB)
    view = S.spmv_get_arrays(h, S.SPMV_FMT_HYB)
    assert abs(f[11] - view.nnz_tail / m.nnz) <= 1e-6
