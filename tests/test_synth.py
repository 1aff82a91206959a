"""The seeded generators: determinism and structure counts (CPU only)."""
import numpy as np
import pytest

import synth
from synth import matrices as SM


def _sorted_distinct(m):
    key = m.row.astype(np.int64) * m.n_cols + m.col
    return bool(np.all(np.diff(key) > 0))


def test_determinism():
    a, b = synth.poisson_random(3000, 17.5, 9), synth.poisson_random(3000, 17.5, 9)
    assert np.array_equal(a.row, b.row) and np.array_equal(a.col, b.col)
    assert np.array_equal(a.values(np.float32), b.values(np.float32))
    assert not np.array_equal(a.values(np.float64), a.values(np.float32).astype(np.float64))


@pytest.mark.parametrize("n,b", [(1000, 1), (500, 64), (100, 99), (10, 20)])
def test_banded_counts(n, b):
    m = synth.banded(n, b)
    bb = min(b, n - 1)
    assert m.nnz == n * (2 * bb + 1) - bb * (bb + 1)
    assert _sorted_distinct(m)
    assert np.abs(m.row.astype(int) - m.col).max() == bb


@pytest.mark.parametrize("g", [3, 10, 53])
def test_stencil_and_laplacian_counts(g):
    assert synth.stencil3d(g).nnz == 7 * g ** 3 - 6 * g ** 2
    assert synth.laplacian2d(g).nnz == 5 * g * g - 4 * g
    assert _sorted_distinct(synth.stencil3d(g))


def test_config1():
    m = synth.config1_matrix()
    assert m.n_rows == 4096 and m.nnz == 20224
    v = m.values(np.float32)
    assert set(v.tolist()) == {4.0, -1.0}
    assert (v == 4).sum() == 4096


def test_random_and_power_law_structure():
    m = synth.poisson_random(20000, 30.0, 2)
    assert _sorted_distinct(m)
    assert abs(m.nnz / m.n_rows - 30.0) < 0.3
    p = synth.power_law(200_000, 77)
    assert _sorted_distinct(p)
    lengths = np.bincount(p.row, minlength=p.n_rows)
    assert lengths.max() <= 50_000
    # E[L] = 16 by construction of x_m; the sample standard error of the mean is ~1.2 at this n
    assert abs(lengths.mean() - 16.0) < 5.0
    assert abs((lengths == 1).mean() - (1 - SM.POWER_LAW_XM ** 0.8)) < 0.01


def test_config2_specs_in_range():
    forced = 0
    for s in SM.CFG2_SEEDS:
        sp = synth.config2_spec(s)
        n = sp["n"]
        assert 1e5 <= n <= 2e6
        fam = sp["family"]
        nnz = {"banded": lambda: n * (2 * sp["b"] + 1) - sp["b"] * (sp["b"] + 1),
               "random": lambda: n * sp["lam"], "blockdiag": lambda: 8 * n,
               "stencil3d": lambda: 7 * sp["g"] ** 3 - 6 * sp["g"] ** 2}[fam]()
        assert 1e6 <= nnz <= 5e7, sp
        forced += nnz >= 2e7
    assert forced >= 10


def test_config4_and_5_specs():
    c4 = synth.config4_specs()
    assert len(c4) == 256 and all(1e3 <= s["n"] <= 2e5 for s in c4)
    c5 = synth.config5_specs(SM.CFG5_TRAIN[:50])
    assert len(c5) == 50 and all(4096 <= s["n"] <= 2e6 for s in c5)


def test_mlp_inputs():
    p = synth.epoch_permutations(3, 17, 4)
    assert p.shape == (4, 17) and all(sorted(r.tolist()) == list(range(17)) for r in p)
