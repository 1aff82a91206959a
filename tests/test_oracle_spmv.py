"""Pins for the oracle SpMV (CPU only): exact rational brute force and closed forms."""
import math

import numpy as np
import pytest

import synth
from oracle import formats as F
from oracle import spmv as S

ALPHA_BETA = [(1.0, 0.0), (1.5, -0.5), (-2.0, 1.0)]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("alpha,beta", ALPHA_BETA)
def test_matches_exact_rational_brute_force(dtype, alpha, beta):
    rng = np.random.default_rng(21)
    for trial in range(12):
        n_rows = int(rng.integers(1, 33))
        n_cols = int(rng.integers(1, 33))
        nnz = int(rng.integers(0, n_rows * n_cols + 1))
        flat = rng.choice(n_rows * n_cols, nnz, replace=False)
        row, col = np.divmod(flat, n_cols)
        val = rng.uniform(-1, 1, nnz).astype(dtype)
        x = rng.uniform(-1, 1, n_cols).astype(dtype)
        y0 = rng.uniform(-1, 1, n_rows).astype(dtype)
        canon = F.canonicalize(n_rows, n_cols, row, col, val)
        y = S.spmv_csr(canon["row_ptr"], canon["col"], canon["val"], x, alpha, beta, y0)
        exact = S.spmv_dense_exact(n_rows, n_cols, row, col, val, x, alpha, beta, y0)
        D = S.row_denominator(canon["row_ptr"], canon["col"], canon["val"], x, alpha, beta, y0)
        for i in range(n_rows):
            err = abs(float(exact[i] - type(exact[i])(y[i])))
            # FP64 sum of at most 32 exact products: error <= 33 u D
            assert err <= 33 * 2.0 ** -53 * D[i] + 1e-300, (trial, i)
        ys, Ds = S.spmv_rows(np.arange(n_rows), canon["row_ptr"], canon["col"], canon["val"], x,
                             alpha, beta, y0)
        assert np.array_equal(ys, y)
        assert np.allclose(Ds, D, rtol=1e-14, atol=0)


def test_beta_zero_does_not_read_y():
    canon = F.canonicalize(2, 2, [0, 1], [1, 0], [2.0, 3.0])
    y = S.spmv_csr(canon["row_ptr"], canon["col"], canon["val"], [5.0, 7.0], 1.0, 0.0,
                   [np.nan, np.inf])
    assert y.tolist() == [14.0, 15.0]


def test_identity():
    n = 50
    canon = F.canonicalize(n, n, np.arange(n), np.arange(n), np.ones(n))
    rng = np.random.default_rng(2)
    x, y0 = rng.standard_normal(n), rng.standard_normal(n)
    y = S.spmv_csr(canon["row_ptr"], canon["col"], canon["val"], x, 0.75, -1.25, y0)
    assert np.array_equal(y, 0.75 * x + -1.25 * y0)


def test_laplacian_row_sums():
    m = synth.config1_matrix()
    canon = F.canonicalize(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float64))
    y = S.spmv_csr(canon["row_ptr"], canon["col"], canon["val"], np.ones(m.n_cols))
    g = 64
    i, j = np.divmod(np.arange(g * g), g)
    missing = (i == 0).astype(int) + (i == g - 1) + (j == 0) + (j == g - 1)
    assert np.array_equal(y, missing.astype(np.float64))  # interior 0, edge 1, corner 2
    assert y.sum() == 256


def test_laplacian_integer_closed_form():
    """f(i,j) = i^2 + j^2: (A f) = -4 + sum of f over the neighbours outside the grid."""
    g = 64
    m = synth.laplacian2d(g)
    canon = F.canonicalize(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float64))
    i, j = np.divmod(np.arange(g * g), g)
    f = (i * i + j * j).astype(np.float64)
    y = S.spmv_csr(canon["row_ptr"], canon["col"], canon["val"], f)
    want = []
    for a, b in zip(i.tolist(), j.tolist()):
        s = -4
        for (p, q) in ((a - 1, b), (a + 1, b), (a, b - 1), (a, b + 1)):
            if not (0 <= p < g and 0 <= q < g):
                s += p * p + q * q
        want.append(s)
    assert np.array_equal(y, np.array(want, np.float64))


@pytest.mark.parametrize("p,q", [(1, 1), (3, 7), (64, 2)])
def test_laplacian_eigenvectors(p, q):
    g = 64
    m = synth.laplacian2d(g)
    canon = F.canonicalize(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float64))
    i, j = np.divmod(np.arange(g * g), g)
    v = np.sin(math.pi * p * (i + 1) / (g + 1)) * np.sin(math.pi * q * (j + 1) / (g + 1))
    lam = 4 - 2 * math.cos(math.pi * p / (g + 1)) - 2 * math.cos(math.pi * q / (g + 1))
    y = S.spmv_csr(canon["row_ptr"], canon["col"], canon["val"], v)
    assert np.max(np.abs(y - lam * v)) < 1e-13


def test_row_sums_of_random_structure_with_integer_values():
    m = synth.poisson_random(2000, 20.0, 4)
    vals = np.random.default_rng(1).integers(-8, 9, m.nnz).astype(np.float64)
    canon = F.canonicalize(m.n_rows, m.n_cols, m.row, m.col, vals)
    y = S.spmv_csr(canon["row_ptr"], canon["col"], canon["val"], np.ones(m.n_cols), n_threads=4)
    want = np.zeros(m.n_rows)
    np.add.at(want, m.row, vals)
    assert np.array_equal(y, want)


def test_max_row_error_metric():
    assert S.max_row_error([1.0, 2.0], [1.0, 2.0], [0.0, 1.0]) == 0.0
    assert S.max_row_error([1.0, 2.5], [1.0, 2.0], [0.0, 1.0]) == 0.5
    assert S.max_row_error([1.5, 2.0], [1.0, 2.0], [0.0, 1.0]) == float("inf")
