"""Seeded parity cases shared by the GPU tests, with their oracle references."""
from __future__ import annotations

import functools

import numpy as np

import synth
from oracle import formats as OF
from oracle import spmv as OS

ALPHA_BETA = [(1.0, 0.0), (1.5, -0.5), (-2.0, 1.0)]
TOL = {np.float32: 1e-5, np.float64: 1e-12}


def _one_long_row(n=3000, seed=41):
    r = np.arange(n)
    rows = np.concatenate([r, np.full(n - 1, n // 2)])
    cols = np.concatenate([r, np.delete(np.arange(n), n // 2)])
    return synth.from_coords("one_long_row", n, n, rows, cols, seed)


CASES = {
    "lap64": lambda: synth.config1_matrix(),
    "random": lambda: synth.poisson_random(5003, 13.7, 101),
    "powerlaw": lambda: synth.power_law(20011, 102, cap=5000, value_dist="uniform"),
    "banded": lambda: synth.banded(3001, 9, 103),
    "blockdiag": lambda: synth.block_diagonal(8 * 513, 8, 104),
    "stencil": lambda: synth.stencil3d(17, 105),
    "sparse_rows": lambda: synth.poisson_random(7001, 0.7, 106),
    "wide": lambda: synth.random_rect(700, 5000, 40000, 107),
    "tall": lambda: synth.random_rect(5000, 30, 9000, 108),
    # x spans several 2 MB column panels (the column-split COO variant applies)
    "very_wide": lambda: synth.random_rect(1500, 1_200_000, 45000, 113),
    "one_long_row": _one_long_row,
    "last_row_only": lambda: synth.from_coords("last_row_only", 4000, 4000,
                                               np.full(1000, 3999), np.arange(0, 4000, 4), 109),
    "single": lambda: synth.from_coords("single", 1, 1, [0], [0], 110),
    "empty": lambda: synth.from_coords("empty", 50, 40, [], [], 111),
    "zero": lambda: synth.from_coords("zero", 0, 0, [], [], 112),
}


@functools.lru_cache(maxsize=None)
def matrix(name):
    return CASES[name]()


@functools.lru_cache(maxsize=None)
def shuffled_input(name, dtype):
    """(row, col, val) of the case in a seeded random order."""
    m = matrix(name)
    r, c, perm = synth.shuffled(m, 5)
    return r, c, m.values(dtype)[perm]


@functools.lru_cache(maxsize=None)
def canonical(name, dtype):
    m = matrix(name)
    r, c, v = shuffled_input(name, dtype)
    return OF.canonicalize(m.n_rows, m.n_cols, r, c, v)


@functools.lru_cache(maxsize=None)
def vectors(name, dtype):
    m = matrix(name)
    x = synth.uniform_vector(m.n_cols, dtype, [m.seed, 3])
    y0 = synth.uniform_vector(m.n_rows, dtype, [m.seed, 4])
    return x, y0


@functools.lru_cache(maxsize=None)
def reference(name, dtype, alpha, beta):
    """(y_ref in FP64, per-row denominator D)."""
    c = canonical(name, dtype)
    x, y0 = vectors(name, dtype)
    a, b = dtype(alpha), dtype(beta)
    y = OS.spmv_csr(c["row_ptr"], c["col"], c["val"], x, a, b, y0)
    d = OS.row_denominator(c["row_ptr"], c["col"], c["val"], x, a, b, y0)
    return y, d
