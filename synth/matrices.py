"""Seeded sparse-matrix structures standing in for the paper's SuiteSparse set.

The paper measures on 30 SuiteSparse matrices with 14,340 < n < 1,489,752 and
800,800 < nnz < 19,235,140 (Experimental Setup, Benchmark). Those matrices are
not used here; these generators produce synthetic stand-ins with the same kind
of structure (banded, uniform random, block diagonal, stencils, power-law row
lengths) over a wider size range. Every function is deterministic in its seed.

Entries come back sorted by (row, col) with distinct columns per row, as int32
index arrays. Values are drawn separately per precision by ``Matrix.values``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# container
# ---------------------------------------------------------------------------


@dataclass
class Matrix:
    name: str
    family: str
    n_rows: int
    n_cols: int
    row: np.ndarray  # int32, sorted by (row, col)
    col: np.ndarray  # int32
    seed: int
    params: dict = field(default_factory=dict)
    value_dist: str = "uniform"  # "uniform" U[-1,1], "normal" N(0,1), "fixed"
    fixed_values: np.ndarray | None = None  # float64, used when value_dist == "fixed"

    @property
    def nnz(self) -> int:
        return int(self.row.shape[0])

    def values(self, dtype) -> np.ndarray:
        """Values of the stored entries, drawn from a stream of their own per precision."""
        dtype = np.dtype(dtype)
        if self.value_dist == "fixed":
            return self.fixed_values.astype(dtype)
        stream = 1 if dtype == np.float32 else 2
        rng = np.random.default_rng([self.seed, stream])
        if self.value_dist == "normal":
            v = rng.standard_normal(self.nnz)
        else:
            v = rng.uniform(-1.0, 1.0, self.nnz)
        return v.astype(dtype)

    def x(self, dtype) -> np.ndarray:
        return uniform_vector(self.n_cols, dtype, [self.seed, 3])


def uniform_vector(n: int, dtype, seed) -> np.ndarray:
    """Dense vector with entries U[-1, 1] from ``seed``."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, int(n)).astype(np.dtype(dtype))


def _from_lengths(lengths: np.ndarray):
    """Row index array and per-entry position inside its row."""
    lengths = np.asarray(lengths, dtype=np.int64)
    n = lengths.shape[0]
    nnz = int(lengths.sum())
    row = np.repeat(np.arange(n, dtype=np.int64), lengths)
    starts = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lengths, out=starts[1:])
    pos = np.arange(nnz, dtype=np.int64) - starts[row]
    return row, pos


def _sorted_random_columns(lengths: np.ndarray, n_cols: int, rng: np.random.Generator):
    """For every row, ``len`` sorted uniform columns in [0, n_cols), collisions dropped.

    Sorted uniform order statistics come from normalised partial sums of
    len+1 exponential draws, so no sort is needed.
    """
    lengths = np.minimum(np.asarray(lengths, dtype=np.int64), n_cols)
    n = lengths.shape[0]
    slots = lengths + 1
    total_slots = int(slots.sum())
    c = np.cumsum(rng.standard_exponential(total_slots))
    end = np.cumsum(slots) - 1
    start = end - lengths
    base = np.where(start > 0, c[np.maximum(start - 1, 0)], 0.0)
    span = c[end] - base
    keep_slot = np.ones(total_slots, dtype=bool)
    keep_slot[end] = False
    row = np.repeat(np.arange(n, dtype=np.int64), lengths)
    u = (c[keep_slot] - base[row]) / span[row]
    del c, keep_slot
    col = np.minimum(np.floor(u * n_cols).astype(np.int64), n_cols - 1)
    del u
    if col.shape[0] > 1:
        dup = np.zeros(col.shape[0], dtype=bool)
        dup[1:] = (col[1:] == col[:-1]) & (row[1:] == row[:-1])
        if dup.any():
            row = row[~dup]
            col = col[~dup]
    return row, col


def _pack(name, family, n_rows, n_cols, row, col, seed, params, value_dist="uniform", fixed=None):
    assert n_rows < 2**31 and n_cols < 2**31
    return Matrix(
        name=name,
        family=family,
        n_rows=int(n_rows),
        n_cols=int(n_cols),
        row=np.ascontiguousarray(row, dtype=np.int32),
        col=np.ascontiguousarray(col, dtype=np.int32),
        seed=int(seed),
        params=dict(params),
        value_dist=value_dist,
        fixed_values=fixed,
    )


# ---------------------------------------------------------------------------
# structure families
# ---------------------------------------------------------------------------


def laplacian2d(g: int, seed: int = 1) -> Matrix:
    """5-point Laplacian on a g x g grid, node (i, j) -> g*i + j, Dirichlet boundary.

    Diagonal 4, neighbours -1; columns of a row in increasing order.
    """
    n = g * g
    node = np.arange(n, dtype=np.int64)
    i, j = np.divmod(node, g)
    offs = [(-g, i > 0), (-1, j > 0), (0, np.ones(n, bool)), (1, j < g - 1), (g, i < g - 1)]
    present = np.stack([m for _, m in offs], axis=1)  # n x 5, in column order
    cols = node[:, None] + np.array([o for o, _ in offs])[None, :]
    vals = np.where(np.array([o for o, _ in offs])[None, :] == 0, 4.0, -1.0)
    vals = np.broadcast_to(vals, present.shape)
    row = np.broadcast_to(node[:, None], present.shape)[present]
    return _pack(f"laplacian2d_g{g}", "laplacian2d", n, n, row, cols[present], seed,
                 {"g": g}, value_dist="fixed", fixed=np.ascontiguousarray(vals[present]))


def banded(n: int, b: int, seed: int = 0) -> Matrix:
    """Full band: row i holds columns max(0, i-b) .. min(n-1, i+b)."""
    i = np.arange(n, dtype=np.int64)
    lo = np.maximum(0, i - b)
    hi = np.minimum(n - 1, i + b)
    row, pos = _from_lengths(hi - lo + 1)
    col = lo[row] + pos
    return _pack(f"banded_n{n}_b{b}", "banded", n, n, row, col, seed, {"b": b})


def poisson_random(n: int, lam: float, seed: int) -> Matrix:
    """Row lengths ~ Poisson(lam); columns uniform, distinct, sorted."""
    rng = np.random.default_rng([seed, 0])
    lengths = rng.poisson(lam, n)
    row, col = _sorted_random_columns(lengths, n, rng)
    return _pack(f"random_n{n}_lam{lam:.2f}", "random", n, n, row, col, seed, {"lam": float(lam)})


def block_diagonal(n: int, bs: int = 8, seed: int = 0) -> Matrix:
    """Dense bs x bs blocks on the diagonal; n must be a multiple of bs."""
    assert n % bs == 0
    row, pos = _from_lengths(np.full(n, bs, dtype=np.int64))
    col = (row // bs) * bs + pos
    return _pack(f"blockdiag_n{n}_bs{bs}", "blockdiag", n, n, row, col, seed, {"bs": bs})


def stencil3d(g: int, seed: int = 0) -> Matrix:
    """7-point stencil on a g^3 grid, node (i, j, k) -> g*g*i + g*j + k."""
    n = g ** 3
    node = np.arange(n, dtype=np.int64)
    i, rem = np.divmod(node, g * g)
    j, k = np.divmod(rem, g)
    g2 = g * g
    offs = [(-g2, i > 0), (-g, j > 0), (-1, k > 0), (0, np.ones(n, bool)),
            (1, k < g - 1), (g, j < g - 1), (g2, i < g - 1)]
    present = np.stack([m for _, m in offs], axis=1)
    cols = node[:, None] + np.array([o for o, _ in offs])[None, :]
    row = np.broadcast_to(node[:, None], present.shape)[present]
    return _pack(f"stencil3d_g{g}", "stencil3d", n, n, row, cols[present], seed, {"g": g})


POWER_LAW_XM = 0.30202  # scale giving E[L] = 16 for density exponent 1.8 and cap 50,000


def power_law(n: int, seed: int, cap: int = 50_000, x_m: float = POWER_LAW_XM,
              density_exponent: float = 1.8, value_dist: str = "normal") -> Matrix:
    """Row lengths from a discretised power law: L = min(cap, ceil(x_m * U**(-1/(a-1)))).

    U ~ (0, 1], a = density exponent. Columns uniform, distinct, sorted.
    """
    rng = np.random.default_rng([seed, 0])
    u = 1.0 - rng.random(n)  # (0, 1]
    lengths = np.minimum(cap, np.ceil(x_m * u ** (-1.0 / (density_exponent - 1.0))))
    lengths = lengths.astype(np.int64)
    row, col = _sorted_random_columns(lengths, n, rng)
    return _pack(f"powerlaw_n{n}_cap{cap}", "powerlaw", n, n, row, col, seed,
                 {"cap": cap, "x_m": x_m, "a": density_exponent}, value_dist=value_dist)


def shuffled(m: Matrix, seed: int):
    """The entries of ``m`` in a seeded random order: (row, col, perm)."""
    perm = np.random.default_rng([seed, 7]).permutation(m.nnz)
    return m.row[perm], m.col[perm], perm


# ---------------------------------------------------------------------------
# workload sets
# ---------------------------------------------------------------------------


def config1_matrix() -> Matrix:
    """2-D 5-point Laplacian, 64 x 64 grid: 4096 rows, 20,224 stored entries."""
    return laplacian2d(64, seed=1)


CFG2_SEEDS = tuple(range(2000, 2030))
CFG2_FAMILIES = ("banded", "random", "blockdiag", "stencil3d")


def _log_uniform_int(rng, lo, hi):
    lo = max(1.0, float(lo))
    hi = max(lo, float(hi))
    return int(math.exp(rng.uniform(math.log(lo), math.log(hi))))


def config2_spec(seed: int) -> dict:
    """Family and size parameters of one single-SpMV matrix (1e5-2e6 rows, 1e6-5e7 nnz)."""
    rng = np.random.default_rng(seed)
    fam = CFG2_FAMILIES[seed % 4]
    forced = (seed % 4 in (0, 1)) and (seed - CFG2_SEEDS[0]) < 20  # 10 matrices >= 2e7 nnz
    nnz_lo = 2e7 if forced else 1e6
    if fam == "banded":
        b = int(rng.integers(5 if forced else 1, 65))
        per = 2 * b + 1
        lo = max(1e5, (nnz_lo + b * (b + 1)) / per)
        hi = min(2e6, 5e7 / per)
        n = _log_uniform_int(rng, lo, hi)
        return {"seed": seed, "family": fam, "n": n, "b": b}
    if fam == "random":
        lam = float(rng.uniform(10.0 if forced else 8.0, 64.0))
        lo = max(1e5, 1.02 * nnz_lo / lam)
        hi = min(2e6, 4.8e7 / lam)
        n = _log_uniform_int(rng, lo, hi)
        return {"seed": seed, "family": fam, "n": n, "lam": lam}
    if fam == "blockdiag":
        n = _log_uniform_int(rng, 1.25e5, 2e6) // 8 * 8
        return {"seed": seed, "family": fam, "n": n, "bs": 8}
    g = int(rng.integers(53, 126))
    return {"seed": seed, "family": fam, "n": g ** 3, "g": g}


def _from_spec(spec: dict) -> Matrix:
    fam, seed = spec["family"], spec["seed"]
    if fam == "banded":
        m = banded(spec["n"], spec["b"], seed)
    elif fam == "random":
        m = poisson_random(spec["n"], spec["lam"], seed)
    elif fam == "blockdiag":
        m = block_diagonal(spec["n"], spec.get("bs", 8), seed)
    elif fam == "stencil3d":
        m = stencil3d(spec["g"], seed)
    elif fam == "laplacian2d":
        m = laplacian2d(spec["g"], seed)
        m = Matrix(**{**m.__dict__, "value_dist": "uniform", "fixed_values": None})
    elif fam == "powerlaw":
        m = power_law(spec["n"], seed, cap=spec["cap"], value_dist=spec.get("dist", "normal"))
    else:
        raise ValueError(fam)
    m.name = f"s{seed}_{m.name}"
    m.seed = seed
    return m


def config2_matrix(seed: int) -> Matrix:
    return _from_spec(config2_spec(seed))


def config3_matrix(seed: int = 3000, n: int = 2_000_000) -> Matrix:
    """2M x 2M, power-law row lengths (mean 16, cap 50K), N(0,1) values."""
    m = power_law(n, seed)
    m.name = f"s{seed}_{m.name}"
    return m


CFG4_SEEDS = tuple(range(4000, 4256))


def config4_specs(seeds=CFG4_SEEDS) -> list:
    """256 uneven matrices: rows log-uniform in [1e3, 2e5], banded / Poisson / power-law."""
    out = []
    for s in seeds:
        rng = np.random.default_rng(s)
        n = _log_uniform_int(rng, 1e3, 2e5)
        fam = ("banded", "random", "powerlaw")[int(rng.integers(3))]
        if fam == "banded":
            out.append({"seed": s, "family": fam, "n": n, "b": int(rng.integers(1, 65))})
        elif fam == "random":
            out.append({"seed": s, "family": fam, "n": n, "lam": float(rng.uniform(8, 64))})
        else:
            out.append({"seed": s, "family": fam, "n": n, "cap": min(50_000, n), "dist": "uniform"})
    return out


def config4_matrix(spec: dict) -> Matrix:
    return _from_spec(spec)


CFG5_TRAIN = tuple(range(5000, 6500))
CFG5_HELDOUT = tuple(range(6500, 7000))
CFG5_NNZ_CAP = 20_000_000
CFG5_FAMILIES = ("laplacian2d", "banded", "random", "blockdiag", "stencil3d")
# extended selector set: the same families plus the power law of the load-imbalanced config
CFG5X_FAMILIES = CFG5_FAMILIES + ("powerlaw",)
CFG5X_TRAIN = tuple(range(7000, 7400))
CFG5X_HELDOUT = tuple(range(7400, 7600))


def config5_specs(seeds, n_lo: float = 4096, n_hi: float = 2e6, nnz_cap: int = CFG5_NNZ_CAP,
                  families=CFG5_FAMILIES) -> list:
    """Selector matrices: 2-D Laplacians and the four single-SpMV families (optionally the
    power law too), nnz <= cap."""
    out = []
    for s in seeds:
        rng = np.random.default_rng(s)
        fam = families[int(rng.integers(len(families)))]
        n = _log_uniform_int(rng, n_lo, n_hi)
        if fam == "laplacian2d":
            g = int(min(1400, max(64, round(math.sqrt(n)))))
            out.append({"seed": s, "family": fam, "g": g, "n": g * g})
        elif fam == "banded":
            b = int(rng.integers(1, 65))
            n = int(min(n, nnz_cap // (2 * b + 1)))
            out.append({"seed": s, "family": fam, "n": n, "b": b})
        elif fam == "random":
            lam = float(rng.uniform(8, 64))
            n = int(min(n, 0.95 * nnz_cap / lam))
            out.append({"seed": s, "family": fam, "n": n, "lam": lam})
        elif fam == "blockdiag":
            out.append({"seed": s, "family": fam, "n": max(8, n // 8 * 8), "bs": 8})
        elif fam == "powerlaw":  # mean row length 16
            n = int(min(n, nnz_cap // 16))
            out.append({"seed": s, "family": fam, "n": n, "cap": min(50_000, n), "dist": "uniform"})
        else:
            g = int(min(125, max(16, round(n ** (1.0 / 3.0)))))
            out.append({"seed": s, "family": fam, "g": g, "n": g ** 3})
    return out


def config5_matrix(spec: dict) -> Matrix:
    return _from_spec(spec)


def random_rect(n_rows: int, n_cols: int, nnz: int, seed: int) -> Matrix:
    """nnz distinct uniformly placed entries of an n_rows x n_cols matrix."""
    rng = np.random.default_rng([seed, 0])
    flat = np.sort(rng.choice(n_rows * n_cols, nnz, replace=False))
    row, col = np.divmod(flat, n_cols)
    return _pack(f"rect_{n_rows}x{n_cols}_{nnz}", "rect", n_rows, n_cols, row, col, seed, {})


def from_coords(name: str, n_rows: int, n_cols: int, row, col, seed: int = 0) -> Matrix:
    """A matrix with the given distinct coordinates (sorted here), uniform values."""
    row = np.asarray(row, np.int64)
    col = np.asarray(col, np.int64)
    o = np.lexsort((col, row))
    return _pack(name, "custom", n_rows, n_cols, row[o], col[o], seed, {})
