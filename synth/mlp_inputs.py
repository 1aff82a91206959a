"""Random draws of the selector network's training: initial weights and epoch orders.

Both the GPU trainer and the oracle take these as inputs, so neither draws
random numbers of its own.

Flat parameter layout (float32), for layer sizes 12-64-64-C: W1[64][12], b1[64],
W2[64][64], b2[64], W3[C][64], b3[C]; each W is stored row-major as [out][in]
(5,252 values for C = 4, 5,382 for C = 6).
"""
from __future__ import annotations

import numpy as np

LAYERS = (12, 64, 64, 4)


def param_count(layers=LAYERS) -> int:
    return sum(o * i + o for i, o in zip(layers[:-1], layers[1:]))


def glorot_params(seed: int, layers=LAYERS) -> np.ndarray:
    """Glorot-uniform weights, U[-l, l] with l = sqrt(6 / (fan_in + fan_out)); zero biases."""
    rng = np.random.default_rng([seed, 11])
    parts = []
    for fan_in, fan_out in zip(layers[:-1], layers[1:]):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-lim, lim, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def epoch_permutations(seed: int, n: int, epochs: int) -> np.ndarray:
    """One seeded shuffle of the n training samples per epoch: int32 [epochs][n]."""
    rng = np.random.default_rng([seed, 12])
    return np.stack([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)
