"""Oracle for the learned format selector, in FP64 NumPy.

Test infrastructure only.

The paper selects the sparse format with a classifier over sparsity features
(Method: predicting optimal configuration parameters, multi-class
classification) and reports an MLP trained with ReLU, Adam and learning rate
0.001 for 200 epochs, other settings left at scikit-learn defaults (Learning
Algorithms section and its model table). Here the network is 12-64-64-C, C = 4 classes (CSR, COO,
ELL, HYB) or 6 (also SELL, BELL):

  h1 = ReLU(W1 z + b1), h2 = ReLU(W2 h1 + b2), logits = W3 h2 + b3,

with z the standardised transformed features. Training minimises the mean
softmax cross-entropy over a minibatch of size B plus (alpha / (2 B)) times the
squared norm of the weight matrices (scikit-learn's documented L2 term, alpha
= 1e-4), with Adam as in Kingma and Ba (2015, Algorithm 1): lr 1e-3,
beta1 0.9, beta2 0.999, eps 1e-8. Initial weights and per-epoch sample orders
are inputs.
"""
from __future__ import annotations

import numpy as np

from .formats import transform_features

LAYERS = (12, 64, 64, 4)
N_PARAMS = 5252
STD_FLOOR = 1e-6
HIDDEN_PARAMS = 12 * 64 + 64 + 64 * 64 + 64  # every parameter before W3


def classes_of(params) -> int:
    """Output classes of a flat parameter vector: 4 (CSR, COO, ELL, HYB) or 6 (also SELL, BELL)."""
    rest = np.asarray(params).size - HIDDEN_PARAMS
    assert rest > 0 and rest % 65 == 0, "not a 12-64-64-C parameter vector"
    return rest // 65


def n_params(classes: int) -> int:
    return HIDDEN_PARAMS + 65 * classes


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    layers = LAYERS[:-1] + (classes_of(p),)
    out = []
    off = 0
    for fi, fo in zip(layers[:-1], layers[1:]):
        W = p[off:off + fo * fi].reshape(fo, fi)
        off += fo * fi
        b = p[off:off + fo]
        off += fo
        out.append((W, b))
    assert off == p.size
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def standardize_stats(T):
    """Per-feature mean and population standard deviation (floored) of the training inputs."""
    T = np.asarray(T, np.float64)
    mean = T.mean(axis=0)
    std = np.maximum(T.std(axis=0), STD_FLOOR)
    return mean, std


def forward(params, Z):
    (W1, b1), (W2, b2), (W3, b3) = unpack(params)
    a1 = Z @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3.T + b3
    return {"Z": Z, "a1": a1, "h1": h1, "a2": a2, "h2": h2, "logits": z}


def softmax(z):
    z = z - z.max(axis=-1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=-1, keepdims=True)


def loss_and_grad(params, Z, labels, l2=1e-4):
    """Mean cross-entropy + l2/(2B) * sum of squared weights, and its gradient (flat)."""
    Z = np.asarray(Z, np.float64)
    labels = np.asarray(labels, np.int64)
    B = Z.shape[0]
    (W1, b1), (W2, b2), (W3, b3) = unpack(params)
    c = forward(params, Z)
    P = softmax(c["logits"])
    ce = -np.mean(np.log(P[np.arange(B), labels]))
    reg = (l2 / (2.0 * B)) * (np.sum(W1 * W1) + np.sum(W2 * W2) + np.sum(W3 * W3))
    dz = P.copy()
    dz[np.arange(B), labels] -= 1.0
    dz /= B
    gW3 = dz.T @ c["h2"] + (l2 / B) * W3
    gb3 = dz.sum(axis=0)
    dh2 = dz @ W3
    da2 = dh2 * (c["a2"] > 0)
    gW2 = da2.T @ c["h1"] + (l2 / B) * W2
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * (c["a1"] > 0)
    gW1 = da1.T @ Z + (l2 / B) * W1
    gb1 = da1.sum(axis=0)
    grad = pack([(gW1, gb1), (gW2, gb2), (gW3, gb3)])
    return ce + reg, grad


def adam_step(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v


def prepare_inputs(F_train):
    """Transform the raw features and standardise them with the training statistics."""
    T = transform_features(F_train)
    mean, std = standardize_stats(T)
    return (T - mean) / std, mean, std


def train(params0, F_train, labels, perms, batch=200, lr=1e-3, l2=1e-4, steps=None):
    """Minibatch Adam over the given epoch orders. Returns (params, mean, std, losses).

    ``steps`` stops after that many updates (for short trajectory checks).
    """
    Z, mean, std = prepare_inputs(F_train)
    labels = np.asarray(labels, np.int64)
    N = Z.shape[0]
    B = min(batch, N)
    theta = np.asarray(params0, np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    t = 0
    losses = []
    for order in perms:
        for s in range(0, N, B):
            idx = np.asarray(order[s:s + B], np.int64)
            loss, g = loss_and_grad(theta, Z[idx], labels[idx], l2)
            t += 1
            theta, m, v = adam_step(theta, g, m, v, t, lr)
            losses.append(loss)
            if steps is not None and t >= steps:
                return theta, mean, std, np.array(losses)
    return theta, mean, std, np.array(losses)


def predict(params, mean, std, F, applicable=None):
    """Argmax of the logits over applicable formats (ties -> lowest index)."""
    Z = (transform_features(np.atleast_2d(F)) - mean) / std
    z = forward(params, Z)["logits"]
    if applicable is not None:
        z = np.where(np.atleast_2d(applicable), z, -np.inf)
    return np.argmax(z, axis=1), z


def labels_from_times(times):
    """Fastest applicable format per matrix (inf = not applicable); ties -> lowest index."""
    return np.argmin(np.asarray(times, np.float64), axis=1)


def regret(times, chosen):
    """Per-matrix t(chosen) / t(best) - 1."""
    t = np.asarray(times, np.float64)
    best = t.min(axis=1)
    return t[np.arange(t.shape[0]), np.asarray(chosen)] / best - 1.0
