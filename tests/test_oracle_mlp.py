"""Pins for the oracle selector network (CPU only).

Finite differences fix the gradient, a hand-built network fixes the forward
pass, the first Adam step has a closed form, and a separable toy problem must
be learned exactly.
"""
import numpy as np
import pytest

import synth
from oracle import formats as F
from oracle import mlp as M


def _rand_batch(seed, B=7):
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((B, 12))
    y = rng.integers(0, 4, B)
    return Z, y


def test_param_layout():
    assert M.N_PARAMS == 12 * 64 + 64 + 64 * 64 + 64 + 64 * 4 + 4 == 5252
    p = synth.glorot_params(0)
    assert p.size == M.N_PARAMS and p.dtype == np.float32
    (W1, b1), (W2, b2), (W3, b3) = M.unpack(p)
    assert W1.shape == (64, 12) and W2.shape == (64, 64) and W3.shape == (4, 64)
    assert not b1.any() and not b2.any() and not b3.any()
    assert np.abs(W1).max() <= np.sqrt(6 / 76) and np.abs(W3).max() <= np.sqrt(6 / 68)
    assert np.array_equal(M.pack(M.unpack(p)), p.astype(np.float64))


def test_forward_hand_built_network():
    layers = [(np.zeros((64, 12)), np.zeros(64)), (np.zeros((64, 64)), np.zeros(64)),
              (np.zeros((4, 64)), np.zeros(4))]
    layers[0][0][0, 0] = 2.0
    layers[0][1][1] = -1.0          # unit 1 stays dead
    layers[1][0][0, 0] = 1.0
    layers[1][1][0] = 0.5
    for c in range(4):
        layers[2][0][c, 0] = c
    layers[2][1][:] = [0.25, 0, 0, 0]
    p = M.pack(layers)
    Z = np.array([[1.5] + [0] * 11, [-3.0] + [0] * 11])
    out = M.forward(p, Z)["logits"]
    # h1[0] = relu(2 z0), h2[0] = relu(h1[0] + 0.5), logits[c] = c h2[0] + b3[c]
    h2 = np.array([3.5, 0.5])
    want = h2[:, None] * np.arange(4)[None, :] + np.array([0.25, 0, 0, 0])
    assert np.array_equal(out, want)


@pytest.mark.parametrize("l2", [0.0, 1e-4, 0.3])
def test_gradient_matches_central_differences(l2):
    Z, y = _rand_batch(3)
    theta = synth.glorot_params(1).astype(np.float64)
    theta[768:832] = np.random.default_rng(2).uniform(-0.1, 0.1, 64)  # nonzero b1
    _, g = M.loss_and_grad(theta, Z, y, l2)
    h = 1e-6
    rng = np.random.default_rng(4)
    idx = np.concatenate([rng.choice(M.N_PARAMS, 400, replace=False), np.arange(5248, 5252)])
    for k in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (M.loss_and_grad(tp, Z, y, l2)[0] - M.loss_and_grad(tm, Z, y, l2)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 + 1e-5 * abs(g[k]), k


def test_output_gradient_is_p_minus_onehot():
    Z, y = _rand_batch(5, B=9)
    theta = synth.glorot_params(2).astype(np.float64)
    _, g = M.loss_and_grad(theta, Z, y, 0.0)
    P = M.softmax(M.forward(theta, Z)["logits"])
    onehot = np.eye(4)[y]
    assert np.allclose(g[5248:5252], (P - onehot).mean(axis=0), rtol=0, atol=1e-15)


def test_l2_term():
    Z, y = _rand_batch(6, B=5)
    theta = synth.glorot_params(3).astype(np.float64)
    l0, g0 = M.loss_and_grad(theta, Z, y, 0.0)
    l1, g1 = M.loss_and_grad(theta, Z, y, 0.2)
    (W1, _), (W2, _), (W3, _) = M.unpack(theta)
    w2 = (W1 ** 2).sum() + (W2 ** 2).sum() + (W3 ** 2).sum()
    assert l1 - l0 == pytest.approx(0.2 / (2 * 5) * w2, rel=1e-12)
    # biases carry no penalty
    assert np.array_equal(g1[768:832], g0[768:832])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(8)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50) * 10.0 ** rng.integers(-4, 3, 50)
    t1, m, v = M.adam_step(theta, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    assert np.allclose(t1, theta - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_two_steps_by_hand():
    # Kingma and Ba, Algorithm 1, worked by hand for one parameter with theta_0 = 0,
    # gradients g_1 = 1 and g_2 = -2, alpha = 1e-3, beta1 = 0.9, beta2 = 0.999, eps = 1e-8:
    #   m_1 = 0.1, v_1 = 0.001, both bias-corrected to 1, theta_1 = -1e-3 / (1 + 1e-8);
    #   m_2 = 0.09 - 0.2 = -0.11, v_2 = 0.000999 + 0.004 = 0.004999,
    #   m_hat = -0.11 / 0.19, v_hat = 0.004999 / 0.001999 (1 - 0.9^2, 1 - 0.999^2),
    #   theta_2 = theta_1 - 1e-3 * m_hat / (sqrt(v_hat) + 1e-8), evaluated to 50 digits.
    th, m, v = M.adam_step(np.zeros(1), np.array([1.0]), np.zeros(1), np.zeros(1), 1)
    assert th[0] == pytest.approx(-0.00099999999000000009999999900000001, rel=1e-15)
    th, m, v = M.adam_step(th, np.array([-2.0]), m, v, 2)
    assert m[0] == pytest.approx(-0.11, rel=1e-15)
    assert v[0] == pytest.approx(0.004999, rel=1e-15)
    assert th[0] == pytest.approx(-0.00063389646527924911794492851072851, rel=1e-14)


def test_adam_constant_gradient_through_train(monkeypatch):
    # With a constant gradient g the bias-corrected moments are g and g^2 at every
    # step t, so each update is exactly -lr * g / (|g| + eps) and after t steps
    # theta_t = theta_0 - t * lr * g / (|g| + eps). Checked through train(), so a
    # step counter that does not advance, or a correction stuck at t = 1, fails.
    rng = np.random.default_rng(12)
    g = rng.standard_normal(M.N_PARAMS) * 10.0 ** rng.integers(-3, 3, M.N_PARAMS)
    monkeypatch.setattr(M, "loss_and_grad", lambda theta, Z, y, l2: (0.0, g.copy()))
    theta0 = synth.glorot_params(13).astype(np.float64)
    N = 10
    Fr = np.abs(rng.standard_normal((N, 12))) + 1.0
    perms = synth.epoch_permutations(13, N, 1)
    for t in range(1, 6):
        theta, _, _, losses = M.train(theta0, Fr, np.zeros(N, np.int64), perms, batch=2,
                                      lr=1e-3, steps=t)
        assert len(losses) == t
        want = theta0 - t * 1e-3 * g / (np.abs(g) + 1e-8)
        assert np.allclose(theta, want, rtol=0, atol=1e-14), t


def test_standardisation():
    rng = np.random.default_rng(9)
    Fr = np.abs(rng.standard_normal((40, 12))) * 100
    Fr[:, 7] = 0.5  # a constant column: std floored, z = 0
    Z, mean, std = M.prepare_inputs(Fr)
    assert np.allclose(Z.mean(axis=0), 0, atol=1e-12)
    keep = [i for i in range(12) if i != 7]
    assert np.allclose(Z[:, keep].std(axis=0), 1, atol=1e-12)
    assert std[7] == M.STD_FLOOR and not Z[:, 7].any()
    assert np.allclose(mean, F.transform_features(Fr).mean(axis=0))


def test_learns_separable_toy_problem():
    rng = np.random.default_rng(10)
    N = 400
    labels = rng.integers(0, 4, N)
    Fr = np.abs(rng.standard_normal((N, 12))) + 0.1
    Fr[:, 2] = 4.0 ** labels * (1 + 0.2 * rng.random(N))   # class encoded in the mean row length
    p0 = synth.glorot_params(5)
    perms = synth.epoch_permutations(5, N, 60)
    theta, mean, std, losses = M.train(p0, Fr, labels, perms, batch=50, lr=1e-2)
    pred, _ = M.predict(theta, mean, std, Fr)
    assert (pred == labels).mean() == 1.0
    assert losses[-1] < 0.2 * losses[0]


def test_predict_masks_and_ties():
    theta = np.zeros(M.N_PARAMS)
    mean, std = np.zeros(12), np.ones(12)
    pred, z = M.predict(theta, mean, std, np.ones((2, 12)),
                        applicable=np.array([[True] * 4, [True, True, False, True]]))
    assert pred.tolist() == [0, 0]  # all logits tie -> lowest index
    theta[5248 + 2] = 1.0  # b3[ELL] = 1
    pred, _ = M.predict(theta, mean, std, np.ones((2, 12)),
                        applicable=np.array([[True] * 4, [True, True, False, True]]))
    assert pred.tolist() == [2, 0]


def test_labels_and_regret():
    t = np.array([[1.0, 2.0, np.inf, 1.0], [3.0, 1.5, 1.2, 4.0]])
    assert M.labels_from_times(t).tolist() == [0, 2]
    assert M.regret(t, [3, 1]).tolist() == [0.0, 0.25]


def test_six_class_layout_and_gradient():
    # the network with SELL and BELL classes: 12-64-64-6, 5382 parameters
    p = synth.glorot_params(21, layers=(12, 64, 64, 6)).astype(np.float64)
    assert p.size == M.n_params(6) == 12 * 64 + 64 + 64 * 64 + 64 + 6 * 64 + 6 == 5382
    assert M.classes_of(p) == 6 and M.classes_of(synth.glorot_params(0)) == 4
    (W1, _), _, (W3, b3) = M.unpack(p)
    assert W3.shape == (6, 64) and b3.shape == (6,)
    # the first layers draw the same numbers as the 4-class network of the same seed
    assert np.array_equal(W1, M.unpack(synth.glorot_params(21))[0][0])
    rng = np.random.default_rng(22)
    Z = rng.standard_normal((9, 12))
    y = rng.integers(0, 6, 9)
    p[4928:4992] = rng.uniform(-0.1, 0.1, 64)
    loss, g = M.loss_and_grad(p, Z, y, 1e-3)
    P = M.softmax(M.forward(p, Z)["logits"])
    assert P.shape == (9, 6)
    assert np.allclose(g[5376:5382], (P - np.eye(6)[y]).mean(axis=0), rtol=0, atol=1e-15)
    h = 1e-6
    for k in np.concatenate([rng.choice(5382, 200, replace=False), np.arange(4992, 5382, 7)]):
        tp, tm = p.copy(), p.copy()
        tp[k] += h
        tm[k] -= h
        fd = (M.loss_and_grad(tp, Z, y, 1e-3)[0] - M.loss_and_grad(tm, Z, y, 1e-3)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 + 1e-5 * abs(g[k]), k
    theta = np.zeros(5382)
    theta[5376 + 5] = 1.0  # b3[BELL]
    pred, _ = M.predict(theta, np.zeros(12), np.ones(12), np.ones((2, 12)),
                        applicable=np.array([[True] * 6, [True] * 5 + [False]]))
    assert pred.tolist() == [5, 0]
