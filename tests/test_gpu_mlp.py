"""GPU selector network against the FP64 oracle: gradients, Adam steps, training, prediction."""
import numpy as np
import pytest

import synth
from oracle import formats as OF
from oracle import mlp as OM

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2302_05662_amd as S  # noqa: E402


def _dev(a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a if dtype is None else a.astype(dtype))).cuda()


def _params(seed):
    p = synth.glorot_params(seed).astype(np.float64)
    rng = np.random.default_rng(seed)
    p[768:832] = rng.uniform(-0.2, 0.2, 64)    # b1
    p[4928:4992] = rng.uniform(-0.2, 0.2, 64)  # b2
    p[5248:5252] = rng.uniform(-0.2, 0.2, 4)   # b3
    return p.astype(np.float32)


def _rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


SEGMENTS = {"W1": (0, 768), "b1": (768, 832), "W2": (832, 4928), "b2": (4928, 4992),
            "W3": (4992, 5248), "b3": (5248, 5252)}


@pytest.mark.parametrize("B,l2", [(200, 1e-4), (37, 0.5), (1, 1e-4)])
def test_loss_and_gradient_match_oracle(B, l2):
    rng = np.random.default_rng(B)
    p = _params(3)
    Z = rng.standard_normal((B, 12)).astype(np.float32)
    y = rng.integers(0, 4, B).astype(np.int32)
    loss, grad = S.spmv_selector_loss_grad(_dev(p), _dev(Z), _dev(y), l2)
    ref_loss, ref_grad = OM.loss_and_grad(p.astype(np.float64), Z.astype(np.float64), y, l2)
    assert abs(float(loss.item()) - ref_loss) <= 1e-5 * abs(ref_loss)
    g = grad.cpu().numpy()
    for name, (a, b) in SEGMENTS.items():
        assert _rel_l2(g[a:b], ref_grad[a:b]) <= 1e-4, name


def _toy(N=300, seed=4):
    """Raw feature vectors whose class is encoded in the mean row length."""
    rng = np.random.default_rng(seed)
    labels = rng.integers(0, 4, N).astype(np.int32)
    F = (np.abs(rng.standard_normal((N, 12))) * 50 + 1).astype(np.float32)
    F[:, 2] = (4.0 ** labels * (1 + 0.2 * rng.random(N))).astype(np.float32)
    F[:, 7] = rng.random(N).astype(np.float32)
    return F, labels


def test_standardisation_and_first_steps_match_oracle():
    F, labels = _toy()
    p0 = synth.glorot_params(6)
    perms = synth.epoch_permutations(6, F.shape[0], 2)
    for steps in (1, 3):
        model = S.spmv_selector_train(_dev(F), _dev(labels), _dev(p0), _dev(perms), epochs=2,
                                      batch=64, max_steps=steps).cpu().numpy()
        theta, mean, std, _ = OM.train(p0, F, labels, perms, batch=64, steps=steps)
        assert np.allclose(model[5252:5264], mean, rtol=1e-6, atol=1e-6)
        assert np.allclose(model[5264:5276], std, rtol=1e-5, atol=1e-6)
        d_gpu = model[:5252].astype(np.float64) - p0
        d_ref = theta - p0
        bad = np.abs(d_gpu - d_ref) > 2e-5 * steps + 1e-3 * np.abs(d_ref)
        assert bad.mean() <= 0.002, (steps, int(bad.sum()))


def test_loss_history_and_training_accuracy():
    F, labels = _toy(N=400, seed=8)
    p0 = synth.glorot_params(8)
    perms = synth.epoch_permutations(8, F.shape[0], 60)
    steps = 60 * int(np.ceil(400 / 50))
    losses = torch.zeros(steps, device="cuda")
    model = S.spmv_selector_train(_dev(F), _dev(labels), _dev(p0), _dev(perms), epochs=60,
                                  batch=50, lr=1e-2, out_losses=losses)
    _, cls = S.spmv_selector_predict(model, _dev(F))
    assert (cls.cpu().numpy() == labels).mean() == 1.0
    h = losses.cpu().numpy()
    assert h[-1] < 0.2 * h[0]
    theta, mean, std, ref_losses = OM.train(p0, F, labels, perms, batch=50, lr=1e-2)
    assert abs(h[0] - ref_losses[0]) <= 1e-5 * ref_losses[0]
    pred_ref, _ = OM.predict(theta, mean, std, F)
    assert (pred_ref == labels).mean() == 1.0


def test_predict_matches_oracle_forward_and_masks():
    rng = np.random.default_rng(11)
    F, _ = _toy(N=257, seed=11)
    model = np.concatenate([_params(12), rng.uniform(0, 5, 12), rng.uniform(0.5, 3, 12)]).astype(np.float32)
    app = (rng.random((257, 4)) < 0.7).astype(np.uint8)
    app[:, 0] = 1
    logits, cls = S.spmv_selector_predict(_dev(model), _dev(F), applicable=_dev(app))
    mean, std = model[5252:5264].astype(np.float64), model[5264:5276].astype(np.float64)
    pred, ref = OM.predict(model[:5252], mean, std, F, applicable=app.astype(bool))
    refz = OM.forward(model[:5252].astype(np.float64), (OF.transform_features(F) - mean) / std)["logits"]
    assert np.allclose(logits.cpu().numpy(), refz, rtol=1e-4, atol=1e-4)
    got = cls.cpu().numpy()
    # where two allowed logits are closer than FP32 noise, either is acceptable
    srt = np.sort(np.where(app.astype(bool), refz, -np.inf), axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 1e-3
    assert np.array_equal(got[clear], pred[clear])
    assert np.all(app[np.arange(257), got] == 1)


def test_select_format_model_mode():
    m = synth.config1_matrix()
    v = m.values(np.float32)
    h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, v)
    S.spmv_selector_set_weights(None)
    with pytest.raises(S.SpmvError) as e:
        S.spmv_select_format(h, S.SPMV_SELECT_MODEL)
    assert e.value.status == "NO_MODEL"
    model = np.zeros(5276, np.float32)
    model[5264:5276] = 1.0
    model[5248 + 3] = 2.0  # b3 favours HYB
    S.spmv_selector_set_weights(model)
    assert np.array_equal(S.spmv_selector_get_weights(), model)
    fmt, scores = S.spmv_select_format(h, S.SPMV_SELECT_MODEL)
    assert fmt == S.SPMV_FMT_HYB and scores[3] == 2.0
    S.spmv_get_arrays(h, S.SPMV_FMT_HYB)  # converted by the selection
    model[5248 + 3] = 0.0
    model[5248 + 2] = 5.0  # ELL, applicable for the Laplacian
    S.spmv_selector_set_weights(model)
    assert S.spmv_select_format(h, S.SPMV_SELECT_MODEL)[0] == S.SPMV_FMT_ELL
    pl = synth.power_law(5000, 3, cap=4000)
    h2 = S.spmv_create(pl.n_rows, pl.n_cols, pl.row, pl.col, pl.values(np.float32))
    model[5248 + 1] = 4.0  # ELL is refused for this matrix: next best is COO
    S.spmv_selector_set_weights(model)
    assert S.spmv_select_format(h2, S.SPMV_SELECT_MODEL)[0] == S.SPMV_FMT_COO
    S.spmv_selector_set_weights(None)


def test_exhaustive_and_rule_selection():
    m = C_banded = synth.banded(20000, 4)
    h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float32))
    fmt, times = S.spmv_select_format(h, S.SPMV_SELECT_EXHAUSTIVE)
    assert np.all(np.isfinite(times)) and fmt == int(np.argmin(times))
    rfmt, votes = S.spmv_select_format(h, S.SPMV_SELECT_RULE)
    assert votes.sum() == 1 and votes[rfmt] == 1
    pl = synth.power_law(5000, 3, cap=4000)
    h2 = S.spmv_create(pl.n_rows, pl.n_cols, pl.row, pl.col, pl.values(np.float32))
    fmt2, times2 = S.spmv_select_format(h2, S.SPMV_SELECT_EXHAUSTIVE)
    assert np.isinf(times2[2]) and fmt2 != S.SPMV_FMT_ELL


def test_train_rejects_bad_orders():
    F, labels = _toy(N=20, seed=1)
    perms = synth.epoch_permutations(1, 20, 2)
    perms[1, 5] = 20
    with pytest.raises(S.SpmvError) as e:
        S.spmv_selector_train(_dev(F), _dev(labels), _dev(synth.glorot_params(1)), _dev(perms),
                              epochs=2, batch=8)
    assert e.value.status == "INVALID_ARG"


# ---- the six-class network (SELL and BELL as classes 4 and 5) -----------------------

L6 = (12, 64, 64, 6)


def _params6(seed):
    p = synth.glorot_params(seed, layers=L6).astype(np.float64)
    rng = np.random.default_rng(seed)
    p[768:832] = rng.uniform(-0.2, 0.2, 64)
    p[4928:4992] = rng.uniform(-0.2, 0.2, 64)
    p[5376:5382] = rng.uniform(-0.2, 0.2, 6)
    return p.astype(np.float32)


@pytest.mark.parametrize("B", [200, 13])
def test_six_class_loss_and_gradient_match_oracle(B):
    rng = np.random.default_rng(B + 100)
    p = _params6(5)
    Z = rng.standard_normal((B, 12)).astype(np.float32)
    y = rng.integers(0, 6, B).astype(np.int32)
    loss, grad = S.spmv_selector_loss_grad(_dev(p), _dev(Z), _dev(y), 1e-4)
    assert grad.numel() == 5382
    ref_loss, ref_grad = OM.loss_and_grad(p.astype(np.float64), Z.astype(np.float64), y, 1e-4)
    assert abs(float(loss.item()) - ref_loss) <= 1e-5 * abs(ref_loss)
    g = grad.cpu().numpy()
    for a, b in ((0, 768), (768, 832), (832, 4928), (4928, 4992), (4992, 5376), (5376, 5382)):
        assert _rel_l2(g[a:b], ref_grad[a:b]) <= 1e-4, (a, b)


def test_six_class_training_steps_and_prediction():
    rng = np.random.default_rng(31)
    N = 300
    labels = rng.integers(0, 6, N).astype(np.int32)
    F = (np.abs(rng.standard_normal((N, 12))) * 50 + 1).astype(np.float32)
    F[:, 2] = (3.0 ** labels * (1 + 0.2 * rng.random(N))).astype(np.float32)
    p0 = synth.glorot_params(31, layers=L6)
    perms = synth.epoch_permutations(31, N, 2)
    for steps in (1, 3):
        model = S.spmv_selector_train(_dev(F), _dev(labels), _dev(p0), _dev(perms), epochs=2,
                                      batch=64, max_steps=steps).cpu().numpy()
        assert model.size == 5406
        theta, mean, std, _ = OM.train(p0, F, labels, perms, batch=64, steps=steps)
        assert np.allclose(model[5382:5394], mean, rtol=1e-6, atol=1e-6)
        assert np.allclose(model[5394:5406], std, rtol=1e-5, atol=1e-6)
        d_gpu = model[:5382].astype(np.float64) - p0
        d_ref = theta - p0
        bad = np.abs(d_gpu - d_ref) > 2e-5 * steps + 1e-3 * np.abs(d_ref)
        assert bad.mean() <= 0.002, (steps, int(bad.sum()))
    app = (rng.random((N, 6)) < 0.6).astype(np.uint8)
    app[:, 0] = 1
    logits, cls = S.spmv_selector_predict(_dev(model), _dev(F), applicable=_dev(app))
    assert tuple(logits.shape) == (N, 6)
    mean, std = model[5382:5394].astype(np.float64), model[5394:5406].astype(np.float64)
    pred, _ = OM.predict(model[:5382], mean, std, F, applicable=app.astype(bool))
    refz = OM.forward(model[:5382].astype(np.float64), (OF.transform_features(F) - mean) / std)["logits"]
    assert np.allclose(logits.cpu().numpy(), refz, rtol=1e-4, atol=1e-4)
    got = cls.cpu().numpy()
    srt = np.sort(np.where(app.astype(bool), refz, -np.inf), axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 1e-3
    assert np.array_equal(got[clear], pred[clear]) and np.all(app[np.arange(N), got] == 1)
    with pytest.raises(S.SpmvError) as e:  # a label past the class count
        bad_labels = labels.copy()
        bad_labels[7] = 6
        S.spmv_selector_train(_dev(F), _dev(bad_labels), _dev(p0), _dev(perms), epochs=2, batch=64)
    assert e.value.status == "INVALID_ARG"


def test_select_format_model_mode_six_classes():
    bd = synth.block_diagonal(8 * 4096, 8, 41)
    h = S.spmv_create(bd.n_rows, bd.n_cols, bd.row, bd.col, bd.values(np.float32))
    model = np.zeros(5406, np.float32)
    model[5394:5406] = 1.0
    model[5376 + 5] = 3.0  # b3 favours BELL
    S.spmv_selector_set_weights(model)
    assert S.spmv_selector_classes() == 6
    assert np.array_equal(S.spmv_selector_get_weights(), model)
    fmt, scores = S.spmv_select_format(h, S.SPMV_SELECT_MODEL)
    assert fmt == S.SPMV_FMT_BELL and scores[5] == 3.0 and len(scores) == 6
    assert S.arrays_to_host(h, S.SPMV_FMT_BELL)["b"] == 8  # converted by the rule's block size
    # SELL is refused for a matrix with one very long row: the next best class is taken
    pl = synth.from_coords("long_row", 4096, 4096, np.r_[np.zeros(3000, int), np.arange(1, 4096)],
                           np.r_[np.arange(3000), np.arange(1, 4096)], 42)
    h2 = S.spmv_create(pl.n_rows, pl.n_cols, pl.row, pl.col, pl.values(np.float32))
    model[5376 + 5] = 0.0
    model[5376 + 4] = 3.0  # SELL first
    model[5376 + 2] = 2.0  # then ELL (refused too), then COO
    model[5376 + 1] = 1.0
    S.spmv_selector_set_weights(model)
    assert S.spmv_select_format(h2, S.SPMV_SELECT_MODEL)[0] == S.SPMV_FMT_COO
    logits, cls = S.spmv_selector_predict(None, _dev(np.ones((3, 12), np.float32)))
    assert tuple(logits.shape) == (3, 6) and (cls.cpu().numpy() == 4).all()
    S.spmv_selector_set_weights(None)
    assert S.spmv_selector_classes() == 0
