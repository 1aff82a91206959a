"""The trained selector on the GPU: held-out regret against exhaustive timing and baselines."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2302_05662_amd as S  # noqa: E402

PKG = os.path.dirname(S.__file__)


def test_learned_selector_gain_over_the_method_without_it():
    d = np.load(os.path.join(PKG, "selector_data_mi355x.npz"), allow_pickle=False)
    model = np.load(os.path.join(PKG, "selector_model.npy"))
    held = d["seed"] >= 6500
    t = d["t_check"][held]
    F = torch.from_numpy(np.ascontiguousarray(d["feats"][held])).cuda()
    app = torch.from_numpy(np.isfinite(t).astype(np.uint8)).cuda()
    _, cls = S.spmv_selector_predict(torch.from_numpy(model).cuda(), F, applicable=app)
    chosen = cls.cpu().numpy()
    best = t.min(axis=1)
    r_model = t[np.arange(len(chosen)), chosen] / best - 1
    r_csr = t[:, 0] / best - 1
    r_rule = t[np.arange(len(chosen)), d["rule"][held]] / best - 1
    print(f"held-out mean regret: model {r_model.mean():.4f}, always-CSR {r_csr.mean():.4f}, "
          f"rule {r_rule.mean():.4f}", flush=True)
    assert r_model.mean() <= 0.05
    assert r_model.mean() < r_csr.mean() and r_model.mean() < r_rule.mean()
    assert np.all(np.isfinite(t[np.arange(len(chosen)), chosen]))  # never an inapplicable format


def test_six_class_selector_on_held_out_matrices():
    """The 6-class network (SELL and BELL added) through the library's predict kernel, on
    the 500 held-out matrices of the six-format collection."""
    d = np.load(os.path.join(PKG, "selector_data6_mi355x.npz"), allow_pickle=False)
    model = np.load(os.path.join(PKG, "selector_model6.npy"))
    held = d["seed"] >= 6500
    t = d["t_check"][held]
    F = torch.from_numpy(np.ascontiguousarray(d["feats"][held])).cuda()
    app = torch.from_numpy(np.isfinite(t).astype(np.uint8)).cuda()
    _, cls = S.spmv_selector_predict(torch.from_numpy(model).cuda(), F, applicable=app)
    chosen = cls.cpu().numpy()
    best = t.min(axis=1)
    r_model = t[np.arange(len(chosen)), chosen] / best - 1
    r_csr = t[:, 0] / best - 1
    four = np.where(np.isfinite(t[:, :4]), t[:, :4], np.inf).min(axis=1) / best - 1
    print(f"6-class held-out mean regret: model {r_model.mean():.4f}, always-CSR {r_csr.mean():.4f}, "
          f"best of CSR/COO/ELL/HYB {four.mean():.4f}", flush=True)
    assert r_model.mean() <= 0.05
    assert r_model.mean() < r_csr.mean() and r_model.mean() < four.mean()
    assert np.all(np.isfinite(t[np.arange(len(chosen)), chosen]))
