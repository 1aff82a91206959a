"""Train the selector network on the GPU and evaluate it on held-out matrices.

Labels are the fastest format of the label pass (ties to the lowest format
number). Training follows the paper's MLP recipe (Setup, learning algorithms:
ReLU, Adam, learning rate 0.001, 200 epochs; scikit-learn defaults otherwise:
minibatch min(200, n), L2 alpha 1e-4), run by ``spmv_selector_train``.
Held-out selections are scored on the independent check-pass timings:
regret = t(chosen) / t(best) - 1, against always-CSR, the rule and the
majority class.

Usage: python -m paper_2302_05662_amd.selector_fit DATA.npz [DATA2.npz ...]
writes selector_model.npy and selector_eval.json next to this file.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(HERE, "selector_model.npy")
EVAL_PATH = os.path.join(HERE, "selector_eval.json")
TRAIN_SEEDS = (5000, 6499)
HELDOUT_SEEDS = (6500, 6999)


def load(paths):
    parts = [np.load(p, allow_pickle=False) for p in paths]
    d = {k: np.concatenate([p[k] for p in parts]) for k in parts[0].files}
    _, first = np.unique(d["seed"], return_index=True)
    return {k: v[first] for k, v in d.items()}


def labels_of(t):
    return np.argmin(np.where(np.isfinite(t), t, np.inf), axis=1).astype(np.int32)


def scores(chosen, t_check):
    best = np.min(t_check, axis=1)
    r = t_check[np.arange(len(chosen)), chosen] / best - 1.0
    return {"mean_regret": float(np.mean(r)), "p95_regret": float(np.percentile(r, 95)),
            "max_regret": float(np.max(r)),
            "total_time_regret": float(t_check[np.arange(len(chosen)), chosen].sum() / best.sum() - 1),
            "within_5pct": float(np.mean(r <= 0.05))}


def fit(d, seed=5, epochs=200):
    import torch

    import paper_2302_05662_amd as S
    import synth

    train = (d["seed"] >= TRAIN_SEEDS[0]) & (d["seed"] <= TRAIN_SEEDS[1])
    held = (d["seed"] >= HELDOUT_SEEDS[0]) & (d["seed"] <= HELDOUT_SEEDS[1])
    F = d["feats"].astype(np.float32)
    y = labels_of(d["t_label"])
    n = int(train.sum())
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    t = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t[0].record()
    model = S.spmv_selector_train(dev(F[train]), dev(y[train]), dev(synth.glorot_params(seed)),
                                  dev(synth.epoch_permutations(seed, n, epochs)), epochs=epochs)
    t[1].record()
    torch.cuda.synchronize()
    train_ms = t[0].elapsed_time(t[1])
    applicable = np.isfinite(d["t_check"]).astype(np.uint8)
    _, cls = S.spmv_selector_predict(model, dev(F), applicable=dev(applicable))
    pred = cls.cpu().numpy()
    tc = d["t_check"]
    majority = int(np.bincount(y[train], minlength=4).argmax())
    ev = {"train_matrices": n, "heldout_matrices": int(held.sum()), "train_ms_gpu": train_ms,
          "label_histogram_train": np.bincount(y[train], minlength=4).tolist(),
          "label_histogram_heldout": np.bincount(y[held], minlength=4).tolist(),
          "train_accuracy": float(np.mean(pred[train] == y[train])),
          "heldout_accuracy": float(np.mean(pred[held] == y[held])),
          "model": scores(pred[held], tc[held]),
          "always_csr": scores(np.zeros(int(held.sum()), np.int64), tc[held]),
          "rule": scores(d["rule"][held].astype(np.int64), tc[held]),
          "majority_class": {"class": majority,
                             **scores(np.where(applicable[held][:, majority] > 0, majority, 0),
                                      tc[held])},
          "label_pass_on_check_timings": scores(y[held], tc[held])}
    return model.cpu().numpy(), ev


if __name__ == "__main__":
    data = load(sys.argv[1:])
    model, ev = fit(data)
    np.save(MODEL_PATH, model)
    with open(EVAL_PATH, "w") as fh:
        json.dump(ev, fh, indent=1)
    print(json.dumps(ev, indent=1))
