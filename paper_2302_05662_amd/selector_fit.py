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

python -m paper_2302_05662_amd.selector_fit --extended DATA.npz EXT.npz evaluates, on a
set that adds the power-law family (seeds 7000-7599), the installed network and one
retrained on both training splits; it writes selector_eval_extended.json and
selector_model_extended.npy and leaves the installed network alone.
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


def _eval(pred, y, tc, fam=None, only=None):
    sel = np.ones(len(y), bool) if only is None else (fam == only)
    if not sel.any():
        return None
    return {"matrices": int(sel.sum()), "accuracy": float(np.mean(pred[sel] == y[sel])),
            **scores(pred[sel], tc[sel])}


def fit_extended(d, dx, seed=5, epochs=200):
    """The installed network and one retrained with the power-law family, on both held-out sets."""
    import torch

    import paper_2302_05662_amd as S
    import synth

    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    tr = (d["seed"] >= TRAIN_SEEDS[0]) & (d["seed"] <= TRAIN_SEEDS[1])
    he = (d["seed"] >= HELDOUT_SEEDS[0]) & (d["seed"] <= HELDOUT_SEEDS[1])
    trx = (dx["seed"] >= synth.CFG5X_TRAIN[0]) & (dx["seed"] <= synth.CFG5X_TRAIN[-1])
    hex_ = (dx["seed"] >= synth.CFG5X_HELDOUT[0]) & (dx["seed"] <= synth.CFG5X_HELDOUT[-1])
    sets = {"heldout": (d, he), "extended_heldout": (dx, hex_)}

    def predict(model, dd):
        applicable = np.isfinite(dd["t_check"]).astype(np.uint8)
        _, cls = S.spmv_selector_predict(model, dev(dd["feats"].astype(np.float32)),
                                         applicable=dev(applicable))
        return cls.cpu().numpy()

    installed = dev(np.load(MODEL_PATH, allow_pickle=False))
    F = np.concatenate([d["feats"][tr], dx["feats"][trx]]).astype(np.float32)
    y = np.concatenate([labels_of(d["t_label"][tr]), labels_of(dx["t_label"][trx])])
    retrained = S.spmv_selector_train(dev(F), dev(y), dev(synth.glorot_params(seed)),
                                      dev(synth.epoch_permutations(seed, len(y), epochs)),
                                      epochs=epochs)
    ev = {"extended_families": list(synth.CFG5X_FAMILIES),
          "extended_train_matrices": int(trx.sum()), "extended_heldout_matrices": int(hex_.sum()),
          "extended_label_histogram": np.bincount(labels_of(dx["t_label"]), minlength=4).tolist(),
          "retrained_on": int(len(y))}
    for name, model in (("installed", installed), ("retrained", retrained)):
        for sname, (dd, m) in sets.items():
            pred = predict(model, dd)[m]
            yy, tc, fam = labels_of(dd["t_label"])[m], dd["t_check"][m], dd["family"][m]
            ev[f"{name}_on_{sname}"] = _eval(pred, yy, tc)
            ev[f"{name}_on_{sname}_powerlaw"] = _eval(pred, yy, tc, fam, "powerlaw")
    for sname, (dd, m) in sets.items():
        tc = dd["t_check"][m]
        ev[f"always_csr_on_{sname}"] = scores(np.zeros(int(m.sum()), np.int64), tc)
        ev[f"rule_on_{sname}"] = scores(dd["rule"][m].astype(np.int64), tc)
    return retrained.cpu().numpy(), ev


if __name__ == "__main__":
    if sys.argv[1] == "--extended":
        model, ev = fit_extended(load([sys.argv[2]]), load([sys.argv[3]]))
        np.save(os.path.join(HERE, "selector_model_extended.npy"), model)
        with open(os.path.join(HERE, "selector_eval_extended.json"), "w") as fh:
            json.dump(ev, fh, indent=1)
        print(json.dumps(ev, indent=1))
        sys.exit(0)
    data = load(sys.argv[1:])
    model, ev = fit(data)
    np.save(MODEL_PATH, model)
    with open(EVAL_PATH, "w") as fh:
        json.dump(ev, fh, indent=1)
    print(json.dumps(ev, indent=1))
