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

python -m paper_2302_05662_amd.selector_fit --four-from-six DATA6.npz does the same on the
first four formats of a six-format collection and writes that view as
selector_data_mi355x.npz (one collection serves both networks).

python -m paper_2302_05662_amd.selector_fit --six DATA6.npz trains the six-class network
(SELL and BELL as classes 4 and 5) on a dataset collected with ``selector_data --six`` and
fits the overhead-aware run-time model on it; it writes selector_model6.npy,
selector_runtime.npy and selector_eval6.json.

python -m paper_2302_05662_amd.selector_fit --energy ENERGY.npz trains the energy head (the
six-class network on the least-energy format per matrix, collected with ``selector_data
--energy``) and a power head, and scores them on the check pass; it writes
selector_model6_energy.npy, selector_model6_power.npy and selector_eval_energy.json.

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


LOG_COLS = (0, 1, 2, 3, 4, 5, 6, 8, 9)  # the selector's log2(1 + v) inputs
NF6 = 6


def runtime_inputs(F):
    """The selector's input map (before standardisation) and an intercept column."""
    T = np.array(F, dtype=np.float64, copy=True)
    T[:, LOG_COLS] = np.log2(1.0 + T[:, LOG_COLS])
    return np.concatenate([T, np.ones((T.shape[0], 1))], axis=1)


def fit_runtime(d, train):
    """Run-time model: per format a least-squares fit of log(time ms) on the selector's inputs,
    and of the conversion latency (ms) on 1, nnz / 1e6 and n_rows / 1e6."""
    X = runtime_inputs(d["feats"])
    params = np.zeros(NF6 * 13 + NF6 * 3)
    for f in range(NF6):
        ok = train & np.isfinite(d["t_label"][:, f])
        w, *_ = np.linalg.lstsq(X[ok], np.log(d["t_label"][ok, f]), rcond=None)
        params[f * 13:(f + 1) * 13] = w
    A = np.stack([np.ones(len(d["nnz"])), d["nnz"] / 1e6, d["n_rows"] / 1e6], axis=1)
    for f in range(2, NF6):
        ok = train & np.isfinite(d["t_label"][:, f])
        c, *_ = np.linalg.lstsq(A[ok], d["t_convert"][ok, f], rcond=None)
        params[NF6 * 13 + f * 3:NF6 * 13 + f * 3 + 3] = c
    return params.astype(np.float32)


def runtime_eval(d, held, pred, params, iterations=(1, 10, 100, 1000, 10000)):
    """Total time of `iterations` SpMVs starting from CSR, per held-out matrix, for: never
    converting, always converting to the network's choice, the overhead-aware decision, and the
    best decision in hindsight (measured check-pass times and measured conversion latencies;
    feature and prediction latencies are paid by every mode that predicts)."""
    X = runtime_inputs(d["feats"][held])
    tc = d["t_check"][held]
    conv = d["t_convert"][held]
    feat = d["t_feat"][held]
    nnz, n = d["nnz"][held] / 1e6, d["n_rows"][held] / 1e6
    p = pred[held]
    W = params[:NF6 * 13].reshape(NF6, 13).astype(np.float64)
    Cc = params[NF6 * 13:].reshape(NF6, 3).astype(np.float64)
    t_est = np.exp(X @ W.T)
    c_est = np.where(np.arange(NF6)[None, :] >= 2,
                     np.maximum(0, Cc[:, 0][None, :] + Cc[:, 1][None, :] * nnz[:, None]
                                + Cc[:, 2][None, :] * n[:, None]), 0.0)
    idx = np.arange(len(p))
    out = {"log_time_abs_error_median": {}, "convert_ms_abs_error_median": {}}
    for f in range(NF6):
        ok = np.isfinite(tc[:, f])
        out["log_time_abs_error_median"][str(f)] = float(np.median(np.abs(np.log(t_est[ok, f]) - np.log(tc[ok, f]))))
        if f >= 2:
            out["convert_ms_abs_error_median"][str(f)] = float(np.median(np.abs(c_est[ok, f] - conv[ok, f])))
    rows = []
    for it in iterations:
        never = tc[:, 0] * it
        always = feat + conv[idx, p] * (p != 0) + tc[idx, p] * it
        gain = (t_est[:, 0] - t_est[idx, p]) * it
        switch = (p != 0) & (gain > feat + c_est[idx, p])
        aware = feat + np.where(switch, conv[idx, p] + tc[idx, p] * it, tc[:, 0] * it)
        allc = np.where(np.isfinite(tc), conv + tc * it, np.inf)
        allc[:, 0] = tc[:, 0] * it
        best = np.minimum(never, feat + allc.min(axis=1))
        rows.append({"iterations": it,
                     "never_convert_over_best": float(never.sum() / best.sum()),
                     "always_convert_over_best": float(always.sum() / best.sum()),
                     "overhead_aware_over_best": float(aware.sum() / best.sum()),
                     "switched_fraction": float(switch.mean())})
    out["total_time_by_iterations"] = rows
    return out


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


def fit6(d, seed=5, epochs=200):
    """Six-class network and run-time model on a dataset collected with --six."""
    import torch

    import paper_2302_05662_amd as S
    import synth

    train = (d["seed"] >= TRAIN_SEEDS[0]) & (d["seed"] <= TRAIN_SEEDS[1])
    held = (d["seed"] >= HELDOUT_SEEDS[0]) & (d["seed"] <= HELDOUT_SEEDS[1])
    F = d["feats"].astype(np.float32)
    y = labels_of(d["t_label"])
    n = int(train.sum())
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    model = S.spmv_selector_train(dev(F[train]), dev(y[train]),
                                  dev(synth.glorot_params(seed, layers=(12, 64, 64, NF6))),
                                  dev(synth.epoch_permutations(seed, n, epochs)), epochs=epochs)
    applicable = np.isfinite(d["t_check"]).astype(np.uint8)
    _, cls = S.spmv_selector_predict(model, dev(F), applicable=dev(applicable))
    pred = cls.cpu().numpy()
    tc = d["t_check"]
    y4 = labels_of(d["t_label"][:, :4])
    ev = {"train_matrices": n, "heldout_matrices": int(held.sum()),
          "label_histogram_train": np.bincount(y[train], minlength=NF6).tolist(),
          "label_histogram_heldout": np.bincount(y[held], minlength=NF6).tolist(),
          "train_accuracy": float(np.mean(pred[train] == y[train])),
          "heldout_accuracy": float(np.mean(pred[held] == y[held])),
          "model": scores(pred[held], tc[held]),
          "always_csr": scores(np.zeros(int(held.sum()), np.int64), tc[held]),
          "rule": scores(d["rule"][held].astype(np.int64), tc[held]),
          "best_of_csr_coo_ell_hyb": scores(y4[held], tc[held]),
          "label_pass_on_check_timings": scores(y[held], tc[held])}
    rt = fit_runtime(d, train)
    ev["runtime_mode"] = runtime_eval(d, held, pred, rt)
    return model.cpu().numpy(), rt, ev


def fit_energy(d, latency_model=None, seed=5, epochs=200):
    """Energy head: the six-class network trained on energy labels (the format with the
    least board energy per SpMV in the label pass), scored on the check pass's energy,
    beside the power objective (least average power) and the latency-trained network
    used for energy. Energy per SpMV and MFLOPS per watt rank formats identically
    (the flops are fixed per matrix), so one label set serves both."""
    import torch

    import paper_2302_05662_amd as S
    import synth

    train = (d["seed"] >= TRAIN_SEEDS[0]) & (d["seed"] <= TRAIN_SEEDS[1])
    held = (d["seed"] >= HELDOUT_SEEDS[0]) & (d["seed"] <= HELDOUT_SEEDS[1])
    F = d["feats"].astype(np.float32)
    y = labels_of(d["e_label"])
    yw = labels_of(d["w_label"])
    yt = labels_of(d["t_label"])
    n = int(train.sum())
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    applicable = np.isfinite(d["e_check"]).astype(np.uint8)

    def train_on(labels):
        return S.spmv_selector_train(dev(F[train]), dev(labels[train]),
                                     dev(synth.glorot_params(seed, layers=(12, 64, 64, NF6))),
                                     dev(synth.epoch_permutations(seed, n, epochs)), epochs=epochs)

    def predict(model):
        _, cls = S.spmv_selector_predict(model, dev(F), applicable=dev(applicable))
        return cls.cpu().numpy()

    model_e = train_on(y)
    model_w = train_on(yw)
    pe, pw = predict(model_e), predict(model_w)
    ec, wc = d["e_check"][held], d["w_check"][held]
    tc = d["ms_check"][held]
    ev = {"train_matrices": n, "heldout_matrices": int(held.sum()),
          "idle_watts_median": float(np.median(d["idle_w"])),
          "energy_label_histogram_train": np.bincount(y[train], minlength=NF6).tolist(),
          "energy_label_histogram_heldout": np.bincount(y[held], minlength=NF6).tolist(),
          "power_label_histogram_heldout": np.bincount(yw[held], minlength=NF6).tolist(),
          "energy_label_equals_latency_label": float(np.mean(y == yt)),
          "energy": {"model_energy": scores(pe[held], ec),
                     "heldout_accuracy": float(np.mean(pe[held] == y[held])),
                     "always_csr": scores(np.zeros(int(held.sum()), np.int64), ec),
                     "rule": scores(d["rule"][held].astype(np.int64), ec),
                     "latency_labels": scores(yt[held], ec),
                     "label_pass_on_check": scores(y[held], ec)},
          "power": {"model_power": scores(pw[held], wc),
                    "heldout_accuracy": float(np.mean(pw[held] == yw[held])),
                    "always_csr": scores(np.zeros(int(held.sum()), np.int64), wc),
                    "latency_labels": scores(yt[held], wc),
                    "energy_model": scores(pe[held], wc)},
          "latency_of_energy_choice": scores(pe[held], tc)}
    if latency_model is not None:
        pl = predict(torch.from_numpy(latency_model).cuda())
        ev["energy"]["latency_model"] = scores(pl[held], ec)
    # spread of power across formats on one matrix: the paper's observation that the
    # format moves power even where latency barely moves
    wl = np.where(np.isfinite(d["w_label"]), d["w_label"], np.nan)
    spread = np.nanmax(wl, axis=1) / np.nanmin(wl, axis=1) - 1
    ev["power_spread_across_formats_median"] = float(np.nanmedian(spread))
    ev["power_spread_across_formats_p95"] = float(np.nanpercentile(spread, 95))
    return model_e.cpu().numpy(), model_w.cpu().numpy(), ev


def four_of_six(d):
    """The four-format view (CSR, COO, ELL, HYB) of a dataset collected with --six."""
    keep = ("seed", "family", "n_rows", "nnz", "feats", "t_label", "t_check", "variant", "rule")
    out = {k: d[k] for k in keep}
    for k in ("t_label", "t_check", "variant"):
        out[k] = np.ascontiguousarray(d[k][:, :4])
    return out


if __name__ == "__main__":
    if sys.argv[1] == "--four-from-six":
        # the installed 4-class network and its dataset, from the six-format collection
        d4 = four_of_six(load([sys.argv[2]]))
        np.savez(os.path.join(HERE, "selector_data_mi355x.npz"), **d4)
        model, ev = fit(d4)
        np.save(MODEL_PATH, model)
        with open(EVAL_PATH, "w") as fh:
            json.dump(ev, fh, indent=1)
        print(json.dumps(ev, indent=1))
        sys.exit(0)
    if sys.argv[1] == "--energy":
        lat = os.path.join(HERE, "selector_model6.npy")
        model_e, model_w, ev = fit_energy(load([sys.argv[2]]),
                                          np.load(lat) if os.path.exists(lat) else None)
        np.save(os.path.join(HERE, "selector_model6_energy.npy"), model_e)
        np.save(os.path.join(HERE, "selector_model6_power.npy"), model_w)
        with open(os.path.join(HERE, "selector_eval_energy.json"), "w") as fh:
            json.dump(ev, fh, indent=1)
        print(json.dumps(ev, indent=1))
        sys.exit(0)
    if sys.argv[1] == "--six":
        model, rt, ev = fit6(load([sys.argv[2]]))
        np.save(os.path.join(HERE, "selector_model6.npy"), model)
        np.save(os.path.join(HERE, "selector_runtime.npy"), rt)
        with open(os.path.join(HERE, "selector_eval6.json"), "w") as fh:
            json.dump(ev, fh, indent=1)
        print(json.dumps(ev, indent=1))
        sys.exit(0)
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
