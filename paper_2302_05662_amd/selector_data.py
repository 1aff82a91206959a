"""Collect the learned selector's data: features and per-format times of seeded matrices.

For each matrix (the 2-D Laplacian and the four single-SpMV families, seeds from
``synth.config5_specs``) this records, all measured on the GPU:

* the 12 sparsity features (``spmv_features``);
* a label pass: every applicable format autotuned over its variants, the
  median of ``tune_reps`` cache-flushed runs of the best variant;
* an independent check pass: ``check_reps`` more flushed runs of each format's
  chosen variant, used only to score selections (so regret is not measured on
  the timings that made the labels);
* the rule baseline's choice;
* with ``--six``: all six formats (CSR, COO, ELL, HYB, SELL, BELL), plus the
  latency of the features call and of each format's conversion (host clock
  around the synchronous calls) and the bytes each tuned variant streams,
  which the overhead-aware run-time mode is fitted on.

Results go to an ``.npz`` file that is rewritten every ``save_every`` matrices;
an interrupted collection resumes from it (seeds already present are skipped).

Usage: python -m paper_2302_05662_amd.selector_data OUT.npz FIRST_SEED LAST_SEED [--with-powerlaw]
       [--six] [--interleave] [--limit-s SECONDS]
       python -m paper_2302_05662_amd.selector_data --energy OUT.npz FIRST LAST STEP [--limit-s S]
(--with-powerlaw draws from the extended family set that adds the power law; --limit-s
stops after that many seconds, the saved file resuming later; --interleave takes the seeds
round-robin over the four quarters of the range, so a partial collection holds held-out
matrices too.)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

FIELDS = ("seed", "family", "n_rows", "nnz", "feats", "t_label", "t_check", "variant", "rule")
FIELDS6 = FIELDS + ("t_feat", "t_convert", "bytes")


def _load(path, fields=FIELDS):
    if not os.path.exists(path):
        return {k: [] for k in fields}
    d = np.load(path, allow_pickle=False)
    return {k: list(d[k]) for k in fields}


def _save(path, rec):
    tmp = path + ".tmp.npz"
    np.savez(tmp, **{k: np.array(v) for k, v in rec.items()})
    os.replace(tmp, path)


def collect(path, seeds, tune_reps=3, check_reps=5, save_every=25, log=print, families=None,
            six=False, limit_s=None):
    import torch

    import paper_2302_05662_amd as S
    import synth

    torch.cuda.set_device(0)
    nf = 6 if six else 4
    fields = FIELDS6 if six else FIELDS
    rec = _load(path, fields)
    done = set(int(s) for s in rec["seed"])
    todo = [s for s in seeds if s not in done]
    t0 = time.perf_counter()
    fams = synth.CFG5_FAMILIES if families is None else families
    for i, spec in enumerate(synth.config5_specs(todo, families=fams)):
        m = synth.config5_matrix(spec)
        h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float32))
        t = time.perf_counter()
        feats = S.spmv_features(h)
        t_feat = (time.perf_counter() - t) * 1e3
        x = torch.from_numpy(m.x(np.float32)).cuda()
        y = torch.zeros(m.n_rows, dtype=torch.float32, device="cuda")
        t_label = np.full(nf, np.inf)
        t_check = np.full(nf, np.inf)
        t_convert = np.zeros(nf)
        nbytes = np.zeros(nf, np.int64)
        variant = np.full(nf, -1)
        for fmt in range(nf):
            try:
                t = time.perf_counter()
                S.spmv_convert(h, fmt)
                t_convert[fmt] = (time.perf_counter() - t) * 1e3
            except S.SpmvError as e:
                if e.status != "NOT_APPLICABLE":
                    raise
                continue
            variant[fmt], t_label[fmt] = S.spmv_tune(h, fmt, x, y, reps=tune_reps, flush=True)
            nbytes[fmt] = S.spmv_stored_bytes(h, fmt)
        for fmt in range(nf):
            if variant[fmt] >= 0:
                t_check[fmt] = float(np.median(S.spmv_time(h, fmt, x, y, warmup=1, reps=check_reps,
                                                           flush=True)))
        rule = S.spmv_select_format(h, S.SPMV_SELECT_RULE)[0]
        vals = [spec["seed"], spec["family"], m.n_rows, m.nnz, feats, t_label, t_check, variant, rule]
        if six:
            vals += [t_feat, t_convert, nbytes]
        for k, v in zip(fields, vals):
            rec[k].append(v)
        S.spmv_destroy(h)
        del m, x, y
        stop = limit_s is not None and time.perf_counter() - t0 > limit_s
        if (i + 1) % save_every == 0 or i + 1 == len(todo) or stop:
            _save(path, rec)
        log(f"[selector-data] {len(rec['seed'])} done, seed {spec['seed']} {spec['family']} "
            f"nnz={rec['nnz'][-1]} label={int(np.argmin(t_label))} "
            f"t={np.round(t_label * 1e3, 1).tolist()} us  ({time.perf_counter() - t0:.0f}s)")
        if stop:
            break
    return rec


FIELDS_ENERGY = ("seed", "family", "n_rows", "nnz", "feats", "variant", "t_label", "rule",
                 "e_label", "w_label", "ms_label", "e_check", "w_check", "ms_check", "idle_w")


def collect_energy(path, seeds, seconds=0.2, tune_reps=3, save_every=10, log=print, limit_s=None,
                   check_from=6500):
    """Energy labels: per matrix, every format (of six) autotuned for time, then the
    board energy and average power of its tuned variant run back to back, all formats
    in one counter sweep (``spmv_energy_formats``): a label pass, and on the held-out
    seeds (>= check_from) an independent check pass used for scoring."""
    import torch

    import paper_2302_05662_amd as S
    import synth

    torch.cuda.set_device(0)
    nf = 6
    rec = _load(path, FIELDS_ENERGY)
    done = set(int(s) for s in rec["seed"])
    todo = [s for s in seeds if s not in done]
    t0 = time.perf_counter()
    for i, spec in enumerate(synth.config5_specs(todo)):
        m = synth.config5_matrix(spec)
        h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float32))
        feats = S.spmv_features(h)
        x = torch.from_numpy(m.x(np.float32)).cuda()
        y = torch.zeros(m.n_rows, dtype=torch.float32, device="cuda")
        variant = np.full(nf, -1)
        t_label = np.full(nf, np.inf)
        e = {k: np.full(nf, np.inf) for k in ("e_label", "w_label", "ms_label", "e_check",
                                              "w_check", "ms_check")}
        for fmt in range(nf):
            try:
                S.spmv_convert(h, fmt)
            except S.SpmvError as err:
                if err.status != "NOT_APPLICABLE":
                    raise
                continue
            variant[fmt], t_label[fmt] = S.spmv_tune(h, fmt, x, y, reps=tune_reps, flush=True)
        if i % 25 == 0:  # the idle draw drifts slowly: measured every 25 matrices
            idle = S.spmv_idle_power(seconds)
        fmts = [f for f in range(nf) if variant[f] >= 0]
        # the check pass (scoring only) is measured on the held-out matrices
        tags = ("label", "check") if spec["seed"] >= check_from else ("label",)
        for tag in tags:
            # one sweep per pass, the formats in a rotated order so no format always
            # follows the same one
            order = fmts[len(rec["seed"]) % len(fmts):] + fmts[:len(rec["seed"]) % len(fmts)]
            res = S.spmv_energy_formats(h, order, x, y, seconds=seconds)
            for fmt, r in zip(order, res):
                e[f"e_{tag}"][fmt] = r["joules_per_run"]
                e[f"w_{tag}"][fmt] = r["watts"]
                e[f"ms_{tag}"][fmt] = r["ms_per_run"]
        rule = S.spmv_select_format(h, S.SPMV_SELECT_RULE)[0]
        vals = [spec["seed"], spec["family"], m.n_rows, m.nnz, feats, variant, t_label, rule,
                e["e_label"], e["w_label"], e["ms_label"], e["e_check"], e["w_check"],
                e["ms_check"], idle]
        for k, v in zip(FIELDS_ENERGY, vals):
            rec[k].append(v)
        S.spmv_destroy(h)
        del m, x, y
        stop = limit_s is not None and time.perf_counter() - t0 > limit_s
        if (i + 1) % save_every == 0 or i + 1 == len(todo) or stop:
            _save(path, rec)
        log(f"[energy-data] {len(rec['seed'])} done, seed {spec['seed']} {spec['family']} "
            f"nnz={rec['nnz'][-1]} uJ={np.round(e['e_label'] * 1e6, 1).tolist()} "
            f"W={np.round(e['w_label'], 0).tolist()} idle={idle:.0f}W "
            f"({time.perf_counter() - t0:.0f}s)")
        if stop:
            break
    return rec


def interleaved(seeds, parts=4):
    """The seeds in round-robin order over `parts` contiguous ranges, so a collection
    stopped early still holds every range (the last quarter of the selector seeds is the
    held-out split)."""
    n = len(seeds)
    stride = max(1, n // parts)
    return [seeds[i] for i in sorted(range(n), key=lambda i: (i % stride, i))]


if __name__ == "__main__":
    if sys.argv[1] == "--energy":
        # --energy OUT.npz FIRST LAST STEP [--limit-s SECONDS]
        out, first, last, step = sys.argv[2], int(sys.argv[3]), int(sys.argv[4]), int(sys.argv[5])
        opts = sys.argv[6:]
        limit = float(opts[opts.index("--limit-s") + 1]) if "--limit-s" in opts else None
        collect_energy(out, interleaved(list(range(first, last + 1, step))),
                       log=lambda s: print(s, flush=True), limit_s=limit)
        sys.exit(0)
    out, first, last = sys.argv[1], int(sys.argv[2]), int(sys.argv[3])
    import synth as _synth

    opts = sys.argv[4:]
    fams = _synth.CFG5X_FAMILIES if "--with-powerlaw" in opts else None
    limit = float(opts[opts.index("--limit-s") + 1]) if "--limit-s" in opts else None
    seeds = list(range(first, last + 1))
    collect(out, interleaved(seeds) if "--interleave" in opts else seeds,
            log=lambda s: print(s, flush=True), families=fams, six="--six" in opts, limit_s=limit)
