"""Collect the learned selector's data: features and per-format times of seeded matrices.

For each matrix (the 2-D Laplacian and the four single-SpMV families, seeds from
``synth.config5_specs``) this records, all measured on the GPU:

* the 12 sparsity features (``spmv_features``);
* a label pass: every applicable format autotuned over its variants, the
  median of ``tune_reps`` cache-flushed runs of the best variant;
* an independent check pass: ``check_reps`` more flushed runs of each format's
  chosen variant, used only to score selections (so regret is not measured on
  the timings that made the labels);
* the rule baseline's choice.

Results go to an ``.npz`` file that is rewritten every ``save_every`` matrices;
an interrupted collection resumes from it (seeds already present are skipped).

Usage: python -m paper_2302_05662_amd.selector_data OUT.npz FIRST_SEED LAST_SEED [--with-powerlaw]
(--with-powerlaw draws from the extended family set that adds the power law.)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

FIELDS = ("seed", "family", "n_rows", "nnz", "feats", "t_label", "t_check", "variant", "rule")


def _load(path):
    if not os.path.exists(path):
        return {k: [] for k in FIELDS}
    d = np.load(path, allow_pickle=False)
    return {k: list(d[k]) for k in FIELDS}


def _save(path, rec):
    tmp = path + ".tmp.npz"
    np.savez(tmp, **{k: np.array(v) for k, v in rec.items()})
    os.replace(tmp, path)


def collect(path, seeds, tune_reps=3, check_reps=5, save_every=25, log=print, families=None):
    import torch

    import paper_2302_05662_amd as S
    import synth

    torch.cuda.set_device(0)
    rec = _load(path)
    done = set(int(s) for s in rec["seed"])
    todo = [s for s in seeds if s not in done]
    t0 = time.perf_counter()
    fams = synth.CFG5_FAMILIES if families is None else families
    for i, spec in enumerate(synth.config5_specs(todo, families=fams)):
        m = synth.config5_matrix(spec)
        h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float32))
        feats = S.spmv_features(h)
        x = torch.from_numpy(m.x(np.float32)).cuda()
        y = torch.zeros(m.n_rows, dtype=torch.float32, device="cuda")
        t_label = np.full(4, np.inf)
        t_check = np.full(4, np.inf)
        variant = np.full(4, -1)
        for fmt in range(4):
            try:
                S.spmv_convert(h, fmt)
            except S.SpmvError as e:
                if e.status != "NOT_APPLICABLE":
                    raise
                continue
            variant[fmt], t_label[fmt] = S.spmv_tune(h, fmt, x, y, reps=tune_reps, flush=True)
        for fmt in range(4):
            if variant[fmt] >= 0:
                t_check[fmt] = float(np.median(S.spmv_time(h, fmt, x, y, warmup=1, reps=check_reps,
                                                           flush=True)))
        rule = S.spmv_select_format(h, S.SPMV_SELECT_RULE)[0]
        for k, v in zip(FIELDS, (spec["seed"], spec["family"], m.n_rows, m.nnz, feats, t_label,
                                 t_check, variant, rule)):
            rec[k].append(v)
        S.spmv_destroy(h)
        del m, x, y
        if (i + 1) % save_every == 0 or i + 1 == len(todo):
            _save(path, rec)
        log(f"[selector-data] {len(rec['seed'])} done, seed {spec['seed']} {spec['family']} "
            f"nnz={rec['nnz'][-1]} label={int(np.argmin(t_label))} "
            f"t={np.round(t_label * 1e3, 1).tolist()} us  ({time.perf_counter() - t0:.0f}s)")
    return rec


if __name__ == "__main__":
    out, first, last = sys.argv[1], int(sys.argv[2]), int(sys.argv[3])
    import synth as _synth

    fams = _synth.CFG5X_FAMILIES if "--with-powerlaw" in sys.argv[4:] else None
    collect(out, list(range(first, last + 1)), log=lambda s: print(s, flush=True), families=fams)
