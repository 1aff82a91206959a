"""Full-size parity of the configurations the benchmark times, on every row.

* Five single-SpMV matrices at their real sizes in FP32, every compiled variant of
  every format (CSR, COO, ELL, HYB, SELL, BELL): the 936K-row banded matrix (seed
  2000, where the packed-index sorted blocks and BELL run), the 835K-row uniform
  random matrix with 50 entries per row (seed 2021), the 1.49M-row random matrix
  whose sorted blocks keep 16-bit rows (seed 2009), the 1.47M-row block-diagonal
  matrix (seed 2002, BELL at 8x8) and the 1.37M-row 3-D stencil (seed 2003, SELL).
* The 256-matrix batch (seeds 4000-4255, 3.6e8 entries) in one persistent launch,
  with the setting the autotuner picks and with the sorted-block tiling.

Every row of y is compared with the FP64 oracle at the FP32 bound of 1e-5
(per-row error over |alpha| sum_j |a_ij x_j| + |beta y_i|).
"""
import os

import numpy as np
import pytest

import synth
from oracle import spmv as OS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2302_05662_amd as S  # noqa: E402

TOL32 = 1e-5
THREADS = min(16, os.cpu_count() or 1)


def _row_ptr(m):
    rp = np.zeros(m.n_rows + 1, np.int64)
    np.cumsum(np.bincount(m.row, minlength=m.n_rows), out=rp[1:])
    return rp


def _reference(rp, col, val, x, a, b, y0):
    """(y_ref, D) over all rows: the oracle's FP64 loop, and the same loop on |A| |x|
    for D = |alpha| sum_j |a_ij x_j| + |beta| |y_i|."""
    y = OS.spmv_csr(rp, col, val, x, a, b, y0, n_threads=THREADS)
    d = OS.spmv_csr(rp, col, np.abs(val), np.abs(x), abs(a), abs(b),
                    np.abs(y0) if y0 is not None else None, n_threads=THREADS)
    return y, d


def _set_variant(h, fmt, var):
    try:
        S.spmv_set_variant(h, fmt, var)
        return True
    except S.SpmvError as e:
        if e.status != "NOT_APPLICABLE":
            raise
        return False


@pytest.mark.parametrize("seed", [2000, 2021, 2009, 2002, 2003])
def test_single_spmv_set_full_size_every_variant(seed):
    m = synth.config2_matrix(seed)
    print(f"[fullsize] {m.name} nnz={m.nnz} f32", flush=True)
    v = m.values(np.float32)
    x = m.x(np.float32)
    rp = _row_ptr(m)
    coo = [torch.from_numpy(a).cuda() for a in (m.row, m.col, v)]
    h = S.spmv_create(m.n_rows, m.n_cols, *coo)  # from device COO, as the benchmark does
    del coo
    xd = torch.from_numpy(x).cuda()
    fmts = [S.SPMV_FMT_CSR, S.SPMV_FMT_COO]
    for fmt in (S.SPMV_FMT_ELL, S.SPMV_FMT_HYB, S.SPMV_FMT_SELL, S.SPMV_FMT_BELL):
        try:
            S.spmv_convert(h, fmt)
            fmts.append(fmt)
        except S.SpmvError as e:
            assert e.status == "NOT_APPLICABLE" and fmt != S.SPMV_FMT_HYB
    cases = [(1.0, 0.0, None), (1.5, -0.5, synth.uniform_vector(m.n_rows, np.float32, [seed, 4]))]
    refs = [_reference(rp, m.col, v, x, a, b, y0) for a, b, y0 in cases]
    ran = 0
    for fmt in fmts:
        for var in range(S.spmv_variant_count(fmt, S.SPMV_F32)):
            if not _set_variant(h, fmt, var):
                continue
            for (a, b, y0), (y_ref, den) in zip(cases, refs):
                yd = (torch.from_numpy(y0).cuda() if y0 is not None
                      else torch.full((m.n_rows,), float("nan"), device="cuda"))
                S.spmv_run(h, fmt, a, xd, b, yd)
                err = OS.max_row_error(yd.cpu().numpy(), y_ref, den)
                assert err <= TOL32, (m.name, S.FORMAT_NAMES[fmt], var, a, b, err)
            ran += 1
    print(f"[fullsize] {m.name}: {ran} variants checked on all {m.n_rows} rows", flush=True)
    S.spmv_destroy(h)


def test_batched_set_full_size():
    specs = synth.config4_specs()
    hs, xs, ys, refs = [], [], [], []
    print(f"[fullsize batch] {len(specs)} matrices", flush=True)
    for sp in specs:
        m = synth.config4_matrix(sp)
        v = m.values(np.float32)
        x = m.x(np.float32)
        hs.append(S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, v))
        xs.append(torch.from_numpy(x).cuda())
        ys.append(torch.full((m.n_rows,), float("nan"), device="cuda"))
        refs.append(_reference(_row_ptr(m), m.col, v, x, 1.0, 0.0, None))
    print(f"[fullsize batch] {sum(h.nnz for h in hs)} entries on the device", flush=True)
    b = S.spmv_batch_create(hs, xs, ys, tune=True)
    tuned, _ = S.spmv_batch_get_config(b)
    settings = [None, dict(tiling=2, unroll=2, passes_per_tile=1, blocks_per_cu=2, lanes_divisor=1)]
    for setting in settings:
        if setting is not None:
            S.spmv_batch_set_config(b, **setting)
        cfg, _ = S.spmv_batch_get_config(b)
        for y in ys:
            y.fill_(float("nan"))
        S.spmv_batch_run(b)
        torch.cuda.synchronize()
        for i, (y_ref, den) in enumerate(refs):
            err = OS.max_row_error(ys[i].cpu().numpy(), y_ref, den)
            assert err <= TOL32, (specs[i], cfg, err)
        print(f"[fullsize batch] setting {cfg['tiling']}/{cfg['unroll']}/{cfg['blocks_per_cu']} "
              f"(tuned {tuned['tiling']}/{tuned['unroll']}/{tuned['blocks_per_cu']}): all rows ok",
              flush=True)
    S.spmv_batch_destroy(b)
