"""Energy, average power and efficiency of an SpMV from the board's energy
counter (paper, Experimental Setup: GPU performance monitoring).

The counter itself has no oracle: these tests check that a measurement is
internally consistent (energy per run = power x time per run, efficiency =
flops per joule), that the time per run agrees with the event timing of the
same variant, that the loaded board draws more than the idle one, that the
loop computed the right y, and the argument errors."""
import numpy as np
import pytest

import synth
from oracle import formats as OF
from oracle import spmv as OS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2302_05662_amd as S  # noqa: E402


@pytest.fixture(scope="module")
def banded():
    m = synth.banded(400_000, 16, 901)
    v = m.values(np.float32)
    h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, v)
    x = torch.from_numpy(m.x(np.float32)).cuda()
    y = torch.zeros(m.n_rows, dtype=torch.float32, device="cuda")
    return m, v, h, x, y


def test_energy_of_a_run_is_consistent(banded):
    m, v, h, x, y = banded
    idle = S.spmv_idle_power(0.2)
    assert 20.0 < idle < 3000.0, idle
    S.spmv_convert(h, S.SPMV_FMT_ELL)
    r = S.spmv_energy(h, S.SPMV_FMT_ELL, x, y, seconds=0.3)
    print({k: round(val, 6) for k, val in r.items()}, "idle", idle)
    assert r["seconds"] >= 0.25 and r["runs"] > 0
    assert 20.0 < r["watts"] < 3000.0
    assert r["watts"] > idle, (r["watts"], idle)
    assert r["joules"] == pytest.approx(r["watts"] * r["seconds"], rel=1e-9)
    assert r["joules_per_run"] == pytest.approx(r["watts"] * r["ms_per_run"] * 1e-3, rel=1e-9)
    assert r["mflops_per_watt"] == pytest.approx(2 * m.nnz / r["joules_per_run"] * 1e-6, rel=1e-9)
    warm = float(np.median(S.spmv_time(h, S.SPMV_FMT_ELL, x, y, warmup=3, reps=20, flush=False)))
    assert 0.5 * warm < r["ms_per_run"] < 2.0 * warm, (r["ms_per_run"], warm)
    # the loop ran y = A x
    canon = OF.canonicalize(m.n_rows, m.n_cols, m.row, m.col, v)
    xs = m.x(np.float32)
    ref = OS.spmv_csr(canon["row_ptr"], canon["col"], canon["val"], xs, 1.0, 0.0, None)
    den = OS.row_denominator(canon["row_ptr"], canon["col"], canon["val"], xs, 1.0, 0.0, None)
    torch.cuda.synchronize()
    assert OS.max_row_error(y.cpu().numpy(), ref, den) <= 1e-5


def test_energy_every_format_small(banded):
    m, v, h, x, y = banded
    for fmt in range(S.SPMV_NUM_FORMATS):
        S.spmv_convert(h, fmt)
        r = S.spmv_energy(h, fmt, x, y, seconds=0.05)
        assert r["runs"] > 0 and r["watts"] > 0 and r["joules_per_run"] > 0, (S.FORMAT_NAMES[fmt], r)


def test_energy_argument_errors(banded):
    m, v, h, x, y = banded
    with pytest.raises(S.SpmvError, match="INVALID_ARG"):
        S.spmv_energy(h, S.SPMV_FMT_CSR, x, y, seconds=0.0)
    with pytest.raises(S.SpmvError, match="INVALID_ARG"):
        S.spmv_energy(h, S.SPMV_FMT_CSR, x, y, seconds=61.0)
    with pytest.raises(S.SpmvError, match="INVALID_ARG"):
        S.spmv_idle_power(-1.0)
    h2 = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, v)
    with pytest.raises(S.SpmvError, match="NOT_CONVERTED"):
        S.spmv_energy(h2, S.SPMV_FMT_SELL, x, y, seconds=0.05)


def test_energy_sweep_of_formats(banded):
    m, v, h, x, y = banded
    fmts = [S.SPMV_FMT_CSR, S.SPMV_FMT_ELL, S.SPMV_FMT_BELL]
    for f in fmts:
        S.spmv_convert(h, f)
    res = S.spmv_energy_formats(h, fmts, x, y, seconds=0.05)
    assert len(res) == len(fmts)
    for f, r in zip(fmts, res):
        assert r["runs"] > 0 and 20.0 < r["watts"] < 3000.0, (S.FORMAT_NAMES[f], r)
        assert r["joules_per_run"] == pytest.approx(r["watts"] * r["ms_per_run"] * 1e-3, rel=1e-9)
        warm = float(np.median(S.spmv_time(h, f, x, y, warmup=3, reps=20, flush=False)))
        assert 0.5 * warm < r["ms_per_run"] < 2.0 * warm, (S.FORMAT_NAMES[f], r["ms_per_run"], warm)
    with pytest.raises(S.SpmvError, match="INVALID_ARG"):
        S.spmv_energy_formats(h, [9], x, y)
    with pytest.raises(ValueError):
        S.spmv_energy_formats(h, fmts, x, y, variants=[0])
