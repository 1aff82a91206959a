"""GPU ingest and conversion parity: every index and value array bit-equal to the oracle's."""
import numpy as np
import pytest

import _cases as C
import synth
from oracle import formats as OF

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2302_05662_amd as S  # noqa: E402

DTYPES = [np.float32, np.float64]


def _create(name, dtype, on_device=False):
    m = C.matrix(name)
    r, c, v = C.shuffled_input(name, dtype)
    if on_device:
        r, c, v = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (r, c, v))
    return S.spmv_create(m.n_rows, m.n_cols, r, c, v)


def _same_bits(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return a.dtype == b.dtype and a.shape == b.shape and a.tobytes() == b.tobytes()


def _check_canonical(h, ref):
    csr = S.arrays_to_host(h, S.SPMV_FMT_CSR)
    assert np.array_equal(csr["row_ptr"], ref["row_ptr"].astype(np.int32))
    assert _same_bits(csr["col"], ref["col"])
    assert _same_bits(csr["val"], ref["val"])
    coo = S.arrays_to_host(h, S.SPMV_FMT_COO)
    assert _same_bits(coo["row"], ref["row"])
    assert _same_bits(coo["col"], ref["col"])
    assert _same_bits(coo["val"], ref["val"])


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("name", list(C.CASES))
def test_canonical_csr_and_coo(name, dtype):
    print(f"[ingest] {name} {dtype.__name__}", flush=True)
    h = _create(name, dtype)
    _check_canonical(h, C.canonical(name, dtype))


@pytest.mark.parametrize("name", ["random", "powerlaw", "lap64", "empty"])
def test_device_input(name):
    print(f"[ingest device] {name}", flush=True)
    h = _create(name, np.float32, on_device=True)
    _check_canonical(h, C.canonical(name, np.float32))


def test_sorted_input_fast_path():
    m = C.matrix("random")
    v = m.values(np.float32)
    h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, v)
    _check_canonical(h, OF.canonicalize(m.n_rows, m.n_cols, m.row, m.col, v))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("name", list(C.CASES))
def test_ell_and_hyb(name, dtype):
    print(f"[convert] {name} {dtype.__name__}", flush=True)
    h = _create(name, dtype)
    ref = C.canonical(name, dtype)
    try:
        e = OF.to_ell(ref)
    except OF.OracleError as err:
        assert err.status == OF.NOT_APPLICABLE
        with pytest.raises(S.SpmvError) as got:
            S.spmv_convert(h, S.SPMV_FMT_ELL)
        assert got.value.status == "NOT_APPLICABLE"
        with pytest.raises(S.SpmvError) as got:
            S.spmv_get_arrays(h, S.SPMV_FMT_ELL)
        assert got.value.status == "NOT_CONVERTED"
    else:
        S.spmv_convert(h, S.SPMV_FMT_ELL)
        g = S.arrays_to_host(h, S.SPMV_FMT_ELL)
        assert (g["K"], g["pitch"]) == (e["K"], e["pitch"])
        assert _same_bits(g["ell_col"], e["ell_col"])
        assert _same_bits(g["ell_val"], e["ell_val"])
    for k in (-1, 0, 1, 3):
        hy = OF.to_hyb(ref, k_override=k)
        S.spmv_convert(h, S.SPMV_FMT_HYB, k)
        g = S.arrays_to_host(h, S.SPMV_FMT_HYB)
        assert (g["K"], g["pitch"], g["nnz_tail"]) == (hy["K"], hy["pitch"], hy["tail_row"].size), k
        for key in ("ell_col", "ell_val", "tail_row", "tail_col", "tail_val"):
            assert _same_bits(g[key], hy[key]), (k, key)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("name", list(C.CASES))
def test_sell_and_bell(name, dtype):
    """SELL (sigma by the rule, 1, 128, 16384) and BELL (size by the rule, 2, 4, 8): every
    array bit-equal to the oracle's layout, or NOT_APPLICABLE where the oracle refuses."""
    print(f"[convert sell/bell] {name} {dtype.__name__}", flush=True)
    h = _create(name, dtype)
    ref = C.canonical(name, dtype)
    for sigma in (-1, 1, 128, 16384):
        try:
            want = OF.to_sell(ref, sigma)
        except OF.OracleError as err:
            assert err.status == OF.NOT_APPLICABLE
            with pytest.raises(S.SpmvError) as got:
                S.spmv_convert(h, S.SPMV_FMT_SELL, sigma)
            assert got.value.status == "NOT_APPLICABLE"
            continue
        S.spmv_convert(h, S.SPMV_FMT_SELL, sigma)
        g = S.arrays_to_host(h, S.SPMV_FMT_SELL)
        assert (g["sigma"], g["n_slices"], g["slots"]) == \
            (want["sigma"], want["n_slices"], int(want["slice_ptr"][-1])), sigma
        assert np.array_equal(g["slice_ptr"], want["slice_ptr"]), sigma
        assert np.array_equal(g["perm"], want["perm"]), sigma
        assert _same_bits(g["col"], want["col"]) and _same_bits(g["val"], want["val"]), sigma
    for b in (-1, 2, 4, 8):
        try:
            want = OF.to_bell(ref, b)
        except OF.OracleError as err:
            assert err.status == OF.NOT_APPLICABLE
            with pytest.raises(S.SpmvError) as got:
                S.spmv_convert(h, S.SPMV_FMT_BELL, b)
            assert got.value.status == "NOT_APPLICABLE"
            continue
        S.spmv_convert(h, S.SPMV_FMT_BELL, b)
        g = S.arrays_to_host(h, S.SPMV_FMT_BELL)
        assert (g["b"], g["K"], g["pitch"]) == (want["b"], want["K"], want["pitch"]), b
        assert _same_bits(g["bcol"], want["bcol"]) and _same_bits(g["bval"], want["bval"]), b
    for bad in ((S.SPMV_FMT_SELL, 0), (S.SPMV_FMT_SELL, 100), (S.SPMV_FMT_BELL, 3), (S.SPMV_FMT_BELL, 16)):
        with pytest.raises(S.SpmvError) as got:
            S.spmv_convert(h, *bad)
        assert got.value.status == "INVALID_ARG"


def test_input_errors():
    def status(*args, **kw):
        with pytest.raises(S.SpmvError) as e:
            S.spmv_create(*args, **kw)
        return e.value.status

    f = np.float32
    assert status(3, 3, np.array([0, 3]), np.array([0, 0]), np.ones(2, f)) == "OUT_OF_BOUNDS"
    assert status(3, 3, np.array([0, 1]), np.array([-1, 0]), np.ones(2, f)) == "OUT_OF_BOUNDS"
    assert status(3, 3, np.array([2, 0, 2]), np.array([1, 0, 1]), np.ones(3, f)) == "DUPLICATE"
    assert status(3, 3, np.array([0, 1, 1]), np.array([0, 2, 2]), np.ones(3, f)) == "DUPLICATE"
    assert status(-1, 3, np.zeros(0), np.zeros(0), np.zeros(0, f)) == "INVALID_ARG"
    assert status(0, 0, np.array([0]), np.array([0]), np.ones(1, f)) == "OUT_OF_BOUNDS"
    with pytest.raises(ValueError):
        S.spmv_create(3, 3, np.array([0]), np.array([0]), np.ones(1, np.int64))


def test_run_errors_and_failed_convert_keeps_formats():
    m = C.matrix("powerlaw")
    r, c, v = C.shuffled_input("powerlaw", np.float32)
    h = S.spmv_create(m.n_rows, m.n_cols, r, c, v)
    x = torch.ones(m.n_cols, device="cuda")
    y = torch.zeros(m.n_rows, device="cuda")
    with pytest.raises(S.SpmvError) as e:
        S.spmv_run(h, S.SPMV_FMT_ELL, 1.0, x, 0.0, y)
    assert e.value.status == "NOT_CONVERTED"
    with pytest.raises(S.SpmvError) as e:
        S.spmv_run(h, S.SPMV_FMT_CSR, 1.0, y, 0.0, y)
    assert e.value.status == "INVALID_ARG"
    with pytest.raises(S.SpmvError) as e:
        S.spmv_run(h, 9, 1.0, x, 0.0, y)
    assert e.value.status == "INVALID_ARG"
    with pytest.raises(S.SpmvError) as e:
        S.spmv_convert(h, S.SPMV_FMT_ELL)
    assert e.value.status == "NOT_APPLICABLE"
    S.spmv_run(h, S.SPMV_FMT_CSR, 1.0, x, 0.0, y)
    torch.cuda.synchronize()
    lengths = np.diff(C.canonical("powerlaw", np.float32)["row_ptr"])
    assert np.all(np.isfinite(y.cpu().numpy())) and lengths.max() > 1000


def test_overlapping_x_and_y_are_refused_by_every_runner():
    """x and y that share bytes (here one element of one buffer) are refused before
    any launch by the run, timing, tuning and energy entry points alike."""
    m = C.matrix("lap64")
    h = S.spmv_create(m.n_rows, m.n_cols, *C.shuffled_input("lap64", np.float32))
    buf = torch.zeros(m.n_rows + m.n_cols - 1, device="cuda")
    x, y = buf[:m.n_cols], buf[m.n_cols - 1:]
    calls = [lambda: S.spmv_run(h, S.SPMV_FMT_CSR, 1.0, x, 0.0, y),
             lambda: S.spmv_time(h, S.SPMV_FMT_CSR, x, y, reps=1, flush=False),
             lambda: S.spmv_tune(h, S.SPMV_FMT_CSR, x, y, reps=1, flush=False),
             lambda: S.spmv_energy(h, S.SPMV_FMT_CSR, x, y, seconds=0.01)]
    for call in calls:
        with pytest.raises(S.SpmvError) as e:
            call()
        assert e.value.status == "INVALID_ARG" and "overlap" in str(e.value)
    torch.cuda.synchronize()
    assert float(buf.abs().sum()) == 0.0  # nothing ran


def test_full_size_power_law_ingest_from_shuffled_input():
    """2M x 2M power-law matrix (about 32M entries) through the radix-sort path."""
    m = synth.config3_matrix()
    r, c, perm = synth.shuffled(m, 9)
    v = m.values(np.float32)[perm]
    print(f"[ingest full] power-law n={m.n_rows} nnz={m.nnz}", flush=True)
    h = S.spmv_create(m.n_rows, m.n_cols, r, c, v)
    ref = OF.canonicalize(m.n_rows, m.n_cols, r, c, v)
    _check_canonical(h, ref)
    hy = OF.to_hyb(ref)
    S.spmv_convert(h, S.SPMV_FMT_HYB)
    g = S.arrays_to_host(h, S.SPMV_FMT_HYB)
    assert (g["K"], g["nnz_tail"]) == (hy["K"], hy["tail_row"].size)
    for key in ("ell_col", "ell_val", "tail_row", "tail_col", "tail_val"):
        assert _same_bits(g[key], hy[key]), key
