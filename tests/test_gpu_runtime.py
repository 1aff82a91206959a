"""The overhead-aware run-time mode: convert only when the gain over the expected number of
SpMVs pays for the overhead (features, prediction, conversion)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2302_05662_amd as S  # noqa: E402


def _model_favouring(fmt, classes=4):
    """A selector network whose logits are its output biases: class fmt wins."""
    size = {4: 5276, 6: 5406}[classes]
    m = np.zeros(size, np.float32)
    m[size - 12:] = 1.0  # std
    b3 = size - 24 - classes
    m[b3 + fmt] = 5.0
    return m


def _runtime_model(t_ms, convert_ms):
    """Constant per-format times (intercepts only) and constant conversion latencies."""
    p = np.zeros(S.SPMV_RUNTIME_MODEL, np.float32)
    for f in range(6):
        p[f * 13 + 12] = np.log(t_ms[f])
        p[78 + f * 3] = convert_ms[f]
    return p


def test_runtime_mode_converts_only_when_it_pays():
    m = synth.banded(200_000, 4, 51)
    h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float32))
    S.spmv_selector_set_weights(_model_favouring(S.SPMV_FMT_ELL))
    # CSR 1 ms, ELL 0.5 ms per SpMV; converting to ELL is estimated at 40 ms
    S.spmv_runtime_set_model(_runtime_model([1.0, 1.0, 0.5, 1.0, 1.0, 1.0], [0, 0, 40.0, 0, 0, 0]))
    d = S.spmv_select_runtime(h, S.SPMV_FMT_CSR, 10)
    assert d["predicted"] == S.SPMV_FMT_ELL and d["chosen"] == S.SPMV_FMT_CSR and not d["converted"]
    assert d["t_current_ms"] == pytest.approx(1.0, rel=1e-5)
    assert d["t_predicted_ms"] == pytest.approx(0.5, rel=1e-5)
    assert d["convert_ms"] == pytest.approx(40.0, rel=1e-6)
    assert d["gain_ms"] == pytest.approx(5.0, rel=1e-5)
    assert d["overhead_ms"] == pytest.approx(40.0 + d["features_ms"] + d["predict_ms"], rel=1e-6)
    assert d["features_ms"] > 0 and d["predict_ms"] > 0
    with pytest.raises(S.SpmvError) as e:  # ELL was not converted
        S.spmv_get_arrays(h, S.SPMV_FMT_ELL)
    assert e.value.status == "NOT_CONVERTED"
    d = S.spmv_select_runtime(h, S.SPMV_FMT_CSR, 100_000)
    assert d["chosen"] == S.SPMV_FMT_ELL and d["converted"] == 1
    assert d["gain_ms"] == pytest.approx(50_000.0, rel=1e-5)
    S.spmv_get_arrays(h, S.SPMV_FMT_ELL)  # converted by the call
    # once built, the conversion costs nothing: a few iterations already pay
    d = S.spmv_select_runtime(h, S.SPMV_FMT_CSR, 1000)
    assert d["convert_ms"] == 0.0 and d["chosen"] == S.SPMV_FMT_ELL and not d["converted"]
    # no switch when the prediction is the current format, whatever the iterations
    d = S.spmv_select_runtime(h, S.SPMV_FMT_ELL, 10**9)
    assert d["chosen"] == S.SPMV_FMT_ELL and d["gain_ms"] == 0.0
    S.spmv_selector_set_weights(None)
    S.spmv_runtime_set_model(None)


def test_runtime_mode_falls_back_when_conversion_is_refused_and_needs_models():
    pl = synth.power_law(5000, 3, cap=4000)
    h = S.spmv_create(pl.n_rows, pl.n_cols, pl.row, pl.col, pl.values(np.float32))
    with pytest.raises(S.SpmvError) as e:
        S.spmv_select_runtime(h, S.SPMV_FMT_CSR, 10)
    assert e.value.status == "NO_MODEL"
    model = _model_favouring(S.SPMV_FMT_ELL, classes=6)
    model[5406 - 24 - 6 + S.SPMV_FMT_BELL] = 4.0  # then BELL, then HYB
    model[5406 - 24 - 6 + S.SPMV_FMT_HYB] = 3.0
    S.spmv_selector_set_weights(model)
    S.spmv_runtime_set_model(_runtime_model([1.0, 1.0, 0.1, 0.2, 1.0, 0.1], [0, 0, 0, 0, 0, 0]))
    d = S.spmv_select_runtime(h, S.SPMV_FMT_CSR, 1000)
    # ELL is refused by its cap, BELL (one entry per block on these random columns) too
    assert d["predicted"] == S.SPMV_FMT_HYB and d["chosen"] == S.SPMV_FMT_HYB
    with pytest.raises(S.SpmvError) as e:
        S.spmv_runtime_set_model(np.full(S.SPMV_RUNTIME_MODEL, np.nan, np.float32))
    assert e.value.status == "INVALID_ARG"
    with pytest.raises(S.SpmvError) as e:
        S.spmv_select_runtime(h, S.SPMV_FMT_SELL, 10)  # current must be built
    assert e.value.status == "NOT_CONVERTED"
    S.spmv_selector_set_weights(None)
    S.spmv_runtime_set_model(None)
