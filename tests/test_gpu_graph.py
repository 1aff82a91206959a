"""spmv_run captured in a HIP graph: once a variant's layout is built, a run is kernel
launches only, so a graph replays it. Every format's variants are captured on one case
and each replay, with eager work and synchronisations between replays, is checked
against the oracle (and, for the variants with a fixed order of additions, bit for bit
against the eager run)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import _cases as C  # noqa: E402
from oracle import formats as OF  # noqa: E402
from oracle import spmv as OS  # noqa: E402

import paper_2302_05662_amd as S  # noqa: E402


def _atomic_order(d):
    """Variants whose FP64 additions land in no fixed order (LDS atomics)."""
    return d["kernel"] == "coo_sorted" or (d["kernel"] == "hyb" and d["pipelined"] == 1)


@pytest.mark.parametrize("name", ["random", "banded"])
def test_runs_replay_from_a_graph(name):
    dtype = np.float32
    print(f"[graph] {name}", flush=True)
    m = C.matrix(name)
    h = S.spmv_create(m.n_rows, m.n_cols, *C.shuffled_input(name, dtype))
    ref = C.canonical(name, dtype)
    fmts = [S.SPMV_FMT_CSR, S.SPMV_FMT_COO]
    for fmt, build in ((S.SPMV_FMT_ELL, OF.to_ell), (S.SPMV_FMT_HYB, OF.to_hyb),
                       (S.SPMV_FMT_SELL, OF.to_sell), (S.SPMV_FMT_BELL, OF.to_bell)):
        try:
            build(ref)
        except OF.OracleError:
            continue
        S.spmv_convert(h, fmt)
        fmts.append(fmt)
    x, y0 = C.vectors(name, dtype)
    xd = torch.from_numpy(x).cuda()
    a, b = C.ALPHA_BETA[1]
    y_ref, den = C.reference(name, dtype, a, b)
    side = torch.cuda.Stream()
    checked = 0
    for fmt in fmts:
        for var in range(S.spmv_variant_count(fmt, h.dtype_code)):
            try:
                S.spmv_set_variant(h, fmt, var)  # builds the variant's layout outside the capture
            except S.SpmvError as e:
                assert e.status == "NOT_APPLICABLE"
                continue
            d = S.spmv_variant_describe(fmt, h.dtype_code, var)
            y_eager = torch.from_numpy(y0.copy()).cuda()
            S.spmv_run(h, fmt, a, xd, b, y_eager)
            y = torch.from_numpy(y0.copy()).cuda()
            y_init = y.clone()
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.stream(side):
                with torch.cuda.graph(g, stream=side):
                    S.spmv_run(h, fmt, a, xd, b, y)
            torch.cuda.synchronize()
            for rep in range(3):
                y.copy_(y_init)
                junk = torch.randn(1 << 16, device="cuda").sum()  # eager work between replays
                g.replay()
                torch.cuda.synchronize()
                got = y.cpu().numpy()
                err = OS.max_row_error(got, y_ref, den)
                assert err <= C.TOL[dtype], (S.FORMAT_NAMES[fmt], d, rep, err)
                if not _atomic_order(d):
                    assert got.tobytes() == y_eager.cpu().numpy().tobytes(), (S.FORMAT_NAMES[fmt], d, rep)
                del junk
            del g
            checked += 1
    assert checked > 40
