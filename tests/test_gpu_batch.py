"""Batched persistent SpMV in a HIP graph: parity with the oracle and with single launches."""
import numpy as np
import pytest

import synth
from oracle import formats as OF
from oracle import spmv as OS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2302_05662_amd as S  # noqa: E402


def _matrices():
    ms = []
    for i, spec in enumerate(synth.config4_specs(range(4000, 4030))):
        spec = dict(spec)
        spec["n"] = max(64, spec["n"] // 20)  # same families, smaller sizes
        if spec["family"] == "powerlaw":
            spec["cap"] = min(spec["cap"], spec["n"])
        ms.append(synth.config4_matrix(spec))
    ms.append(synth.from_coords("empty_rows", 300, 200, [5, 5, 299], [0, 7, 199], 9))
    ms.append(synth.from_coords("no_entries", 50, 50, [], [], 10))
    ms.append(synth.random_rect(10, 4000, 9000, 11))  # ten rows of ~900 entries
    ms.append(synth.power_law(3000, 12, cap=3000, value_dist="uniform"))  # rows past 2048
    # columns too wide for a packed row index: sorted blocks keep 16-bit rows beside them
    ms.append(synth.random_rect(5000, (1 << 22) + 9, 20000, 13))
    return ms


def _setup(dtype, seed):
    ms = _matrices()
    hs, xs, ys, refs, y0s = [], [], [], [], []
    rng = np.random.default_rng(seed)
    alphas = rng.uniform(-2, 2, len(ms)).round(2).tolist()
    betas = [0.0 if i % 3 == 0 else 0.5 for i in range(len(ms))]
    for m, a, b in zip(ms, alphas, betas):
        v = m.values(dtype)
        h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, v)
        x = synth.uniform_vector(m.n_cols, dtype, [m.seed, seed])
        y0 = synth.uniform_vector(m.n_rows, dtype, [m.seed, seed + 1])
        c = OF.canonicalize(m.n_rows, m.n_cols, m.row, m.col, v)
        av, bv = dtype(a), dtype(b)
        refs.append((OS.spmv_csr(c["row_ptr"], c["col"], c["val"], x, av, bv, y0),
                     OS.row_denominator(c["row_ptr"], c["col"], c["val"], x, av, bv, y0)))
        hs.append(h)
        xs.append(torch.from_numpy(x).cuda())
        ys.append(torch.from_numpy(y0).cuda())
        y0s.append(y0)
    return ms, hs, xs, ys, refs, y0s, alphas, betas


def _single_variant(dtype_code, lanes, unroll):
    for i in range(S.spmv_variant_count(S.SPMV_FMT_CSR, dtype_code)):
        d = S.spmv_variant_describe(S.SPMV_FMT_CSR, dtype_code, i)
        if d["kernel"] == "csr_vector" and d["vec"] == 4 and d["lanes"] == lanes and d["unroll"] == unroll:
            return i
    raise AssertionError((lanes, unroll))


@pytest.mark.parametrize("dtype,tune", [(np.float32, True), (np.float64, False)])
def test_batch_matches_oracle_and_single_launches(dtype, tune):
    ms, hs, xs, ys, refs, y0s, alphas, betas = _setup(dtype, 21)
    print(f"[batch] {len(ms)} matrices {dtype.__name__} tune={tune}", flush=True)
    b = S.spmv_batch_create(hs, xs, ys, alphas, betas, tune=tune)
    tol = 1e-5 if dtype == np.float32 else 1e-12
    settings = [None, dict(tiling=1, unroll=2, passes_per_tile=1, lanes_divisor=2),
                dict(tiling=0, unroll=1), dict(tiling=0, unroll=2, passes_per_tile=16),
                dict(tiling=2, unroll=1, blocks_per_cu=1), dict(tiling=2, unroll=2, blocks_per_cu=2),
                dict(tiling=2, unroll=4, blocks_per_cu=1)]
    for setting in settings:
        if setting is not None:
            S.spmv_batch_set_config(b, **setting)
        cfg, lanes = S.spmv_batch_get_config(b)
        assert cfg["total_tiles"] > 0 and cfg["grid"] > 0
        for i in range(len(ms)):
            ys[i].copy_(torch.from_numpy(y0s[i]))
        S.spmv_batch_run(b)
        torch.cuda.synchronize()
        for i, m in enumerate(ms):
            got = ys[i].cpu().numpy()
            assert OS.max_row_error(got, *refs[i]) <= tol, (setting, m.name)
            if cfg["tiling"] != 0:
                continue
            # per-matrix tiling: bit-equal to the single CSR vector launch with the
            # same lanes and unroll
            var = _single_variant(hs[i].dtype_code, int(lanes[i]), cfg["unroll"])
            S.spmv_set_variant(hs[i], S.SPMV_FMT_CSR, var)
            ys_single = torch.from_numpy(y0s[i].copy()).cuda()
            S.spmv_run(hs[i], S.SPMV_FMT_CSR, alphas[i], xs[i], betas[i], ys_single)
            assert ys_single.cpu().numpy().tobytes() == got.tobytes(), (setting, m.name)


@pytest.mark.parametrize("tiling", [1, 2])
def test_graph_replays_with_new_vectors_and_eager_work_between(tiling):
    dtype = np.float32
    ms, hs, xs, ys, refs, y0s, alphas, betas = _setup(dtype, 31)
    print(f"[batch replay] tiling {tiling}", flush=True)
    zero_b = [0.0] * len(ms)
    b = S.spmv_batch_create(hs, xs, ys, alphas, zero_b, tune=False)
    if tiling == 2:
        S.spmv_batch_set_config(b, tiling=2, unroll=2, blocks_per_cu=2)
    for rep in range(4):
        new_x = [torch.from_numpy(synth.uniform_vector(m.n_cols, dtype, [m.seed, 100 + rep])).cuda()
                 for m in ms]
        if rep % 2 == 0:
            S.spmv_batch_update(b, xs=new_x)
            junk = torch.randn(1 << 20, device="cuda")
            S.spmv_batch_run(b)
        else:  # new vectors and scales passed to the run itself
            alphas = [round(a * 0.5 - 0.25, 2) for a in alphas]
            junk = torch.randn(1 << 20, device="cuda")
            S.spmv_batch_run(b, alphas=alphas, xs=new_x, betas=zero_b)
        junk.mul_(2).sum().item()  # eager work and a sync between replays
        torch.cuda.synchronize()
        for i, m in enumerate(ms):
            c = OF.canonicalize(m.n_rows, m.n_cols, m.row, m.col, m.values(dtype))
            x = new_x[i].cpu().numpy()
            a = dtype(alphas[i])
            ref = OS.spmv_csr(c["row_ptr"], c["col"], c["val"], x, a, 0.0)
            den = OS.row_denominator(c["row_ptr"], c["col"], c["val"], x, a, 0.0, None)
            assert OS.max_row_error(ys[i].cpu().numpy(), ref, den) <= 1e-5, (rep, m.name)


def test_batch_argument_errors():
    ms, hs, xs, ys, refs, y0s, alphas, betas = _setup(np.float32, 41)
    b = S.spmv_batch_create(hs[:3], xs[:3], ys[:3], tune=False)
    with pytest.raises(S.SpmvError) as e:
        S.spmv_batch_update(b, xs=[ys[0], xs[1], xs[2]], ys=[ys[0], ys[1], ys[2]])
    assert e.value.status == "INVALID_ARG"
    with pytest.raises(S.SpmvError) as e:  # 16 entries per lane only with the sorted tiling
        S.spmv_batch_set_config(b, tiling=0, unroll=4)
    assert e.value.status == "INVALID_ARG"
    S.spmv_batch_run(b)  # still valid with the old pointers
    torch.cuda.synchronize()
    # one launch computes every product: a y may not overlap another matrix's x or y
    pool = torch.zeros(ms[0].n_rows + ms[1].n_rows + 8, dtype=torch.float32, device="cuda")
    y_shared0 = pool[:ms[0].n_rows]
    y_shared1 = pool[ms[0].n_rows - 4:ms[0].n_rows - 4 + ms[1].n_rows]
    with pytest.raises(S.SpmvError) as e:
        S.spmv_batch_run(b, ys=[y_shared0, y_shared1, ys[2]])
    assert e.value.status == "INVALID_ARG"
    xy = torch.zeros(max(ms[0].n_rows, ms[1].n_cols), dtype=torch.float32, device="cuda")
    with pytest.raises(S.SpmvError) as e:  # x of matrix 1 is y of matrix 0
        S.spmv_batch_update(b, xs=[xs[0], xy[:ms[1].n_cols], xs[2]], ys=[xy[:ms[0].n_rows], ys[1], ys[2]])
    assert e.value.status == "INVALID_ARG"
    # shared x vectors are fine (they are only read)
    if ms[0].n_cols == ms[1].n_cols:
        S.spmv_batch_update(b, xs=[xs[0], xs[0], xs[2]])
    S.spmv_batch_run(b)
    torch.cuda.synchronize()
    h64 = S.spmv_create(4, 4, np.arange(4), np.arange(4), np.ones(4))
    with pytest.raises(S.SpmvError) as e:
        S.spmv_batch_create([hs[0], h64], [xs[0], torch.ones(4, dtype=torch.float64, device="cuda")],
                            [ys[0], torch.zeros(4, dtype=torch.float64, device="cuda")], tune=False)
    assert e.value.status == "INVALID_ARG"
