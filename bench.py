#!/usr/bin/env python3
"""Single-GPU benchmark of the SpMV hot path on 30 seeded single-SpMV matrices.

Workload: the 30 synthetic matrices standing in for the paper's SuiteSparse set
(banded, uniform random, 8x8 block diagonal and 3-D 7-point stencil; 1e5-2e6
rows, 1e6-5e7 stored entries; FP32 values, int32 indices), all resident in HBM.

Setup (untimed): ingest each COO matrix, build ELL and HYB, autotune every
format's kernel variants with cache-flushed timings, and pick the fastest
format per matrix (exhaustive selection). A timed step is one SpMV
y = A x per matrix, in its selected format and variant, back to back on one
stream. ``value`` is useful bytes (the CSR byte count: values + column indices
+ row pointers + x + y) over the step time; the roofline entry uses each
kernel's own format bytes.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "SpMV effective HBM GB/s (% of peak) per format; selector regret vs exhaustive"
FMT_NAMES = ("CSR", "COO", "ELL", "HYB", "SELL", "BELL")
NF = len(FMT_NAMES)
NF4 = 4  # the 4-class selector network's formats: CSR, COO, ELL, HYB


def format_bytes(fmt, n_rows, n_cols, nnz, vb, K=0, pitch=0, tail=0):
    """Algorithmic bytes of one SpMV with beta = 0: matrix arrays once, x once, y written once."""
    xy = n_cols * vb + n_rows * vb
    if fmt == 0:
        return nnz * (vb + 4) + (n_rows + 1) * 4 + xy
    if fmt == 1:
        return nnz * (vb + 8) + xy
    if fmt == 2:
        return pitch * K * (vb + 4) + xy
    return pitch * K * (vb + 4) + tail * (vb + 8) + xy


def kernel_source_hash(kernel_key=None):
    """Hash of the sources a kernel group is compiled from: the streaming and sorted-block
    COO kernels live in panel.hip, every other SpMV kernel in kernels.hip; both include the
    device helpers and the common header."""
    files = ("kernels.hip", "panel.hip", "device.hpp", "common.hpp")
    if kernel_key and kernel_key.startswith(("coo_sorted", "coo_panel", "coo_tiles")):
        files = ("panel.hip", "device.hpp", "common.hpp")
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2302_05662_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_key):
    """HBM bytes per launch from committed rocprofv3 counters, if taken on the current kernels."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash_by_kernel", {}).get(kernel_key) != kernel_source_hash(kernel_key):
        return None
    t = d.get("kernels", {}).get(kernel_key)
    return float(t) if t is not None else None


def kernel_symbols(fmt, info, dtype="float"):
    """Substrings of the HIP kernel names one spmv_run of (fmt, variant) launches, main kernel first."""
    b, l, u, v, pp = info["block"], info["lanes"], info["unroll"], info["vec"], info["pipelined"]
    if info["kernel"] == "csr_scalar":
        return [f"csr_scalar_kernel<{dtype}, {b}, {u}>"]
    if info["kernel"] == "csr_stream":
        return [f"csr_stream_kernel<{dtype}, {b}>"]
    if info["kernel"] == "csr_vector" and pp:
        return [f"csr_pipe_kernel<{dtype}, {b}, {l}, {pp}>"]
    if info["kernel"] == "ell" and info.get("ksplit", 1) > 1:
        return [f"ell_ksplit_kernel<{dtype}, {info['ksplit']}, {l}>"]
    if info["kernel"] == "sell":
        tf = "true" if pp else "false"
        if info.get("ksplit", 1) > 1:
            return [f"sell_ksplit_kernel<{dtype}, {info['ksplit']}, {u}, {tf}, "]
        return [f"sell_kernel<{dtype}, {b}, {u}, {tf}, "]
    if info["kernel"] == "bell":
        # the block edge (second template argument) is the matrix's layout
        return [f"bell_kernel<{dtype}, "]
    if info["kernel"] == "ell" and pp:
        return [f"ell_pipe_kernel<{dtype}, {b}, {l}, {pp}>"]
    if info["kernel"] == "csr_vector":
        name = "csr_vector4_kernel" if v == 4 else "csr_vector_kernel"
        return [f"{name}<{dtype}, {b}, {l}, {u}>"]
    if info["kernel"] == "coo_panel":
        return [f"coo_panel_kernel<{dtype}, {l}>"]
    if info["kernel"] == "coo_sorted" and info.get("ksplit", 1) > 1:
        # column tiles, then the second half's row sums added to y
        return [f"coo_tiles_kernel<{dtype}, {l}, ", f"sorted_tiles_combine<{dtype}>"]
    if info["kernel"] == "coo_sorted":
        # the third template argument (16-bit rows or packed) depends on the matrix
        return [f"coo_sorted_kernel<{dtype}, {l}, "]
    if info["kernel"] == "coo_split":
        return [f"coo_tile_kernel<{dtype}, {b}, {l}, false>", f"coo_tile_kernel<{dtype}, {b}, {l}, true>"]
    if info["kernel"] == "coo":
        return [f"coo_tile_kernel<{dtype}, {b}, {l}, false>", f"coo_fixup<{dtype}, {b * l}, false>"]
    if info["kernel"] == "ell":
        return [f"ell_kernel<{dtype}, {b}, {l}, {u}>"]
    # HYB: the ELL part (grouped, or slot-split over `ksplit` waves), then the tail
    ell = (f"ell_ksplit_kernel<{dtype}, {info['ksplit']}, {l}>" if info.get("ksplit", 1) > 1
           else f"ell_kernel<{dtype}, {b}, {l}, 4>")
    if pp:  # the tail runs through the sorted-block COO kernel
        return [ell, f"coo_sorted_kernel<{dtype}, {u}, "]
    # the tiled tail kernel always runs 256-thread workgroups
    return [ell, f"coo_tile_kernel<{dtype}, 256, {u}, true>", f"coo_fixup<{dtype}, {256 * u}, true>"]


def roofline_symbols(rf):
    """Name substrings of every kernel one launch of the roofline group runs (main first)."""
    return rf.get("kernel_symbols") or [rf["kernel_symbol"]]


def trace_summary(trace_csv, bench_json):
    """Average duration of the roofline kernel over the timed launches, from a rocprofv3 kernel trace.
    A launch of several kernels counts the sum of their average durations."""
    import csv

    with open(bench_json) as fh:
        line = [l for l in fh if l.startswith("{")][-1]
    rf = json.loads(line)["roofline"]
    syms, n = roofline_symbols(rf), rf["launches"]
    with open(trace_csv) as fh:
        all_rows = list(csv.DictReader(fh))
    avg = 0.0
    for sym in syms:
        rows = [r for r in all_rows if sym in r["Kernel_Name"]]
        rows.sort(key=lambda r: int(r["Start_Timestamp"]))
        timed = rows[-n:]
        dur_us = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in timed]
        a = sum(dur_us) / len(dur_us)
        avg += a
        print(f"kernel: {sym}")
        print(f"dispatches in trace: {len(rows)}; timed-region dispatches used: {len(timed)}")
        if len(syms) > 1:
            print(f"rocprofv3 average duration of this kernel over the timed launches: {a:.3f} us")
    print(f"rocprofv3 average duration over the timed launches: {avg:.3f} us")
    print(f"bench HIP-event average per launch: {rf['avg_launch_us']:.3f} us")
    print(f"algorithmic bytes per launch (mean): {rf['bytes_per_launch']:.0f}")
    print(f"achieved from rocprofv3 duration: {rf['bytes_per_launch'] / avg / 1e3:.1f} GB/s "
          f"(bench: {rf['achieved']} GB/s)")


def counter_summary(fetch_csv, write_csv, bench_json, out_json):
    """HBM bytes per launch of the roofline kernel from two rocprofv3 --pmc runs.

    Both runs time the same plan; the counters of the kernel's last ``launches``
    dispatches (the timed steps) are averaged, and each counter is scaled by what
    it reads for the device copy of known size that ends the run.
    """
    import csv

    with open(bench_json) as fh:
        line = [l for l in fh if l.startswith("{")][-1]
    res = json.loads(line)
    rf, mib = res["roofline"], res["copy_calibration_mib"]
    syms, n = roofline_symbols(rf), rf["launches"]
    sym = " + ".join(syms)

    def read(path, counter):
        with open(path) as fh:
            rows = [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        copy = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]][-3:]
        if min(copy, default=0.0) < mib * 1024.0 / 4:
            raise SystemExit(f"{path}: the last device copies are not the {mib} MiB calibration")
        total = 0.0
        for one in syms:  # a launch of several kernels: the sum of their means
            kern = [float(r["Counter_Value"]) for r in rows if one in r["Kernel_Name"]][-n:]
            if len(kern) != n or len(copy) != 3:
                raise SystemExit(f"{path}: {len(kern)} dispatches of {one} (want {n}), "
                                 f"{len(copy)} calibration copies (want 3)")
            total += sum(kern) / n
        return total, sum(copy) / 3

    fetch, fetch_copy = read(fetch_csv, "FETCH_SIZE")
    write, write_copy = read(write_csv, "WRITE_SIZE")
    known_kib = mib * 1024.0
    fs, ws = known_kib / fetch_copy, known_kib / write_copy
    traffic = (fetch * fs + write * ws) * 1024.0
    d = {"note": "HBM bytes per launch over the timed steps: FETCH_SIZE x fetch scale + "
                 "WRITE_SIZE x write scale (KiB x 1024); each kernel's figure holds while the "
                 "sources it is compiled from hash to source_hash_by_kernel",
         "fetch_scale": round(fs, 6), "write_scale": round(ws, 6), "kernels": {},
         "source_hash_by_kernel": {}}
    if os.path.exists(out_json):  # the other kernels' figures stay
        with open(out_json) as fh:
            old = json.load(fh)
        d = {**old, **{k: v for k, v in d.items() if k not in ("kernels", "source_hash_by_kernel")},
             "kernels": dict(old.get("kernels", {})),
             "source_hash_by_kernel": dict(old.get("source_hash_by_kernel", {}))}
        d.pop("kernel_source_hash", None)
    d["kernels"][rf["kernel"]] = round(traffic)
    d["source_hash_by_kernel"][rf["kernel"]] = kernel_source_hash(rf["kernel"])
    with open(out_json, "w") as fh:
        json.dump(d, fh, indent=1)
        fh.write("\n")
    print(f"kernel: {sym} ({rf['kernel']}), {n} timed dispatches")
    print(f"| FETCH_SIZE per launch (raw) | {fetch:.1f} KiB |")
    print(f"| WRITE_SIZE per launch (raw) | {write:.1f} KiB |")
    print(f"| calibration: {mib} MiB device copy (3 runs) | FETCH {fetch_copy:.1f} KiB, "
          f"WRITE {write_copy:.1f} KiB |")
    print(f"| scale factors (known bytes / counter) | fetch {fs:.4f}, write {ws:.4f} |")
    print(f"| HBM traffic per launch (scaled) | {traffic / 1e6:.1f} MB |")
    print(f"| algorithmic bytes per launch | {rf['bytes_per_launch'] / 1e6:.1f} MB |")
    print(f"| traffic / algorithmic | {traffic / rf['bytes_per_launch']:.3f} |")


REQ_COUNTERS = ("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum",
                "TCC_EA0_RDREQ_sum")


def request_summary(csv_path, bench_json, out_json):
    """L2-to-memory read bytes of the roofline kernel by request size (32, 64 and 128 B),
    from one rocprofv3 pass of the four TCC_EA0_RDREQ counters over a --copy-calibration
    run; the calibration copy checks the formula against bytes known in advance."""
    import csv

    with open(bench_json) as fh:
        line = [l for l in fh if l.startswith("{")][-1]
    res = json.loads(line)
    rf, mib = res["roofline"], res["copy_calibration_mib"]
    syms, n = roofline_symbols(rf), rf["launches"]
    sym = " + ".join(syms)
    per = {}
    with open(csv_path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] in REQ_COUNTERS:
                per.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"]})[r["Counter_Name"]] = \
                    float(r["Counter_Value"])
    ids = sorted(per)
    by_sym = [[per[i] for i in ids if one in per[i]["name"]][-n:] for one in syms]
    copy = [per[i] for i in ids if "copyBuffer" in per[i]["name"]][-3:]
    if any(len(k) != n for k in by_sym) or len(copy) != 3:
        raise SystemExit(f"{csv_path}: {[len(k) for k in by_sym]} dispatches of {syms} (want {n}), "
                         f"{len(copy)} copies")
    # one row per launch: the counters of its kernels added
    kern = [{c: sum(k[j][c] for k in by_sym) for c in REQ_COUNTERS} for j in range(n)]

    def bytes_of(d):
        return (32 * d[REQ_COUNTERS[0]] + 64 * d[REQ_COUNTERS[1]] + 128 * d[REQ_COUNTERS[2]])

    def mean(rows, f):
        return sum(f(d) for d in rows) / len(rows)

    kb, cb = mean(kern, bytes_of), mean(copy, bytes_of)
    known = mib * 1024.0 * 1024.0
    unclassified = mean(kern, lambda d: d[REQ_COUNTERS[3]] - d[REQ_COUNTERS[0]] - d[REQ_COUNTERS[1]]
                        - d[REQ_COUNTERS[2]])
    print(f"kernel: {sym} ({rf['kernel']}), {n} timed dispatches")
    print("| quantity | value |")
    print("|---|---|")
    for c in REQ_COUNTERS:
        print(f"| {c} per launch | {mean(kern, lambda d: d[c]):.0f} |")
    print(f"| requests in none of the three sizes, per launch | {unclassified:.0f} |")
    print(f"| read bytes by request size per launch (32/64/128 B) | {kb / 1e6:.1f} MB |")
    print(f"| same formula on the {mib} MiB calibration copy | {cb / known:.4f} of the bytes read |")
    print(f"| algorithmic bytes per launch | {rf['bytes_per_launch'] / 1e6:.1f} MB |")
    print(f"| reads by request size / algorithmic bytes | {kb / rf['bytes_per_launch']:.3f} |")
    d = {}
    if os.path.exists(out_json):
        with open(out_json) as fh:
            d = json.load(fh)
    d.setdefault("read_bytes_by_request_size", {})[rf["kernel"]] = round(kb)
    d["read_bytes_by_request_size_copy_check"] = round(cb / known, 4)
    with open(out_json, "w") as fh:
        json.dump(d, fh, indent=1)
        fh.write("\n")


def pmc_summary(csv_path, bench_json):
    """Per-launch means of every counter in a rocprofv3 --pmc CSV over the roofline kernel's
    timed dispatches, and per stored entry for a one-matrix run (--seeds S)."""
    import csv

    with open(bench_json) as fh:
        line = [l for l in fh if l.startswith("{")][-1]
    res = json.loads(line)
    rf = res["roofline"]
    syms, n = roofline_symbols(rf), rf["launches"]
    sym = " + ".join(syms)
    per = {}
    with open(csv_path) as fh:
        for r in csv.DictReader(fh):
            per.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"]})[r["Counter_Name"]] = \
                float(r["Counter_Value"])
    by_sym = [[per[i] for i in sorted(per) if one in per[i]["name"]][-n:] for one in syms]
    if any(len(k) != n for k in by_sym):
        raise SystemExit(f"{csv_path}: {[len(k) for k in by_sym]} dispatches of {syms} (want {n})")
    names = [c for c in by_sym[0][0] if c != "name"]
    kern = [{c: sum(k[j][c] for k in by_sym) for c in names} for j in range(n)]
    nnz = res["config"]["total_nnz"] if res["config"]["matrices"] == 1 else None
    print(f"kernel: {sym} ({rf['kernel']}), {n} timed dispatches"
          + (f", {nnz} stored entries per launch" if nnz else ""))
    print("| counter | per launch | per entry |")
    print("|---|---|---|")
    for c in sorted(kern[0]):
        m = sum(d[c] for d in kern) / n
        print(f"| {c} | {m:.4g} | {m / nnz:.4g} |" if nnz else f"| {c} | {m:.4g} | |")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(mats, budget_s, threads):
    """The FP64 oracle's CSR SpMV on the host, over the first matrices until the budget is used.

    The oracle's output for each timed matrix is also compared row by row with the y the
    GPU left in the timed steps (y = A x, FP32 bound 1e-5); a miss ends the run with an error.
    """
    from oracle import spmv as OS

    names, checked, worst = [], 0, 0.0
    for m in mats:
        if sum(t for _, t in names) * 5 >= budget_s:
            break
        rp = np.zeros(m["n_rows"] + 1, np.int64)
        np.cumsum(np.bincount(m["row"], minlength=m["n_rows"]), out=rp[1:])
        val = m["val"].astype(np.float64)
        x = m["x"].astype(np.float64)
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            y_ref = OS.spmv_csr(rp, m["col"], val, x, 1.0, 0.0, None, n_threads=threads)
            ts.append(time.perf_counter() - t0)
        names.append((m["name"], float(np.median(ts))))
        den = OS.spmv_csr(rp, m["col"], np.abs(val), np.abs(x), 1.0, 0.0, None, n_threads=threads)
        err = OS.max_row_error(m["y_gpu"], y_ref, den)
        worst = max(worst, err)
        checked += 1
        if not err <= 1e-5:
            raise SystemExit(f"{m['name']}: GPU y differs from the oracle (row error {err:.3g} > 1e-5)")
    batch_rows, batch_worst = 0, 0.0
    for c in BATCH_CHECKS:  # the batched launch's sampled rows
        k = len(c["cols"])
        rp = np.zeros(k + 1, np.int64)
        np.cumsum([len(a) for a in c["cols"]], out=rp[1:])
        col = np.concatenate(c["cols"]).astype(np.int64)
        val = np.concatenate(c["vals"]).astype(np.float64)
        x = c["x"].astype(np.float64)
        y_ref, den = OS.spmv_rows(np.arange(k), rp, col, val, x, 1.0, 0.0, None)
        err = OS.max_row_error(c["y"], y_ref, den)
        batch_worst = max(batch_worst, err)
        batch_rows += k
        if not err <= 1e-5:
            raise SystemExit(f"batched launch: GPU y differs from the oracle (row error {err:.3g})")
    if not names:
        return None
    tot_t = sum(t for _, t in names)
    tot_b = sum(mm["useful_bytes"] for mm in mats[:len(names)])
    one_b, one_t = 0.0, 0.0
    for m in mats[:2]:  # one thread on the first two matrices, for scale
        rp = np.zeros(m["n_rows"] + 1, np.int64)
        np.cumsum(np.bincount(m["row"], minlength=m["n_rows"]), out=rp[1:])
        val, x = m["val"].astype(np.float64), m["x"].astype(np.float64)
        t0 = time.perf_counter()
        OS.spmv_csr(rp, m["col"], val, x, 1.0, 0.0, None, n_threads=1)
        one_t += time.perf_counter() - t0
        one_b += m["useful_bytes"]
    return {"value": round(tot_b / tot_t / 1e9, 3), "unit": "GB/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "gflops": round(2 * sum(mm["nnz"] for mm in mats[:len(names)]) / tot_t / 1e9, 3),
            "single_thread_value": round(one_b / one_t / 1e9, 3),
            "checked_matrices": checked, "max_row_error_vs_gpu": float(f"{worst:.3g}"),
            "checked_batched_rows": batch_rows,
            "max_row_error_batched": float(f"{batch_worst:.3g}"),
            "sample": f"first {len(names)} of {len(mats)} matrices, FP64 CSR loop (FP32 inputs "
                      f"promoted) on {threads} threads (the CPU share of this process), median "
                      f"of 5 runs each, same useful-byte formula; single_thread_value: first 2 "
                      f"matrices, one run each, 1 thread"}


def total_nnz_of(mats):
    return float(sum(e["nnz"] for e in mats))


MODEL_PATH = os.path.join(ROOT, "paper_2302_05662_amd", "selector_model.npy")
MODEL6_PATH = os.path.join(ROOT, "paper_2302_05662_amd", "selector_model6.npy")


def selector_section(S, torch, mats, step, steps):
    """Regret of the learned, rule and always-CSR choices against exhaustive timing.

    The 4-class network (CSR, COO, ELL, HYB) is scored against the best of those four
    formats; the 6-class network, when present, against the best of all six.
    """
    def regret(key, best):
        r = [e["times"][e[key]] / e["times"][e[best]] - 1.0 for e in mats]
        return {"mean": round(float(np.mean(r)), 4), "p95": round(float(np.percentile(r, 95)), 4),
                "max": round(float(np.max(r)), 4),
                "within_5pct": round(float(np.mean(np.array(r) <= 0.05)), 4),
                "sum_time_ratio": round(sum(e["times"][e[key]] for e in mats)
                                        / sum(e["times"][e[best]] for e in mats) - 1.0, 4)}
    for e in mats:
        e["csr"] = 0
        e["rule"] = S.spmv_select_format(e["h"], S.SPMV_SELECT_RULE)[0]
    out = {"labels": "exhaustive autotuned cold medians (setup)", "always_csr": regret("csr", "fmt4"),
           "rule": regret("rule", "fmt4"), "model": None, "model6": None}

    def timed(key):
        for _ in range(2):
            step(key=key)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            step(key=key)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / steps

    for path, key, best, name in ((MODEL_PATH, "mlp", "fmt4", "model"),
                                  (MODEL6_PATH, "mlp6", "fmt", "model6")):
        if not os.path.exists(path):
            continue
        S.spmv_selector_set_weights(np.load(path))
        lat = []
        for e in mats:
            t = time.perf_counter()
            e[key] = S.spmv_select_format(e["h"], S.SPMV_SELECT_MODEL)[0]
            lat.append(time.perf_counter() - t)
        model = regret(key, best)
        model["classes"] = S.spmv_selector_classes()
        model["accuracy"] = round(float(np.mean([e[key] == e[best] for e in mats])), 4)
        model["select_ms_mean"] = round(1e3 * float(np.mean(lat)), 3)
        ms_best, ms_mlp = timed(best), timed(key)
        model[f"step_ms_exhaustive_plan"] = round(ms_best, 4)
        model["step_ms_model_plan"] = round(ms_mlp, 4)
        model["step_regret"] = round(ms_mlp / ms_best - 1.0, 4)
        out[name] = model
    S.spmv_selector_set_weights(None)
    return out


def ingest_unsorted(S, torch, synth, tune=True):
    """The 2M-row power-law matrix: ingest from shuffled COO (the radix-sort path), then every
    applicable format tuned with cache-flushed timing."""
    m = synth.config3_matrix()
    r, c, perm = synth.shuffled(m, 17)
    v = m.values(np.float32)[perm]
    coo = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (r, c, v)]
    torch.cuda.synchronize()
    t = time.perf_counter()
    h = S.spmv_create(m.n_rows, m.n_cols, *coo)
    dt = time.perf_counter() - t
    del coo
    rates = {"ingest_unsorted_nnz_per_s": round(m.nnz / dt, 0),
             "ingest_unsorted_matrix": f"{m.name}, {m.nnz} entries, shuffled"}
    if not tune:
        S.spmv_destroy(h)
        return rates, None
    x = torch.from_numpy(m.x(np.float32)).cuda()
    y = torch.zeros(m.n_rows, dtype=torch.float32, device="cuda")
    useful = format_bytes(0, m.n_rows, m.n_cols, m.nnz, 4)
    per = {}
    for fmt in range(NF):
        try:
            S.spmv_convert(h, fmt)
        except S.SpmvError as e:
            if e.status != "NOT_APPLICABLE":
                raise
            per[FMT_NAMES[fmt]] = None
            continue
        var, ms = S.spmv_tune(h, fmt, x, y, reps=5, flush=True)
        info = S.spmv_variant_describe(fmt, S.SPMV_F32, var)
        per[FMT_NAMES[fmt]] = {"us": round(ms * 1e3, 1), "useful_gbps": round(useful / ms / 1e6, 1),
                               "gflops": round(2 * m.nnz / ms / 1e6, 1), "kernel": info["kernel"],
                               "lanes": info["lanes"], "block": info["block"]}
    # CSR scalar, CSR stream and CSR vector at each lane count: the best variant of each
    csr_by_lanes = {}
    for var in range(S.spmv_variant_count(S.SPMV_FMT_CSR, S.SPMV_F32)):
        info = S.spmv_variant_describe(S.SPMV_FMT_CSR, S.SPMV_F32, var)
        key = {"csr_scalar": "scalar", "csr_stream": "stream"}.get(
            info["kernel"], f"vector_lanes_{info['lanes']}")
        t = float(np.median(S.spmv_time(h, S.SPMV_FMT_CSR, x, y, variant=var, warmup=1, reps=3,
                                        flush=True))) * 1e3
        csr_by_lanes[key] = min(csr_by_lanes.get(key, float("inf")), round(t, 1))
    S.spmv_destroy(h)
    ok = {k: v for k, v in per.items() if v is not None}
    best = min(ok, key=lambda k: ok[k]["us"])
    power_law = {"matrix": f"{m.name}: {m.n_rows} rows, {m.nnz} entries, row lengths Zipf-like "
                           f"(mean 16, cap 50000), FP32", "per_format_tuned_cold": per,
                 "csr_us_by_kernel": csr_by_lanes,
                 "best": best, "best_frac_of_peak": round(ok[best]["useful_gbps"] / HBM_PEAK_GBPS, 4)}
    return rates, power_law


def fp64_section(S, torch, synth, seeds):
    """The single-SpMV set in FP64: every applicable format tuned (cache-flushed), best per matrix."""
    tot_useful, tot_best, tot_nnz, chosen = 0.0, 0.0, 0, {n: 0 for n in FMT_NAMES}
    per_fmt = {n: [0.0, 0.0] for n in FMT_NAMES}
    for s in seeds:
        m = synth.config2_matrix(s)
        h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float64))
        x = torch.from_numpy(m.x(np.float64)).cuda()
        y = torch.zeros(m.n_rows, dtype=torch.float64, device="cuda")
        useful = format_bytes(0, m.n_rows, m.n_cols, m.nnz, 8)
        best, best_fmt = float("inf"), None
        for fmt in range(NF):
            try:
                S.spmv_convert(h, fmt)
            except S.SpmvError as e:
                if e.status != "NOT_APPLICABLE":
                    raise
                continue
            _, ms = S.spmv_tune(h, fmt, x, y, reps=3, flush=True)
            per_fmt[FMT_NAMES[fmt]][0] += useful
            per_fmt[FMT_NAMES[fmt]][1] += ms
            if ms < best:
                best, best_fmt = ms, FMT_NAMES[fmt]
        chosen[best_fmt] += 1
        tot_useful += useful
        tot_best += best
        tot_nnz += m.nnz
        S.spmv_destroy(h)
        del x, y
    return {"matrices": len(seeds), "dtype": "f64",
            "best_plan_useful_gbps": round(tot_useful / tot_best / 1e6, 1),
            "best_plan_frac_of_peak": round(tot_useful / tot_best / 1e6 / HBM_PEAK_GBPS, 4),
            "best_plan_gflops": round(2 * tot_nnz / tot_best / 1e6, 1),
            "per_format_useful_gbps": {k: round(v[0] / v[1] / 1e6, 1) for k, v in per_fmt.items() if v[1] > 0},
            "chosen": chosen,
            "timing": "sum over matrices of the best format's tuned cold median (not a timed step)"}


ENERGY_EVAL_PATH = os.path.join(ROOT, "paper_2302_05662_amd", "selector_eval_energy.json")


def energy_section(S, mats, names=("s2000_", "s2001_", "s2003_")):
    """Board energy and average power of every tuned format on a banded, a random-column and
    a stencil matrix (one counter sweep each, the formats in turn), beside the energy head's
    held-out result when it has been trained."""
    try:
        idle = S.spmv_idle_power(0.2)
    except S.SpmvError as err:  # no energy counter on this device
        return {"unavailable": str(err)}
    out = {"idle_watts": round(idle, 1), "matrices": {}, "unit": "uJ per SpMV, W, MFLOPS/W",
           "method": "spmv_energy_formats: each format's tuned variant back to back for one "
                     "board energy counter period (about 1 s), board power including idle"}
    for e in mats:
        if not e["name"].startswith(names):
            continue
        fmts = [f for f in range(NF) if np.isfinite(e["times"][f])]
        try:
            res = S.spmv_energy_formats(e["h"], fmts, e["xd"], e["y"], seconds=0.2)
        except S.SpmvError as err:  # a counter that stops advancing: reported, not fatal
            out["matrices"][e["name"]] = {"unavailable": str(err)}
            continue
        out["matrices"][e["name"]] = {
            FMT_NAMES[f]: {"uJ": round(r["joules_per_run"] * 1e6, 2), "W": round(r["watts"], 1),
                           "MFLOPS_per_W": round(r["mflops_per_watt"], 1),
                           "us": round(r["ms_per_run"] * 1e3, 2)} for f, r in zip(fmts, res)}
        best_e = min(fmts, key=lambda f: res[fmts.index(f)]["joules_per_run"])
        best_w = min(fmts, key=lambda f: res[fmts.index(f)]["watts"])
        out["matrices"][e["name"]]["least_energy"] = FMT_NAMES[best_e]
        out["matrices"][e["name"]]["least_power"] = FMT_NAMES[best_w]
        out["matrices"][e["name"]]["fastest"] = FMT_NAMES[e["fmt"]]
    if os.path.exists(ENERGY_EVAL_PATH):
        with open(ENERGY_EVAL_PATH) as fh:
            ev = json.load(fh)
        out["energy_head_heldout"] = {k: ev["energy"][k] for k in ("model_energy", "always_csr",
                                                                   "latency_labels")}
        out["power_head_heldout"] = ev["power"]["model_power"]
    return out


BATCH_CHECKS = []  # sampled rows of the batched outputs, checked in the CPU leg


def batched_section(S, torch, synth, count):
    """256 uneven SpMVs: one persistent graph launch vs 256 eager launches vs a graph of them."""
    specs = synth.config4_specs()[:count]
    hs, xs, ys, useful, nnz = [], [], [], 0, 0
    t0 = time.perf_counter()
    for sp in specs:
        m = synth.config4_matrix(sp)
        h = S.spmv_create(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float32))
        hs.append(h)
        xs.append(torch.from_numpy(m.x(np.float32)).cuda())
        ys.append(torch.zeros(m.n_rows, dtype=torch.float32, device="cuda"))
        useful += format_bytes(0, m.n_rows, m.n_cols, m.nnz, 4)
        nnz += m.nnz
    gen_s = time.perf_counter() - t0
    print(f"[batched] {len(hs)} matrices, {nnz} entries, generated in {gen_s:.1f}s",
          file=sys.stderr, flush=True)
    fmts = []
    for h, x, y in zip(hs, xs, ys):  # best single variant per matrix (CSR or COO), warm timing
        _, t_csr = S.spmv_tune(h, S.SPMV_FMT_CSR, x, y, reps=3, flush=False)
        _, t_coo = S.spmv_tune(h, S.SPMV_FMT_COO, x, y, reps=3, flush=False)
        fmts.append(S.SPMV_FMT_CSR if t_csr <= t_coo else S.SPMV_FMT_COO)
    b = S.spmv_batch_create(hs, xs, ys, tune=True)
    cfg, _ = S.spmv_batch_get_config(b)
    stream = torch.cuda.current_stream()

    def time_it(fn, reps=10):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ts = []
        for _ in range(reps):
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    def eager():
        for h, x, y, f in zip(hs, xs, ys, fmts):
            S.spmv_run(h, f, 1.0, x, 0.0, y)

    persistent = time_it(lambda: S.spmv_batch_run(b))
    # rows of every matrix as the persistent launch left them (first, last, longest and five
    # seeded ones), with their entries, for the CPU leg's check against the oracle
    for y in ys:
        y.fill_(float("nan"))
    S.spmv_batch_run(b)
    torch.cuda.synchronize()
    rng = np.random.default_rng(4999)
    for sp, x, y in zip(specs, xs, ys):
        m = synth.config4_matrix(sp)
        rp = np.zeros(m.n_rows + 1, np.int64)
        np.cumsum(np.bincount(m.row, minlength=m.n_rows), out=rp[1:])
        rows = np.unique(np.concatenate([[0, m.n_rows - 1, int(np.argmax(np.diff(rp)))],
                                         rng.integers(0, m.n_rows, 5)]))
        v = m.values(np.float32)
        BATCH_CHECKS.append({"cols": [m.col[rp[r]:rp[r + 1]] for r in rows],
                             "vals": [v[rp[r]:rp[r + 1]] for r in rows],
                             "x": m.x(np.float32), "y": y.cpu().numpy()[rows]})
    eager_ms = time_it(eager)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        eager()
    graph_ms = time_it(g.replay)
    return {"matrices": len(hs), "total_nnz": int(nnz), "useful_bytes": int(useful),
            "persistent_graph_ms": round(persistent, 4), "eager_launches_ms": round(eager_ms, 4),
            "graph_of_launches_ms": round(graph_ms, 4),
            "persistent_useful_gbps": round(useful / persistent / 1e6, 1),
            "eager_useful_gbps": round(useful / eager_ms / 1e6, 1),
            "config": {k: cfg[k] for k in ("tiling", "unroll", "passes_per_tile", "blocks_per_cu",
                                           "lanes_divisor", "grid", "total_tiles")},
            "eager_formats": {"CSR": fmts.count(S.SPMV_FMT_CSR), "COO": fmts.count(S.SPMV_FMT_COO)},
            "timing": "median of 10 warm runs, HIP events on the launch stream; eager launches use "
                      "each matrix's fastest tuned CSR or COO variant"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--matrices", type=int, default=30, help="first N of the 30 seeds")
    ap.add_argument("--seeds", help="comma-separated seeds of the 30 (e.g. 2001,2009) instead of "
                    "the first N: a per-matrix measurement for profiles")
    ap.add_argument("--tune-reps", type=int, default=5)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle CPU work")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 256-matrix batched section")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 pass over the same matrices")
    ap.add_argument("--kernels-only", action="store_true",
                    help="profile runs: only setup, the cold plan and the timed steps (no selector, "
                         "power-law, FP64, batched or CPU sections)")
    ap.add_argument("--batched-matrices", type=int, default=256)
    ap.add_argument("--format", choices=("CSR", "COO", "ELL", "HYB", "SELL", "BELL"),
                    help="time this format (its tuned variant) on every matrix where it applies, "
                         "instead of the fastest format: a per-kernel measurement for profiles")
    ap.add_argument("--plan", help="JSON of a previous run: reuse its format/variant per matrix "
                    "instead of tuning")
    ap.add_argument("--roofline-kernel", metavar="KEY",
                    help="report this kernel group (a previous run's roofline.kernel) as the "
                         "roofline kernel, for counter runs under a profiler")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the timed steps, copy MIB MiB three times (counter calibration)")
    ap.add_argument("--trace-summary", nargs=2, metavar=("KERNEL_TRACE_CSV", "BENCH_JSON"),
                    help="summarise a rocprofv3 kernel trace of a previous run and exit")
    ap.add_argument("--request-summary", nargs=3, metavar=("RDREQ_CSV", "BENCH_JSON", "OUT_JSON"),
                    help="L2 read bytes of the roofline kernel by request size from one rocprofv3 "
                         "pass of the TCC_EA0_RDREQ counters; merges into OUT_JSON and exits")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("PMC_CSV", "BENCH_JSON"),
                    help="per-launch means of the counters of a rocprofv3 --pmc run for the "
                         "roofline kernel's timed dispatches, and exit")
    ap.add_argument("--counter-summary", nargs=4,
                    metavar=("FETCH_CSV", "WRITE_CSV", "BENCH_JSON", "OUT_JSON"),
                    help="HBM traffic of the roofline kernel from rocprofv3 FETCH_SIZE and "
                         "WRITE_SIZE runs of a --copy-calibration bench; writes OUT_JSON and exits")
    args = ap.parse_args()
    if args.kernels_only:
        args.no_batched = args.no_fp64 = args.no_cpu = True
    if args.trace_summary:
        trace_summary(*args.trace_summary)
        return
    if args.counter_summary:
        counter_summary(*args.counter_summary)
        return
    if args.request_summary:
        request_summary(*args.request_summary)
        return
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the library "
              "runs each SpMV on one GPU, and sharding rows across GPUs is designed, not "
              "implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2302_05662_amd as S
    import synth

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    seeds = list(synth.matrices.CFG2_SEEDS)[: args.matrices]
    if args.seeds:
        seeds = [int(t) for t in args.seeds.split(",")]
        bad = [t for t in seeds if t not in synth.matrices.CFG2_SEEDS]
        if bad:
            sys.exit(f"--seeds: {bad} are not among the 30 single-SpMV seeds")

    plan = None
    if args.plan:
        with open(args.plan) as fh:
            line = [l for l in fh if l.startswith("{")][-1]
        plan = {p["name"]: p for p in json.loads(line)["plan"]}

    mats = []
    t_setup = time.perf_counter()
    for s in seeds:
        m = synth.config2_matrix(s)
        v = m.values(np.float32)
        x = m.x(np.float32)
        coo = [torch.from_numpy(a).cuda() for a in (m.row, m.col, v)]  # COO resident in HBM
        torch.cuda.synchronize()
        t = time.perf_counter()
        h = S.spmv_create(m.n_rows, m.n_cols, *coo)  # synchronises
        t_ingest = time.perf_counter() - t
        del coo
        t = time.perf_counter()
        feats = S.spmv_features(h)
        t_feat = time.perf_counter() - t
        xd = torch.from_numpy(x).cuda()
        yd = torch.zeros(m.n_rows, dtype=torch.float32, device="cuda")
        entry = {"name": m.name, "family": m.family, "n_rows": m.n_rows, "n_cols": m.n_cols,
                 "nnz": m.nnz, "h": h, "xd": xd, "y": yd, "times": {}, "variant": {}, "bytes": {},
                 "default_ms": {}, "feats": feats, "t_ingest": t_ingest, "t_feat": t_feat,
                 "t_convert": {}}
        xy = 4 * (m.n_rows + m.n_cols)
        for fmt in range(NF):
            t = time.perf_counter()
            try:
                S.spmv_convert(h, fmt)
            except S.SpmvError as e:
                if e.status != "NOT_APPLICABLE":
                    raise
                entry["times"][fmt] = float("inf")
                continue
            entry["t_convert"][fmt] = time.perf_counter() - t
            if plan is not None:
                pm = plan[m.name]
                entry["times"][fmt] = pm["times"][fmt] if pm["times"][fmt] is not None else float("inf")
                entry["variant"][fmt] = pm["variants"][fmt]
                S.spmv_set_variant(h, fmt, pm["variants"][fmt])
            else:
                # the default variant (the library's choice from the row lengths) before tuning:
                # the tuned-over-default gain is the compile-time mode's result here
                dv = S.spmv_get_variant(h, fmt)
                entry["default_ms"][fmt] = float(np.median(S.spmv_time(
                    h, fmt, xd, yd, variant=dv, warmup=1, reps=args.tune_reps, flush=True)))
                var, ms = S.spmv_tune(h, fmt, xd, yd, reps=args.tune_reps, flush=True)
                entry["times"][fmt] = ms
                entry["variant"][fmt] = var
            # bytes as stored: the layout the chosen variant streams, x once, y once
            entry["bytes"][fmt] = S.spmv_stored_bytes(h, fmt) + xy
        if plan is None:
            # the tiled segmented COO kernel on its own (the sorted-block COO kernels read a
            # reordered copy): its best variant's cold median, priced at nnz * 12 + x + y
            tiled = [var for var in range(S.spmv_variant_count(S.SPMV_FMT_COO, S.SPMV_F32))
                     if S.spmv_variant_describe(S.SPMV_FMT_COO, S.SPMV_F32, var)["kernel"] == "coo"]
            entry["coo_tiled_ms"] = min(float(np.median(S.spmv_time(
                h, S.SPMV_FMT_COO, xd, yd, variant=var, warmup=1, reps=args.tune_reps, flush=True)))
                for var in tiled)
            entry["coo_tiled_bytes"] = m.nnz * 12 + xy
            S.spmv_set_variant(h, S.SPMV_FMT_COO, entry["variant"][S.SPMV_FMT_COO])
        for fmt in range(NF):
            entry["variant"].setdefault(fmt, -1)
        entry["fmt"] = int(np.argmin([entry["times"][f] for f in range(NF)]))
        if args.format and np.isfinite(entry["times"][FMT_NAMES.index(args.format)]):
            entry["fmt"] = FMT_NAMES.index(args.format)
        entry["fmt4"] = int(np.argmin([entry["times"][f] for f in range(NF4)]))
        entry["useful_bytes"] = format_bytes(0, m.n_rows, m.n_cols, m.nnz, 4)
        if not args.no_cpu:
            entry.update(row=m.row, col=m.col, val=v, x=x)  # host copies for the CPU baseline
        mats.append(entry)
        print(f"[setup] {m.name}: nnz={m.nnz} best={FMT_NAMES[entry['fmt']]} "
              f"ms={[round(entry['times'][f], 4) for f in range(NF)]}", file=sys.stderr, flush=True)
    setup_s = time.perf_counter() - t_setup

    def step(events=None, key="fmt"):
        for i, e in enumerate(mats):
            pair = events[i] if events is not None else None
            if pair is not None:
                pair[0].record(stream)
            S.spmv_run(e["h"], e[key], 1.0, e["xd"], 0.0, e["y"])
            if pair is not None:
                pair[1].record(stream)

    # Everything else that launches kernels runs before the timed region, so the
    # timed launches are the last SpMV dispatches of the run (a kernel trace's last
    # `launches` dispatches of the roofline kernel are exactly the timed ones).
    selector = None if args.kernels_only else selector_section(S, torch, mats, step, args.steps)
    setup_rates = {
        "ingest_nnz_per_s": round(total_nnz_of(mats) / sum(e["t_ingest"] for e in mats), 0),
        "features_nnz_per_s": round(total_nnz_of(mats) / sum(e["t_feat"] for e in mats), 0),
        "convert_nnz_per_s": {FMT_NAMES[f]: round(
            sum(e["nnz"] for e in mats if f in e["t_convert"])
            / max(sum(e["t_convert"][f] for e in mats if f in e["t_convert"]), 1e-12), 0)
            for f in range(2, NF)},
        "note": "host wall clock around each synchronous call, COO already in HBM; the paper's "
                "CPU figures are about 4.8e5 (features) and 4.3e5 (conversion) nnz/s",
    }
    power_law = None
    if not args.kernels_only:
        rates, power_law = ingest_unsorted(S, torch, synth, tune=plan is None)
        setup_rates.update(rates)
    fp64 = None if (args.no_fp64 or plan is not None) else fp64_section(S, torch, synth, seeds)
    energy = None if args.kernels_only else energy_section(S, mats)
    batched = None if args.no_batched else batched_section(S, torch, synth,
                                                           args.batched_matrices)

    def group_key(e):
        """Launches of one kernel function (all its template instances) form a group when a
        launch is that one kernel; launches of several kernels group by exact variant."""
        info = S.spmv_variant_describe(e["fmt"], S.SPMV_F32, e["variant"][e["fmt"]])
        syms = kernel_symbols(e["fmt"], info)
        if len(syms) == 1:
            fn = syms[0].split("<")[0]
            return f"{fn}_f32", info, [f"{fn}<float, "]
        if syms[0].startswith("coo_tiles_kernel<"):  # kernels no other variant runs
            return "coo_tiles_kernel_f32", info, ["coo_tiles_kernel<float, ", syms[1]]
        key = (f"{info['kernel']}_b{info['block']}_l{info['lanes']}_u{info['unroll']}"
               f"_v{info['vec']}_p{info['pipelined']}_k{info['ksplit']}_f32")
        return key, info, syms

    def new_events(n):
        return [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                for _ in range(n)]

    # The chosen plan, each SpMV timed alone after a cache scrub: median, mean and p95
    # over 20 runs per matrix, summed over the matrices (before the timed steps, so
    # the timed launches stay the run's last SpMV dispatches).
    cold = np.array([S.spmv_time(e["h"], e["fmt"], e["xd"], e["y"], variant=e["variant"][e["fmt"]],
                                 warmup=1, reps=20, flush=True) for e in mats])  # ms, [30, 20]
    useful_all = sum(e["useful_bytes"] for e in mats)
    cold_plan = {"reps": 20, "median_ms": round(float(np.median(cold, axis=1).sum()), 4),
                 "mean_ms": round(float(cold.mean(axis=1).sum()), 4),
                 "p95_ms": round(float(np.percentile(cold, 95, axis=1).sum()), 4)}
    cold_plan["useful_gbps_median"] = round(useful_all / (cold_plan["median_ms"] * 1e-3) / 1e9, 1)
    cold_plan["frac_of_peak_median"] = round(cold_plan["useful_gbps_median"] / HBM_PEAK_GBPS, 4)
    cold_plan["stored_gbps_median"] = round(
        sum(e["bytes"][e["fmt"]] for e in mats) / (cold_plan["median_ms"] * 1e-3) / 1e9, 1)
    cold_med = {id(e): float(np.median(cold[i])) for i, e in enumerate(mats)}

    # Warmup steps carry a pair of events on every launch: they give the kernel time per
    # step and pick the roofline kernel, the (format, variant) group with the largest
    # share of kernel time.
    warm = [0.0 for _ in mats]
    for _ in range(max(args.warmup, 1)):
        ev = new_events(len(mats))
        step(ev)
        torch.cuda.synchronize()
        for i, (a, b) in enumerate(ev):
            warm[i] += a.elapsed_time(b) / max(args.warmup, 1)
    kernel_ms_per_step = sum(warm)
    groups = {}
    for i, e in enumerate(mats):
        key, info, syms = group_key(e)
        g = groups.setdefault(key, {"warm_ms": 0.0, "members": [], "symbols": syms})
        g["warm_ms"] += warm[i]
        g["members"].append(i)
    dom_key = max(groups, key=lambda k: groups[k]["warm_ms"])
    if args.roofline_kernel and args.roofline_kernel in groups:
        # counter runs: the kernel the timed run found dominant (profilers reorder the shares)
        dom_key = args.roofline_kernel
    dom = groups[dom_key]
    members = set(dom["members"])

    # Timed steps: the matrices are independent, so each step runs the roofline kernel's
    # launches first, back to back, bracketed by one pair of events (per-launch events
    # would add their own dispatch gaps), then the others; all K steps are enqueued
    # without waiting, so launch overhead overlaps the kernels.
    # Inside the group the launches are ordered by kernel instance, with one more event
    # at each change of instance, which gives each instance its own achieved rate.
    def instance(e):
        info = S.spmv_variant_describe(e["fmt"], S.SPMV_F32, e["variant"][e["fmt"]])
        sym = kernel_symbols(e["fmt"], info)[0]
        if sym.startswith("coo_tiles_kernel<"):  # the tile count is a launch argument
            sym += f"... ({info['ksplit']} tiles)"
        return sym

    order = sorted(range(len(mats)),
                   key=lambda i: (i not in members, instance(mats[i]) if i in members else "", i))
    mats[:] = [mats[i] for i in order]
    n_dom = len(members)
    inst = [instance(mats[i]) for i in range(n_dom)]
    bounds = [0] + [i for i in range(1, n_dom) if inst[i] != inst[i - 1]] + [n_dom]

    def timed_step(evl):
        for i, e in enumerate(mats):
            if i == 0:
                evl[0].record(stream)
            S.spmv_run(e["h"], e["fmt"], 1.0, e["xd"], 0.0, e["y"])
            if i + 1 in bounds[1:]:
                evl[bounds.index(i + 1)].record(stream)

    evs = [[torch.cuda.Event(enable_timing=True) for _ in bounds] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        timed_step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dom["ms"] = sum(evl[0].elapsed_time(evl[-1]) for evl in evs)
    dom["launches"] = n_dom * args.steps
    dom["bytes"] = args.steps * sum(e["bytes"][e["fmt"]] for e in mats[:n_dom])
    instances = []
    for j in range(len(bounds) - 1):
        a, b = bounds[j], bounds[j + 1]
        ms = sum(evl[j].elapsed_time(evl[j + 1]) for evl in evs)
        nb = args.steps * sum(e["bytes"][e["fmt"]] for e in mats[a:b])
        gbps = nb / (ms * 1e-3) / 1e9
        instances.append({"kernel_symbol": inst[a], "launches": (b - a) * args.steps,
                          "avg_launch_us": round(ms * 1e3 / ((b - a) * args.steps), 3),
                          "achieved": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBPS, 4)})
    for e in mats:  # outputs of the last timed step, for the CPU leg's check
        e["y_gpu"] = e["y"].cpu().numpy()
    if args.copy_calibration:  # the run's last device work: three copies of known size
        src = torch.zeros(args.copy_calibration * 2**18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ms_per_step = wall * 1e3 / args.steps

    useful = sum(e["useful_bytes"] for e in mats)
    cold_dom_ms = sum(cold_med[id(e)] for e in mats[:n_dom])
    cold_dom_achieved = sum(e["bytes"][e["fmt"]] for e in mats[:n_dom]) / (cold_dom_ms * 1e-3) / 1e9
    value = useful / (ms_per_step * 1e-3) / 1e9
    achieved = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
    traffic = load_traffic(dom_key)

    def rate(pairs):
        tb = sum(bb for bb, _ in pairs)
        tt = sum(tm for _, tm in pairs) * 1e-3
        return round(tb / tt / 1e9, 1), round(tb / tt / 1e9 / HBM_PEAK_GBPS, 4)

    per_format = {}
    for fmt in range(NF):
        ok = [e for e in mats if np.isfinite(e["times"][fmt])]
        if not ok:
            continue
        g, f = rate([(e["bytes"][fmt], e["times"][fmt]) for e in ok])
        d = {"matrices": len(ok), "gbps": g, "frac_of_peak": f}
        large = [e for e in ok if e["bytes"][fmt] >= 256e6]
        if large:
            d["large_matrices"] = len(large)
            d["large_gbps"], d["large_frac"] = rate([(e["bytes"][fmt], e["times"][fmt]) for e in large])
        per_format[FMT_NAMES[fmt]] = d
    if all("coo_tiled_ms" in e for e in mats):
        g, f = rate([(e["coo_tiled_bytes"], e["coo_tiled_ms"]) for e in mats])
        d = {"matrices": len(mats), "gbps": g, "frac_of_peak": f,
             "kernel": "tiled segmented COO (row, col, val triplets), best of its variants"}
        large = [e for e in mats if e["coo_tiled_bytes"] >= 256e6]
        if large:
            d["large_matrices"] = len(large)
            d["large_gbps"], d["large_frac"] = rate([(e["coo_tiled_bytes"], e["coo_tiled_ms"]) for e in large])
        per_format["COO_tiled"] = d
    # each format's useful (CSR-byte) rate per structure family, tuned cold medians
    by_family = {}
    for fam in sorted({e["family"] for e in mats}):
        fm = [e for e in mats if e["family"] == fam]
        row = {}
        for fmt in range(NF):
            ok = [e for e in fm if np.isfinite(e["times"][fmt])]
            if len(ok) == len(fm):
                row[FMT_NAMES[fmt]] = rate([(e["useful_bytes"], e["times"][fmt]) for e in ok])[0]
        by_family[fam] = row
    # the compile-time mode's result here: tuned variant against the library's default one
    autotune = None
    if all(e["default_ms"] for e in mats):
        autotune = {}
        for fmt in range(NF):
            sp = [e["default_ms"][fmt] / e["times"][fmt] for e in mats if fmt in e["default_ms"]
                  and np.isfinite(e["times"][fmt]) and e["times"][fmt] > 0]
            if sp:
                autotune[FMT_NAMES[fmt]] = {
                    "matrices": len(sp), "mean_speedup": round(float(np.mean(sp)), 3),
                    "max_speedup": round(float(np.max(sp)), 3),
                    "sum_default_over_tuned": round(
                        sum(e["default_ms"][fmt] for e in mats if fmt in e["default_ms"]
                            and np.isfinite(e["times"][fmt]))
                        / sum(e["times"][fmt] for e in mats if fmt in e["default_ms"]
                              and np.isfinite(e["times"][fmt])), 3)}
        autotune["note"] = ("cold medians of each format's default variant (chosen from the row "
                            "lengths) over its tuned variant (fastest of all compiled variants)")
    chosen = {FMT_NAMES[f]: sum(1 for e in mats if e["fmt"] == f) for f in range(NF)}

    cpu = None
    if not args.no_cpu:
        # the cores this process may use (its affinity, and the OpenMP share when one is set)
        threads = len(os.sched_getaffinity(0))
        if os.environ.get("OMP_NUM_THREADS", "").isdigit():
            threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
        cpu = cpu_baseline(mats, args.cpu_budget, max(1, threads))

    total_nnz = sum(e["nnz"] for e in mats)
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "accumulate": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{len(mats)} seeded single-SpMV matrices (banded, uniform random, "
                        "8x8 block diagonal, 3-D 7-point stencil; 1e5-2e6 rows, 1e6-5e7 nnz), "
                        "FP32 values, int32 indices, one y=A*x per matrix per step in the "
                        "format (CSR, COO, ELL, HYB, SELL, BELL) and variant chosen by "
                        "exhaustive autotuned timing"
                        + (f"; diagnostic run: {args.format} forced where it applies"
                           if args.format else ""),
            "matrices": len(mats),
            "total_nnz": int(total_nnz),
            "useful_bytes_per_step": int(useful),
        },
        "value_frac_of_peak": round(value / HBM_PEAK_GBPS, 4),
        "value_cold_scrubbed": cold_plan["useful_gbps_median"],
        "value_cold_frac_of_peak": cold_plan["frac_of_peak_median"],
        "gflops": round(2 * total_nnz / (ms_per_step * 1e-3) / 1e9, 1),
        "kernel_ms_per_step": round(kernel_ms_per_step, 4),
        "roofline": {
            "bound": "hbm",
            "kernel": dom_key,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "share_of_kernel_time": round(dom["warm_ms"] / kernel_ms_per_step, 3),
            "kernel_symbol": dom["symbols"][0],
            # every kernel of a launch where each runs on every launch (the column-tile pair);
            # otherwise the main kernel (a HYB launch skips its tail kernels when the tail is empty)
            "kernel_symbols": dom["symbols"] if dom_key == "coo_tiles_kernel_f32" else dom["symbols"][:1],
            "kernels_per_launch": len(dom["symbols"]),
            "launches": dom["launches"],
            "avg_launch_us": round(dom["ms"] * 1e3 / dom["launches"], 3),
            "bytes_per_launch": round(dom["bytes"] / dom["launches"], 1),
            "instances": instances,
            "cold_achieved": round(cold_dom_achieved, 1),
            "cold_frac": round(cold_dom_achieved / HBM_PEAK_GBPS, 4),
            "bytes": "as stored: the layout the chosen variant streams (padding, reordered "
                     "copies, 16-bit rows and pointer arrays included), x once, y once",
        },
        "cpu_baseline": cpu,
        "copy_calibration_mib": args.copy_calibration,
        "per_format_tuned_cold": per_format,
        "by_family_useful_gbps": by_family,
        "autotune_vs_default": autotune,
        "cold_plan": cold_plan,
        "selected_formats": chosen,
        "setup_s": round(setup_s, 1),
        "setup_rates": setup_rates,
        "selector": selector,
        "batched": batched,
        "energy": energy,
        "power_law": power_law,
        "fp64": fp64,
        "plan": [{"name": e["name"], "fmt": e["fmt"],
                  "variants": [e["variant"][f] for f in range(NF)],
                  "times": [e["times"][f] if np.isfinite(e["times"][f]) else None
                            for f in range(NF)]} for e in mats],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
