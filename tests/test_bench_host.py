"""Host-side logic of bench.py (CPU only): byte formulas and the trace summary."""
import csv
import json

import numpy as np

import bench
import synth
from oracle import formats as OF


def test_format_bytes_follow_the_layouts():
    m = synth.config1_matrix()
    c = OF.canonicalize(m.n_rows, m.n_cols, m.row, m.col, m.values(np.float32))
    e, h = OF.to_ell(c), OF.to_hyb(c)
    xy = 4096 * 4 * 2
    assert bench.format_bytes(0, 4096, 4096, 20224, 4) == 20224 * 8 + 4097 * 4 + xy
    assert bench.format_bytes(1, 4096, 4096, 20224, 4) == 20224 * 12 + xy
    assert bench.format_bytes(2, 4096, 4096, 20224, 4, e["K"], e["pitch"]) == e["ell_col"].size * 8 + xy
    tail = h["tail_row"].size
    assert bench.format_bytes(3, 4096, 4096, 20224, 4, h["K"], h["pitch"], tail) == \
        h["ell_col"].size * 8 + tail * 12 + xy
    assert bench.format_bytes(0, 4096, 4096, 20224, 8) == 20224 * 12 + 4097 * 4 + 4096 * 8 * 2


def test_kernel_symbols_name_every_family():
    base = {"block": 256, "lanes": 8, "unroll": 2, "vec": 4, "pipelined": 0, "ksplit": 1}
    assert bench.kernel_symbols(0, dict(base, kernel="csr_vector")) == ["csr_vector4_kernel<float, 256, 8, 2>"]
    assert bench.kernel_symbols(0, dict(base, kernel="csr_vector", pipelined=4)) == ["csr_pipe_kernel<float, 256, 8, 4>"]
    assert bench.kernel_symbols(2, dict(base, kernel="ell", lanes=4, ksplit=4, pipelined=1)) == \
        ["ell_ksplit_kernel<float, 4, 4>"]
    assert len(bench.kernel_symbols(3, dict(base, kernel="hyb", lanes=2, unroll=4))) == 3


def test_trace_summary_uses_the_last_timed_launches(tmp_path, capsys):
    trace = tmp_path / "t.csv"
    with open(trace, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for i in range(10):  # 6 tuning launches of 1 us, then 4 timed launches of 2 us
            d = 1000 if i < 6 else 2000
            w.writerow({"Kernel_Name": "void spmv::k<float, 256>(int)", "Start_Timestamp": 10000 * i,
                        "End_Timestamp": 10000 * i + d})
        w.writerow({"Kernel_Name": "other", "Start_Timestamp": 1, "End_Timestamp": 99999})
    js = tmp_path / "b.json"
    js.write_text("noise\n" + json.dumps({"roofline": {"kernel_symbol": "k<float, 256>", "launches": 4,
                                                      "avg_launch_us": 2.1, "bytes_per_launch": 4e6,
                                                      "achieved": 1900.0}}) + "\n")
    bench.trace_summary(str(trace), str(js))
    out = capsys.readouterr().out
    assert "timed-region dispatches used: 4" in out
    assert "2.000 us" in out and "2000.0 GB/s" in out
