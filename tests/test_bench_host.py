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
    # HYB's tiled tail runs 256-thread workgroups whatever the ELL part's workgroup size
    assert bench.kernel_symbols(3, dict(base, kernel="hyb", block=1024, lanes=2, unroll=8)) == \
        ["ell_kernel<float, 1024, 2, 4>", "coo_tile_kernel<float, 256, 8, true>",
         "coo_fixup<float, 2048, true>"]
    # HYB with its ELL part split over 4 waves
    assert bench.kernel_symbols(3, dict(base, kernel="hyb", lanes=4, unroll=8, ksplit=4))[0] == \
        "ell_ksplit_kernel<float, 4, 4>"
    assert bench.kernel_symbols(4, dict(base, kernel="sell", unroll=2, pipelined=1)) == \
        ["sell_kernel<float, 256, 2, true, "]
    assert bench.kernel_symbols(5, dict(base, kernel="bell")) == ["bell_kernel<float, "]
    # sorted-block COO in column tiles: the tile kernel, then the combine
    assert bench.kernel_symbols(1, dict(base, kernel="coo_sorted", block=1024, lanes=16, ksplit=2)) == \
        ["coo_tiles_kernel<float, 16, ", "sorted_tiles_combine<float>"]
    assert bench.kernel_symbols(1, dict(base, kernel="coo_sorted", block=1024, lanes=16)) == \
        ["coo_sorted_kernel<float, 16, "]


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


def _counter_csv(path, counter, rows):
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": value})


def test_counter_summary_scales_by_the_calibration_copy(tmp_path, capsys):
    k = "void spmv::csr_vector4_kernel<float, 256, 16, 2>(int)"
    copy = "__amd_rocclr_copyBuffer"
    # a tuning dispatch, then 2 timed dispatches, then three 4 MiB calibration copies;
    # the FETCH counter reads half of the true bytes, WRITE reads them exactly
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE",
                 [(k, 9999.0), (k, 1000.0), (k, 3000.0)] + [(copy, 2048.0)] * 3)
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE",
                 [(k, 9999.0), (k, 100.0), (k, 300.0)] + [(copy, 4096.0)] * 3)
    (tmp_path / "b.json").write_text(json.dumps({
        "copy_calibration_mib": 4,
        "roofline": {"kernel": "csr_key", "kernel_symbol": "csr_vector4_kernel<float, 256, 16, 2>",
                     "launches": 2, "bytes_per_launch": 4.0e6}}) + "\n")
    bench.counter_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"),
                          str(tmp_path / "b.json"), str(tmp_path / "t.json"))
    t = json.loads((tmp_path / "t.json").read_text())
    assert t["fetch_scale"] == 2.0 and t["write_scale"] == 1.0
    assert t["kernels"]["csr_key"] == (2000.0 * 2.0 + 200.0) * 1024
    assert t["source_hash_by_kernel"]["csr_key"] == bench.kernel_source_hash("csr_key")
    assert bench.kernel_source_hash("coo_sorted_kernel_f32") != bench.kernel_source_hash("csr_key")
    assert "traffic / algorithmic" in capsys.readouterr().out


def test_request_summary_prices_reads_by_request_size(tmp_path, capsys):
    path = tmp_path / "req.csv"
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    mib = 1
    rows = []
    disp = 0
    # one tuning dispatch, then 2 timed dispatches: 10 x 32 B, 20 x 64 B, 30 x 128 B each
    for k, (a, b, c) in enumerate([(1, 1, 1), (10, 20, 30), (10, 20, 30)]):
        disp += 1
        for name, v in zip(bench.REQ_COUNTERS, (a, b, c, a + b + c)):
            rows.append((disp, "void spmv::k<float, 4>()", name, v))
    for _ in range(3):  # the calibration copy: 1 MiB in 128-byte requests
        disp += 1
        for name, v in zip(bench.REQ_COUNTERS, (0, 0, 8192, 8192)):
            rows.append((disp, "__amd_rocclr_copyBuffer", name, v))
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(fields)
        w.writerows(rows)
    js = tmp_path / "b.json"
    js.write_text(json.dumps({"roofline": {"kernel_symbol": "k<float, ", "launches": 2, "kernel": "k_f32",
                                           "bytes_per_launch": 5000.0},
                              "copy_calibration_mib": mib}) + "\n")
    out = tmp_path / "traffic.json"
    out.write_text(json.dumps({"kernel_source_hash": "x", "kernels": {"other": 1}}))
    bench.request_summary(str(path), str(js), str(out))
    d = json.loads(out.read_text())
    assert d["read_bytes_by_request_size"]["k_f32"] == 10 * 32 + 20 * 64 + 30 * 128
    assert d["read_bytes_by_request_size_copy_check"] == 1.0
    assert d["kernels"] == {"other": 1}  # the other figures stay
    assert "| requests in none of the three sizes, per launch | 0 |" in capsys.readouterr().out


def test_trace_summary_adds_the_kernels_of_one_launch(tmp_path, capsys):
    """A roofline group whose launch runs two kernels: the per-launch duration is the sum of
    the two kernels' averages over their last `launches` dispatches."""
    trace = tmp_path / "t.csv"
    with open(trace, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        t = 0
        for i in range(5):  # 2 untimed then 3 timed launches: main 10/20 us, combine 2/3 us
            for name, d in (("void spmv::coo_tiles_kernel<float, 8, false, true>(int)", 10000 if i < 2 else 20000),
                            ("void spmv::sorted_tiles_combine<float>(long)", 2000 if i < 2 else 3000)):
                w.writerow({"Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + d})
                t += 100000
    js = tmp_path / "b.json"
    js.write_text(json.dumps({"roofline": {"kernel_symbol": "coo_tiles_kernel<float, ",
                                           "kernel_symbols": ["coo_tiles_kernel<float, ",
                                                              "sorted_tiles_combine<float>"],
                                           "launches": 3, "avg_launch_us": 23.5,
                                           "bytes_per_launch": 1e8, "achieved": 4255.3}}) + "\n")
    bench.trace_summary(str(trace), str(js))
    out = capsys.readouterr().out
    assert "rocprofv3 average duration over the timed launches: 23.000 us" in out
    assert "achieved from rocprofv3 duration: 4347.8 GB/s" in out


def test_counter_summary_adds_the_kernels_of_one_launch(tmp_path, capsys):
    """Two kernels per launch (column tiles and their combine): each kernel's last `launches`
    dispatches are averaged and the two means added."""
    k1 = "void spmv::coo_tiles_kernel<float, 8, false, true>(int)"
    k2 = "void spmv::sorted_tiles_combine<float>(long)"
    copy = "__amd_rocclr_copyBuffer"
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE",
                 [(k1, 1.0), (k2, 1.0), (k1, 1000.0), (k2, 100.0), (k1, 3000.0), (k2, 300.0)]
                 + [(copy, 2048.0)] * 3)
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE",
                 [(k1, 1.0), (k2, 1.0), (k1, 10.0), (k2, 50.0), (k1, 30.0), (k2, 150.0)]
                 + [(copy, 4096.0)] * 3)
    (tmp_path / "b.json").write_text(json.dumps({
        "copy_calibration_mib": 4,
        "roofline": {"kernel": "coo_tiles_kernel_f32", "kernel_symbol": "coo_tiles_kernel<float, ",
                     "kernel_symbols": ["coo_tiles_kernel<float, ", "sorted_tiles_combine<float>"],
                     "launches": 2, "bytes_per_launch": 4.0e6}}) + "\n")
    bench.counter_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"),
                          str(tmp_path / "b.json"), str(tmp_path / "t.json"))
    t = json.loads((tmp_path / "t.json").read_text())
    # fetch (2000 + 200) x 2, write 20 + 100, per launch
    assert t["kernels"]["coo_tiles_kernel_f32"] == ((2000.0 + 200.0) * 2.0 + 20.0 + 100.0) * 1024
    assert bench.kernel_source_hash("coo_tiles_kernel_f32") == bench.kernel_source_hash("coo_sorted_kernel_f32")
    assert "coo_tiles_kernel<float,  + sorted_tiles_combine<float>" in capsys.readouterr().out
