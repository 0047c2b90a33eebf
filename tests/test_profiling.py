"""CPU: the rocprofv3 summary used for the roofline's traffic field.

Synthetic CSVs in rocprofv3's column layout stand in for a counter run: the
summary must scale each counter by the copy kernel's bytes per counter unit,
average per dispatch, and be ignored by the benchmark once the kernel's
sources no longer match the recorded hash."""
from __future__ import annotations

import csv
import os

from paper_1410_5561_amd import profiling


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def _runs(tmp_path):
    row = "void mwd::mwd_row_kernel<1, double, 8, 1>(mwd::MwdArgs<double>, mwd::MwdRow)"
    copy = "mwd::stream_copy_kernel(u32x4*, u32x4 const*, long long)"
    trace = tmp_path / "trace" / "host"
    _write(str(trace / "1_kernel_trace.csv"),
           ["Kind", "Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [["K", 1, row, 1000, 3001000], ["K", 2, row, 4000000, 9000000], ["K", 3, copy, 0, 500000]])
    _write(str(trace / "1_kernel_stats.csv"), ["Name", "Calls", "AverageNs", "MinNs", "MaxNs"],
           [[row, 2, 4000000, 3000000, 5000000]])
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    # FETCH_SIZE reads half the bytes for the copy (1 KiB per 2048 B): two
    # row dispatches of 1000 and 3000 units; counters split over two rows
    # of the same dispatch are summed
    _write(str(tmp_path / "fetch" / "h" / "2_counter_collection.csv"), hdr,
           [[1, row, "FETCH_SIZE", 600], [1, row, "FETCH_SIZE", 400], [2, row, "FETCH_SIZE", 3000],
            [7, copy, "FETCH_SIZE", 1024 * 1024]])
    _write(str(tmp_path / "write" / "h" / "3_counter_collection.csv"), hdr,
           [[1, row, "WRITE_SIZE", 100], [2, row, "WRITE_SIZE", 300], [7, copy, "WRITE_SIZE", 2 * 1024 * 1024]])
    return tmp_path


def test_counter_and_duration_averages(tmp_path):
    d = _runs(tmp_path)
    n, us = profiling.kernel_durations(str(d / "trace"), "mwd_row_kernel")
    assert n == 2 and abs(us - 4000.0) < 1e-9
    n, v = profiling.counter_per_dispatch(str(d / "fetch"), "mwd_row_kernel", "FETCH_SIZE")
    assert n == 2 and v == 2000.0
    n, v = profiling.counter_per_dispatch(str(d / "write"), "stream_copy_kernel", "WRITE_SIZE")
    assert n == 1 and v == 2 * 1024 * 1024


def test_summary_scales_by_copy_kernel_and_gates_on_source_hash(tmp_path, monkeypatch):
    d = _runs(tmp_path)
    out = tmp_path / "profiles" / "x.txt"
    monkeypatch.setattr(profiling, "PROFILES", str(tmp_path / "profiles"))
    out = profiling.summary_path("mwd_row_kernel", "wl^1", "f64", "8x64")
    rc = profiling.main(["--trace", str(d / "trace"), "--fetch", str(d / "fetch"), "--write", str(d / "write"),
                         "--kernel", "mwd_row_kernel", "--workload", "wl^1", "--dtype", "f64", "--shape", "8x64",
                         "--model-bytes-per-launch", "4000000", "--copy-bytes", str(2 << 30),
                         "--cmd-trace", "t", "--cmd-fetch", "f", "--cmd-write", "w", "--out", out])
    assert rc == 0
    s = profiling.read_summary(out)
    # copy: 2 GiB over 1 Mi units = 2048 B per FETCH unit, 1024 B per WRITE unit
    assert abs(float(s["fetch_scale_bytes_per_kib"]) - 2048.0) < 1e-6
    assert abs(float(s["write_scale_bytes_per_kib"]) - 1024.0) < 1e-6
    assert float(s["traffic_bytes_per_launch"]) == 2000 * 2048 + 200 * 1024
    assert profiling.traffic_for("mwd_row_kernel", "wl^1", "f64", "8x64") == 2000 * 2048 + 200 * 1024
    # a summary taken from other sources is not used
    with open(out) as f:
        text = f.read()
    with open(out, "w") as f:
        f.write(text.replace("source_hash: " + s["source_hash"], "source_hash: 0000"))
    assert profiling.traffic_for("mwd_row_kernel", "wl^1", "f64", "8x64") is None
    assert profiling.traffic_for("mwd_row_kernel", "other", "f64", "8x64") is None


def test_sq_summary_averages_and_ratios(tmp_path):
    """SQ counters from two --pmc runs: per-dispatch averages (counters of one
    dispatch split over rows are summed), wait fractions, the L2 hit rate and
    per-wave instruction counts."""
    k = "void mwd::naive_sweep_kernel<2, float, 64, 16>(float const*, float*)"
    other = "mwd::stream_copy_kernel(u32x4*, u32x4 const*, long long)"
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    _write(str(tmp_path / "a" / "h" / "1_counter_collection.csv"), hdr,
           [[1, k, "SQ_WAVES", 100], [1, k, "SQ_WAVE_CYCLES", 600], [1, k, "SQ_WAVE_CYCLES", 400],
            [1, k, "SQ_WAIT_INST_ANY", 250], [2, k, "SQ_WAVES", 100], [2, k, "SQ_WAVE_CYCLES", 1000],
            [2, k, "SQ_WAIT_INST_ANY", 250], [1, k, "SQ_INSTS_VALU", 5000], [2, k, "SQ_INSTS_VALU", 5000],
            [3, other, "SQ_WAVES", 7]])
    _write(str(tmp_path / "b" / "h" / "2_counter_collection.csv"), hdr,
           [[1, k, "TCC_HIT_sum", 30], [1, k, "TCC_MISS_sum", 70]])
    vals, n = profiling.sq_counters([str(tmp_path / "a"), str(tmp_path / "b")], "naive_sweep_kernel")
    assert n == 2 and vals["SQ_WAVES"] == 100 and vals["SQ_WAVE_CYCLES"] == 1000
    lines = profiling.sq_summary_lines(vals, n, "naive_sweep_kernel", "w", "f32", "naive", ["cmd a", "cmd b"])
    d = dict(l.split(": ", 1) for l in lines if not l.startswith("#"))
    assert float(d["wait_inst_any_over_wave_cycles"]) == 0.25
    assert float(d["l2_hit_rate"]) == 0.3
    assert float(d["sq_insts_valu_per_wave"]) == 50.0
    assert "# run: cmd b" in lines
