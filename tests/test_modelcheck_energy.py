"""CPU: the traffic-model table (measured bytes per update against Eq. (5))
and the energy meter's arithmetic.

Synthetic counter files in rocprofv3's column layout stand in for the runs;
the model column is checked against the library's own Eq. (5) entry point,
and the energy measurement against a meter with a known counter."""
from __future__ import annotations

import csv
import os

import pytest

import paper_1410_5561_amd as S
from paper_1410_5561_amd import energy, modelcheck

ROW = "void mwd::mwd_row_kernel<1, double, 8, 1>(mwd::MwdArgs<double>, mwd::MwdRow)"
GATHER = "void mwd::mwd_gather_kernel<double, 1, 8>(mwd::MwdArgs<double>)"
COPY = "mwd::stream_copy_kernel(u32x4*, u32x4 const*, long long)"
HDR = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "LDS_Block_Size", "Workgroup_Size",
       "Scratch_Size"]


def _write(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HDR)
        w.writerows(rows)


@pytest.mark.parametrize("kind,elem,dw", [("7v", 8, 8), ("7v", 4, 4), ("25c", 8, 16), ("7c", 8, 0), ("25v", 4, 32)])
def test_model_matches_library(kind, elem, dw):
    assert modelcheck.model_bytes_per_lup(kind, elem, dw) == pytest.approx(
        S.stencil_model_bytes_per_lup(kind, "f64" if elem == 8 else "f32", dw), rel=1e-12)


def test_table_scales_sums_and_divides(tmp_path):
    root = tmp_path / "w"
    # copy: 2048 bytes per FETCH unit, 1024 per WRITE unit; two row dispatches
    # (one split over two counter rows) and a gather
    _write(str(root / "8x64" / "fetch" / "a" / "1_counter_collection.csv"),
           [[1, ROW, "FETCH_SIZE", 600, 78848, 512, 0], [1, ROW, "FETCH_SIZE", 400, 78848, 512, 0],
            [2, ROW, "FETCH_SIZE", 3000, 78848, 512, 0], [3, GATHER, "FETCH_SIZE", 500, 0, 256, 0],
            [4, COPY, "FETCH_SIZE", 1024, 0, 256, 0], [5, COPY, "FETCH_SIZE", 1024, 0, 256, 0]])
    _write(str(root / "8x64" / "write" / "a" / "2_counter_collection.csv"),
           [[1, ROW, "WRITE_SIZE", 1000, 78848, 512, 0], [2, ROW, "WRITE_SIZE", 1000, 78848, 512, 0],
            [3, GATHER, "WRITE_SIZE", 1000, 0, 256, 0], [4, COPY, "WRITE_SIZE", 2048, 0, 256, 0]])
    out = tmp_path / "t.txt"
    modelcheck.main(["--root", str(root), "--workload", "w", "--kind", "7v", "--dtype", "f64",
                     "--lups-per-run", "1000", "--copy-bytes", str(2048 * 1024), "--cmd", "c",
                     "--out", str(out), "8x64"])
    line = [l for l in out.read_text().splitlines() if l.startswith("8x64")][0].split()
    # tile: (4000 * 2048 + 2000 * 1024) / 1000; all adds the gather's 500 * 2048 + 1000 * 1024
    assert float(line[1]) == pytest.approx(22.0)
    assert float(line[2]) == pytest.approx((4000 * 2048 + 2000 * 1024) / 1000, rel=1e-4)
    assert float(line[3]) == pytest.approx((4500 * 2048 + 3000 * 1024) / 1000, rel=1e-4)
    assert "LDS 78848 B" in out.read_text()


def test_table_refuses_mixed_runs(tmp_path):
    root = tmp_path / "w"
    for n in (1, 2):
        _write(str(root / "naive" / "fetch" / "a" / ("%d_counter_collection.csv" % n)),
               [[1, COPY, "FETCH_SIZE", 1, 0, 256, 0]])
    with pytest.raises(SystemExit):
        modelcheck.counter_sums(str(root / "naive" / "fetch"), "FETCH_SIZE")


class _FakeMeter:
    """A counter that advances 300 J per run and whose timestamps run at the
    same rate as the region's wall time."""
    ok = True

    def __init__(self):
        import time
        self.j = 1000.0
        self.t = time.perf_counter

    def read(self):
        return self.j, self.t()

    def power_w(self):
        return 250.0


def test_energy_measure_counts_runs_and_joules():
    m = _FakeMeter()

    def run():
        m.j += 300.0

    reps, dt, joules, pw = energy.measure(m, run, lambda: None, min_seconds=0.0, max_reps=8)
    # energy = (counter difference / counter time) x wall time: equal up to
    # the few instructions between the wall clock's and the counter's reads
    assert reps >= 1 and joules == pytest.approx(300.0 * reps, rel=0.2) and pw == 250.0 and dt >= 0.0


class _SteppedMeter(_FakeMeter):
    """A counter that reports a stale update time: the counter's own
    timestamps, not the wall time between reads, give the power."""

    def read(self):
        return self.j, self.stamp

    def power_w(self):
        return None


def test_energy_uses_counter_timestamps():
    m = _SteppedMeter()
    m.stamp = 10.0

    def run():
        m.j += 500.0
        m.stamp += 1.0  # 500 J per counter second: 500 W

    reps, dt, joules, pw = energy.measure(m, run, lambda: None, min_seconds=0.0, max_reps=4)
    assert joules == pytest.approx(500.0 * dt) and pw is None


def test_energy_meter_without_device_reports_error():
    m = energy.EnergyMeter()
    # in a container without a GPU the library cannot open a device; either way
    # the meter says whether it works instead of raising
    assert isinstance(m.ok, bool)
    if not m.ok:
        assert m.error
    m.close()


def test_cacheblock_tool_matches_the_worked_example_and_radius4_values():
    """The cache-block table's Eq. (3) against the worked example (R = 1) and the
    hand-evaluated radius-4 values kept in tests/golden/."""
    import json
    from paper_1410_5561_amd import cacheblock
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    g1 = json.load(open(os.path.join(here, "cache_block_example.json")))
    kind = "7c"  # N_D = 2, R = 1 as in the example
    assert cacheblock.cache_block(kind, 8, g1["Dw"], 1, nf=g1["N_F"]) == 8 * g1["C_S_per_Nxb"]
    g4 = json.load(open(os.path.join(here, "cache_block_r4.json")))
    for c in g4["cases"]:
        k = {2: "25c", 15: "25v"}[c["N_D"]]
        assert cacheblock.cache_block(k, 4, c["Dw"], 32, nf=c["N_F"]) == 128 * c["C_S_per_Nxb"]
