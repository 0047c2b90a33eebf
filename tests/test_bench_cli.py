"""CPU: the parts of the benchmark that need no GPU: the one-GPU refusal,
the oracle baseline's sampling and fields, and the FP32 error bound."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import gridgen  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_cpu_baseline_sample_and_fields():
    w = dict(name="7v-small", kind="7v", dtype="f64", n=(12, 10, 8), T=3, field=(0.0, 1.0), coeffs="7v")
    r = bench.cpu_baseline(w, "f64", 2, 3, min_s=0.0, max_reps=2)
    assert r["unit"] == "GLUP/s" and r["kind"] == "oracle" and r["value"] > 0
    assert r["cores"] >= 1 and "12x10x8" in r["sample"] and "3 steps" in r["sample"]


@pytest.mark.parametrize("kind,ops", [("7c", 10), ("7v", 13), ("25c", 37), ("25v", 37)])
def test_flops_per_update(kind, ops):
    # flops of one update without FMA: 7c 4 mul + 6 add, 7v 7 + 6, 25-point 13 + 24
    assert bench.FLOPS_PER_LUP[kind] == ops
    assert gridgen.RADIUS[kind] in (1, 4)
