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


def test_25v_workload_form():
    """--kind 25v: workload 3's grid, field and T with 13 seeded weight arrays,
    non-negative, each point's weights summing to 0.999 (so a sweep does not
    amplify the max norm); the 7-point variable draws are unchanged by the
    shared generator (its first seven arrays are the 7-point recipe's draws,
    rescaled by another sum)."""
    w = bench.workload(3, "25v")
    w3 = gridgen.workloads()[3]
    assert (w["kind"], w["coeffs"], w["n"], w["T"], w["field"]) == ("25v", "25v", w3["n"], w3["T"], w3["field"])
    n, R = (9, 7, 5), 4
    c25 = gridgen.coeffs_25v(17, *n, R)
    c7 = gridgen.coeffs_7v(17, *n, 1)
    assert len(c25) == 13 and all(c.shape == (n[2] + 8, n[1] + 8, n[0] + 8) for c in c25)
    inner25 = [c[R:-R, R:-R, R:-R] for c in c25]
    inner7 = [c[1:-1, 1:-1, 1:-1] for c in c7]
    assert min(float(c.min()) for c in inner25) > 0
    assert abs(float(sum(inner25).max()) - 0.999) < 1e-12 and abs(float(sum(inner25).min()) - 0.999) < 1e-12
    assert all(float(abs(c[:R]).max()) == 0 for c in c25)   # zero halo
    # the same raw draws: the ratio of two arrays does not depend on the sum
    import numpy as np
    assert np.allclose(inner25[1] / inner25[0], inner7[1] / inner7[0], rtol=1e-13)
    with pytest.raises(SystemExit):
        bench.workload(2, "25v")
