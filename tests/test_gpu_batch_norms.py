"""GPU: the batched form (one hipGraph: batched naive sweeps for some grids,
MWD row groups for others) and the FP64 reductions, through the C ABI,
against the CPU oracle."""
from __future__ import annotations

import numpy as np
import pytest

import gridgen
import oracle
import paper_1410_5561_amd as S
from gpu_util import device_coeffs, device_grid, run_gpu
from oracle import norms as onorms

pytestmark = pytest.mark.gpu

SPECS = [("7c", (40, 33, 20)), ("25c", (50, 37, 18)), ("7c", (17, 70, 9)), ("25c", (33, 16, 40)),
         ("7c", (130, 5, 7)), ("25c", (64, 64, 11)), ("7c", (3, 2, 1)), ("25c", (1, 9, 30)),
         ("7c", (96, 48, 32)), ("7v", (45, 20, 13))]


def _inputs(kind, n, dtype, seed):
    R = gridgen.RADIUS[kind]
    u0 = gridgen.field(seed, *n, R, -1.0, 1.0, dtype)
    if kind == "7v":
        co = [c.astype(dtype) for c in gridgen.coeffs_7v(seed, *n, R)]
    else:
        co = gridgen.C7 if kind == "7c" else gridgen.C25
    return u0, co


@pytest.mark.parametrize("dts", ["f32", "f64"])
@pytest.mark.parametrize("T", [16, 5])
@pytest.mark.parametrize("sched", ["auto", "naive", "mwd"])
def test_batched_mixed_grids_bitexact_and_replay(dts, T, sched, monkeypatch):
    """Every grid of a mixed batch matches the oracle bit for bit after each
    of three replays of the same graph, with the schedule the tuner picks per
    grid, and with every grid forced onto the batched naive sweep or onto the
    batched MWD tiles (kinds without a batched tile shape stay naive)."""
    import torch
    if sched != "auto":
        monkeypatch.setenv("MWD_TUNE", sched)
    dtype = np.float64 if dts == "f64" else np.float32
    print("batched", dts, "T", T, sched, flush=True)
    inputs = [_inputs(k, n, dtype, 100 + i) for i, (k, n) in enumerate(SPECS)]
    grids, keep, coeffs = [], [], []
    for (kind, n), (u0, co) in zip(SPECS, inputs):
        g, bufs = device_grid(u0, gridgen.RADIUS[kind], 0)
        c, _ = device_coeffs(kind, co, dtype)
        grids.append(g)
        keep.append(bufs)
        coeffs.append(c)
    plan = S.Plan("mixed", dts)
    for rep in (1, 2, 3):
        plan.run_batched(grids, coeffs, T)
        torch.cuda.synchronize()
        for i, ((kind, n), (u0, co)) in enumerate(zip(SPECS, inputs)):
            got = keep[i][grids[i].cur].cpu().numpy()
            gotm1 = keep[i][grids[i].cur ^ 1].cpu().numpy()
            uT, uTm1 = oracle.run(kind, u0, co, rep * T)
            assert np.array_equal(got, uT), "grid %d (%s %s) after %d runs" % (i, kind, n, rep)
            assert np.array_equal(gotm1, uTm1), "grid %d u_{T-1}" % i
    plan.close()


# every shape compiled into the batched tile kernel: (dtype, dw, lanes)
BATCH_SHAPES = [("f32", 8, 128), ("f32", 4, 256), ("f32", 16, 64),
                ("f64", 8, 128), ("f64", 4, 256)]


@pytest.mark.parametrize("shape", BATCH_SHAPES, ids=lambda c: "%s-dw%d-lx%d" % c)
def test_batched_each_tile_shape(shape, monkeypatch):
    """Each batched tile shape pinned explicitly (MWD_TUNE=mwd:<dw>:<lanes>):
    the grids of a kind with that shape run it, the others the batched naive
    sweep; every grid bit-exact against the oracle after two replays."""
    import torch
    dts, dw, lanes = shape
    monkeypatch.setenv("MWD_TUNE", "mwd:%d:%d" % (dw, lanes))
    dtype = np.float64 if dts == "f64" else np.float32
    print("batched shape", shape, flush=True)
    specs = [s for s in SPECS if dts == "f32" or s[0] != "7v"]
    inputs = [_inputs(k, n, dtype, 300 + i) for i, (k, n) in enumerate(specs)]
    grids, keep, coeffs = [], [], []
    for (kind, n), (u0, co) in zip(specs, inputs):
        g, bufs = device_grid(u0, gridgen.RADIUS[kind], 0)
        c, _ = device_coeffs(kind, co, dtype)
        grids.append(g)
        keep.append(bufs)
        coeffs.append(c)
    plan = S.Plan("mixed", dts)
    T = 9
    for rep in (1, 2):
        plan.run_batched(grids, coeffs, T)
        torch.cuda.synchronize()
        for i, ((kind, n), (u0, co)) in enumerate(zip(specs, inputs)):
            got = keep[i][grids[i].cur].cpu().numpy()
            uT, _ = oracle.run(kind, u0, co, rep * T)
            assert np.array_equal(got, uT), "grid %d (%s %s) after %d runs" % (i, kind, n, rep)
    plan.close()


@pytest.mark.parametrize("dts", ["f64", "f32"])
def test_norms_against_oracle(dts):
    import torch
    dtype = np.float64 if dts == "f64" else np.float32
    n, T = (70, 45, 33), 7
    print("norms", dts, flush=True)
    u0 = gridgen.field(9, *n, 1, 0.0, 1.0, dtype)
    C = [c.astype(dtype) for c in gridgen.coeffs_7v(9, *n, 1)]
    g, bufs = device_grid(u0, 1, 0)
    c, _ = device_coeffs("7v", C, dtype)
    plan = S.Plan("7v", dts, *n, mode="mwd", dw=8, lanes=64)
    plan.run(g, c, T)
    torch.cuda.synchronize()
    uT, uTm1 = oracle.run("7v", u0, C, T)
    l2, mx = S.stencil_norms(g, 0)
    rl2, rmx = onorms.grid_norms(uT, 1)
    # sum of n squares in another order: |err| <= n * u * sum (a loose bound);
    # the tree order here stays far below it
    assert abs(l2 - rl2) <= 1e-13 * rl2 and mx == rmx
    rl2, rmx = onorms.residual_norms(uT, uTm1, 1)
    l2, mx = S.stencil_norms(g, 1)
    assert abs(l2 - rl2) <= 1e-13 * rl2 and mx == rmx
    # diff norms between grids of different precision
    u64 = u0.astype(np.float64)
    g2, bufs2 = device_grid(u64, 1, 0)
    d2 = S.stencil_diff_norms(g, g2)
    rd = onorms.diff_norms(uT, u64, 1, 1)
    assert abs(d2[0] - rd[0]) <= 1e-13 * rd[0] and d2[1] == rd[1]
    plan.close()


@pytest.mark.parametrize("dts", ["f32", "f64"])
def test_batched_many_naive_groups(dts, monkeypatch):
    """Groups small enough that every naive grid forms its own group: the
    graph alternates groups between its two concurrent branches and joins
    them; every grid matches the oracle after two replays."""
    import torch
    monkeypatch.setenv("MWD_TUNE", "naive")
    monkeypatch.setenv("MWD_BATCH_GROUP_BYTES", "200000")
    dtype = np.float64 if dts == "f64" else np.float32
    T = 7
    print("batched many groups", dts, flush=True)
    inputs = [_inputs(k, n, dtype, 300 + i) for i, (k, n) in enumerate(SPECS)]
    grids, keep, coeffs = [], [], []
    for (kind, n), (u0, co) in zip(SPECS, inputs):
        g, bufs = device_grid(u0, gridgen.RADIUS[kind], 0)
        c, ck = device_coeffs(kind, co, dtype)
        grids.append(g)
        keep.append((bufs, ck))
        coeffs.append(c)
    plan = S.Plan("mixed", dts)
    for rep in (1, 2):
        plan.run_batched(grids, coeffs, T)
        torch.cuda.synchronize()
        for i, ((kind, n), (u0, co)) in enumerate(zip(SPECS, inputs)):
            bufs = keep[i][0]
            uT, uTm1 = oracle.run(kind, u0, co, rep * T)
            assert np.array_equal(bufs[grids[i].cur].cpu().numpy(), uT), "grid %d after %d runs" % (i, rep)
            assert np.array_equal(bufs[grids[i].cur ^ 1].cpu().numpy(), uTm1), "grid %d u_{T-1}" % i
    plan.close()


def test_batched_workload5_every_grid_against_oracle():
    """The batching workload as configured (256 grids, sides 32..256, half
    7-point and half 25-point constant, FP32, T = 16), with the schedule the
    tuner picks per grid: every grid bit-exact against the oracle."""
    import torch
    w = gridgen.workloads()[5]
    T = w["T"]
    specs = gridgen.batch_specs(count=w["count"])
    print("workload 5: generating", len(specs), "grids", flush=True)
    grids, keep, coeffs, fields = [], [], [], []
    for sp in specs:
        u0 = gridgen.batch_field(sp, np.float32)
        fields.append(u0)
        d = torch.from_numpy(u0).cuda()
        keep.append((d, d.clone()))
        grids.append(S.make_grid(keep[-1][0], keep[-1][1], sp["halo"], 0))
        coeffs.append(S.make_coeffs(sp["kind"], consts=sp["coeffs"]))
    plan = S.Plan("mixed", "f32")
    print("workload 5: running", flush=True)
    plan.run_batched(grids, coeffs, T)
    torch.cuda.synchronize()
    for i, sp in enumerate(specs):
        uT, uTm1 = oracle.run(sp["kind"], fields[i], sp["coeffs"], T)
        got = keep[i][grids[i].cur].cpu().numpy()
        assert np.array_equal(got, uT), "grid %d (%s %s)" % (i, sp["kind"], sp["n"])
        assert np.array_equal(keep[i][grids[i].cur ^ 1].cpu().numpy(), uTm1), "grid %d u_{T-1}" % i
        if i % 32 == 31:
            print("workload 5: %d grids checked" % (i + 1), flush=True)
    plan.close()


@pytest.mark.parametrize("dts", ["f64", "f32"])
def test_norms_propagate_nan(dts):
    """One NaN in the interior makes both norms NaN; NaN in the halo does not
    enter."""
    dtype = np.float64 if dts == "f64" else np.float32
    n = (33, 20, 9)
    u0 = gridgen.field(12, *n, 1, 0.0, 1.0, dtype)
    u0[0, 0, 0] = np.nan                       # a halo corner
    g, bufs = device_grid(u0, 1, 0)
    l2, mx = S.stencil_norms(g, 0)
    rl2, rmx = onorms.grid_norms(u0, 1)
    assert np.isfinite(l2) and mx == rmx and abs(l2 - rl2) <= 1e-13 * rl2
    u0[5, 7, 11] = np.nan
    g, bufs = device_grid(u0, 1, 0)
    l2, mx = S.stencil_norms(g, 0)
    assert np.isnan(l2) and np.isnan(mx)
