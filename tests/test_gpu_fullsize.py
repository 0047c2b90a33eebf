"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (plans created without parameters: the autotuned schedule).

The oracle cannot sweep a 512^3 grid 64 times in a test, so it recomputes
sampled outputs one by one from their dependency cones (tests/cone.py),
bit for bit; properties that hold at any size (positivity and the maximum
principle for non-negative weights summing to < 1) are checked on the whole
result with the library's FP64 norms.
"""
from __future__ import annotations

import numpy as np
import pytest

import cone
import gridgen
import oracle
import paper_1410_5561_amd as S
from oracle import norms as onorms

pytestmark = pytest.mark.gpu


def _run_full(windex, dtype, kind=None):
    """Workload windex at full size with the autotuned plan; kind "25v" turns
    workload 3 into its variable-weight form (13 seeded weight arrays), as
    the benchmark's --kind 25v does."""
    import torch
    w = dict(gridgen.workloads()[windex])
    if kind == "25v":
        assert windex == 3
        w.update(kind="25v", coeffs="25v", name="25v-512^3-T32")
    kind, (nx, ny, nz), T = w["kind"], w["n"], w["T"]
    R = gridgen.RADIUS[kind]
    seed = gridgen.seed_for_config(windex)
    npdt = np.float64 if dtype == "f64" else np.float32
    print("workload", windex, w["name"], dtype, "generating", flush=True)
    u0 = gridgen.field(seed, nx, ny, nz, R, *w["field"], dtype=npdt)
    if w["coeffs"] in ("7v", "25v"):
        gen = gridgen.coeffs_7v if w["coeffs"] == "7v" else gridgen.coeffs_25v
        co = gen(seed, nx, ny, nz, R, dtype=npdt)
        c_dev = [torch.from_numpy(c).cuda() for c in co]
        coeffs = S.make_coeffs(kind, arrays=c_dev)
    else:
        co = list(w["coeffs"])
        c_dev = []
        coeffs = S.make_coeffs(kind, consts=co)
    a = torch.from_numpy(u0).cuda()
    b = a.clone()
    g = S.make_grid(a, b, R, 0)
    plan = S.Plan(kind, dtype, nx, ny, nz)   # autotuned, as the benchmark
    print("workload", windex, "running", flush=True)
    plan.run(g, coeffs, T)
    torch.cuda.synchronize()
    desc = plan.describe()
    print("workload", windex, "schedule", desc, flush=True)
    return w, u0, co, g, (a, b), plan, c_dev


def _check_samples(w, u0, co, g, bufs, count):
    kind, n, T = w["kind"], w["n"], w["T"]
    R = gridgen.RADIUS[kind]
    res = bufs[g.cur]
    for p in cone.sample_points(n, count, seed=T):
        got = res[p[2] + R, p[1] + R, p[0] + R].item()
        ref = cone.subbox_value(kind, u0, co, T, R, p)
        assert got == ref, "point %s: gpu %r oracle %r" % (p, got, ref)
    # whole x rows and y columns: every x tile seam and every diamond they cross
    checked = count
    for lo, hi in cone.line_boxes(n, T, R, seed=T):
        got = res[lo[2] + R:hi[2] + R, lo[1] + R:hi[1] + R, lo[0] + R:hi[0] + R].cpu().numpy()
        ref = cone.box_values(kind, u0, co, T, R, lo, hi)
        bad = np.argwhere(got != ref)
        assert bad.size == 0, "box %s-%s: %d points differ, first at %s" % (lo, hi, len(bad), bad[0])
        checked += got.size
    print("workload %s: %d sampled points bit-exact" % (w["name"], checked), flush=True)


@pytest.mark.parametrize("windex,dtype,count", [(2, "f64", 10), (3, "f64", 5), (3, "f32", 5),
                                                (4, "f32", 5)])
def test_fullsize_sampled_bitexact(windex, dtype, count):
    w, u0, co, g, bufs, plan, keep = _run_full(windex, dtype)
    _check_samples(w, u0, co, g, bufs, count)
    l2, mx = S.stencil_norms(g, 0)
    u0max = float(np.max(np.abs(u0)))
    assert np.isfinite(l2) and mx <= u0max   # weights are non-negative with sum < 1
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fullsize_25v_sampled_bitexact(dtype):
    """The variable-weight 25-point form of workload 3 (512^3, T = 32, 13
    weight arrays) at full size with the autotuned plan, as the benchmark's
    --kind 25v line runs it: sampled points, whole x rows and y columns."""
    import torch
    w, u0, co, g, bufs, plan, keep = _run_full(3, dtype, kind="25v")
    _check_samples(w, u0, co, g, bufs, 5)
    plan.close()
    del bufs, keep, g
    torch.cuda.empty_cache()


def test_f32_error_subrun_against_f64_oracle():
    """The FP32 precision form on the 256^3 sub-run of the 7-point variable
    workload (T = 100): max-norm error against the FP64 oracle on the same
    FP32-rounded inputs, within the bound T (m + 1) u32 ||u_0|| (m = 13)."""
    import torch
    n, T = (256, 256, 256), 100
    seed = gridgen.seed_for_config(4)
    u0 = gridgen.field(seed, *n, 1, 0.0, 1.0, dtype=np.float32)
    C = gridgen.coeffs_7v(seed, *n, 1, dtype=np.float32)
    print("f32 sub-run 256^3 T=100", flush=True)
    a = torch.from_numpy(u0).cuda()
    b = a.clone()
    g = S.make_grid(a, b, 1, 0)
    cdev = [torch.from_numpy(c).cuda() for c in C]
    plan = S.Plan("7v", "f32", *n)
    plan.run(g, S.make_coeffs("7v", arrays=cdev), T)
    torch.cuda.synchronize()
    got = (a, b)[g.cur].cpu().numpy().astype(np.float64)
    ref, refm1 = oracle.run("7v", u0.astype(np.float64), [c.astype(np.float64) for c in C], T)
    err = float(np.max(np.abs(got - ref)))
    bound = T * 14 * 2.0 ** -24 * float(np.max(u0))
    print("f32 max-norm error %.3e (relative %.3e), bound %.3e" % (err, err / np.max(np.abs(ref)), bound),
          flush=True)
    assert err <= bound
    # the GPU's FP64 residual norms of the FP32 run against the oracle's FP32 run
    r32, r32m1 = oracle.run("7v", u0, C, T)
    l2, mx = S.stencil_norms(g, 1)
    rl2, rmx = onorms.residual_norms(r32, r32m1, 1)
    assert abs(l2 - rl2) <= 1e-12 * rl2 and mx == rmx
    plan.close()


def test_autotuned_plan_on_a_plane_of_4gib_runs_naive():
    """A padded plane of 4 GiB or more (FP32, 32769^2 elements) is beyond the
    MWD tile kernel's 32-bit plane offsets: the autotuner does not time MWD
    on it and the plan runs the naive sweep, whose 64-bit addressing is
    checked bit for bit on whole x rows and y columns (one step: each
    output needs only its neighbours, so the oracle runs on three rows or
    columns of the input with their true neighbours as the fixed boundary).
    About 26 GB of device memory."""
    import torch
    nx = ny = 32767
    nz, R, T = 1, 1, 1
    nxp = nx + 2 * R
    assert nxp * nxp * 4 >= (1 << 32)
    print("plane of 4 GiB: 7c f32 %dx%dx%d, allocating" % (nx, ny, nz), flush=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1410)
    a = torch.empty((nz + 2 * R, nxp, nxp), dtype=torch.float32, device="cuda")
    a.uniform_(-1.0, 1.0, generator=gen)
    b = a.clone()
    g = S.make_grid(a, b, R, 0)
    coeffs = S.make_coeffs("7c", consts=list(gridgen.C7))
    plan = S.Plan("7c", "f32", nx, ny, nz)   # autotuned
    print("plane of 4 GiB: running", flush=True)
    plan.run(g, coeffs, T)
    torch.cuda.synchronize()
    desc = plan.describe()
    print("plane of 4 GiB: schedule", desc, flush=True)
    assert desc["mode"] == S.MODE["naive"]
    assert g.cur == 1
    rng = np.random.default_rng(1410)
    ys = [0, 1, ny // 2, ny - 1, int(rng.integers(ny))]
    xs = [0, nx // 2 - 1, nx - 1, int(rng.integers(nx))]
    checked = 0
    for y in ys:   # interior row y: input rows y - 1 .. y + 1 of every plane
        sub = np.ascontiguousarray(a[:, y:y + 3, :].cpu().numpy())
        ref, _ = oracle.run("7c", sub, gridgen.C7, T, halo=R)
        got = b[R:R + nz, y + R:y + R + 1, R:R + nx].cpu().numpy()
        assert np.array_equal(got, ref[R:R + nz, R:R + 1, R:R + nx]), "row y=%d differs" % y
        checked += got.size
    for x in xs:   # interior column x
        sub = np.ascontiguousarray(a[:, :, x:x + 3].cpu().numpy())
        ref, _ = oracle.run("7c", sub, gridgen.C7, T, halo=R)
        got = b[R:R + nz, R:R + ny, x + R:x + R + 1].cpu().numpy()
        assert np.array_equal(got, ref[R:R + nz, R:R + ny, R:R + 1]), "column x=%d differs" % x
        checked += got.size
    print("plane of 4 GiB: %d points bit-exact" % checked, flush=True)
    plan.close()
    del a, b, g
    torch.cuda.empty_cache()
