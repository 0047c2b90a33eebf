"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar: bit-exact.  The kernels evaluate each update in the listings' order with
separately rounded operations, like the oracle, so FP64 and FP32 results are
identical to the oracle run in the same precision; the FP32 form is also
held to a stated error bound against the FP64 oracle.
"""
from __future__ import annotations

import numpy as np
import pytest

import gridgen
import oracle
from gpu_util import run_gpu

pytestmark = pytest.mark.gpu


def _inputs(kind, n, dtype, seed=11):
    R = gridgen.RADIUS[kind]
    u0 = gridgen.field(seed, *n, R, -1.0, 1.0, dtype)
    if kind == "7c":
        co = gridgen.C7
    elif kind == "25c":
        co = gridgen.C25
    elif kind == "7v":
        co = [c.astype(dtype) for c in gridgen.coeffs_7v(seed, *n, R)]
    else:
        rng = np.random.default_rng(seed)
        co = [rng.uniform(0, 0.07, size=u0.shape).astype(dtype) for _ in range(13)]
    return u0, co


def _check(kind, u0, co, T, got_T, got_Tm1):
    uT, uTm1 = oracle.run(kind, u0, co, T)
    assert np.array_equal(got_T, uT), "u_T differs: max |d| = %g" % np.nanmax(np.abs(got_T - uT))
    if T > 0:
        assert np.array_equal(got_Tm1, uTm1), "u_{T-1} differs"


KINDS = ["7c", "7v", "25c", "25v"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_naive_bitexact(kind, dtype):
    n = (70, 37, 21)   # two x blocks, ragged y and z; z chunks of 2 planes
    print("naive", kind, np.dtype(dtype).name, n, flush=True)
    u0, co = _inputs(kind, n, dtype)
    got = run_gpu(kind, u0, co, 5, mode="naive")
    _check(kind, u0, co, 5, *got)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_naive_bitexact_z_chunks(kind, dtype):
    # several z chunks of the naive block (the launch halves its 64 or 128
    # planes per block until it has two workgroups per CU: 8 or 16 here),
    # each with its steady-state plane loop, and a ragged last chunk; two y
    # blocks even where a block holds several rows per thread
    n = (70, 75, 300)
    print("naive z chunks", kind, np.dtype(dtype).name, n, flush=True)
    u0, co = _inputs(kind, n, dtype)
    got = run_gpu(kind, u0, co, 3, mode="naive")
    _check(kind, u0, co, 3, *got)


# every compiled (diamond width, x lanes) shape
MWD_SHAPES = {
    ("7c", "f64"): [(4, 64), (4, 128), (4, 256), (8, 64), (8, 128)],
    ("7c", "f32"): [(4, 64), (4, 128), (4, 256), (8, 64), (8, 128), (16, 64)],
    ("7v", "f64"): [(4, 64), (4, 128), (4, 256), (8, 64), (8, 128)],
    ("7v", "f32"): [(4, 64), (4, 128), (4, 256), (8, 64), (8, 128), (10, 64), (16, 64)],
    ("25c", "f64"): [(8, 64), (8, 128), (16, 64)],
    ("25c", "f32"): [(8, 64), (8, 128), (16, 64)],
    ("25v", "f64"): [(8, 64), (8, 128), (16, 64)],
    ("25v", "f32"): [(8, 64), (8, 128), (16, 64)],
}
MWD_CASES = [(k, d, dw, lx) for (k, d), shapes in MWD_SHAPES.items() for (dw, lx) in shapes]


@pytest.mark.parametrize("case", MWD_CASES, ids=lambda c: "%s-%s-dw%d-lx%d" % c)
def test_mwd_bitexact(case):
    kind, dts, dw, lanes = case
    dtype = np.float64 if dts == "f64" else np.float32
    # several x tiles with a ragged last one, several diamonds per row with
    # half diamonds at both y edges, many rows
    n = (150, 45, 19) if kind in ("7c", "7v") else (140, 53, 17)
    if lanes == 256:
        n = (530, 45, 19)   # several 256-lane x tiles and a ragged one
    T = 13 if kind in ("7c", "7v") else 7
    print("mwd", case, n, T, flush=True)
    u0, co = _inputs(kind, n, dtype)
    got = run_gpu(kind, u0, co, T, mode="mwd", dw=dw, lanes=lanes)
    _check(kind, u0, co, T, *got)


@pytest.mark.parametrize("case", MWD_CASES, ids=lambda c: "%s-%s-dw%d-lx%d" % c)
def test_mwd_bitexact_steady_state(case):
    """Deep enough in z that the tile runs several chunks of its steady-state
    step body (every plane inside the domain) between the checked boundary
    steps, wide enough in x and y that some tiles have no lane outside the
    domain and others straddle each edge."""
    kind, dts, dw, lanes = case
    dtype = np.float64 if dts == "f64" else np.float32
    n = (160, 40, 70) if kind in ("7c", "7v") else (150, 60, 70)
    if lanes == 256:
        n = (600, 40, 70)
    T = 6
    print("mwd steady", case, n, T, flush=True)
    u0, co = _inputs(kind, n, dtype, seed=23)
    got = run_gpu(kind, u0, co, T, mode="mwd", dw=dw, lanes=lanes)
    _check(kind, u0, co, T, *got)


@pytest.mark.parametrize("case", [("7c", np.float64, "naive", 0, 0, 5), ("7c", np.float64, "naive", 0, 0, 4),
                                  ("7v", np.float32, "mwd", 8, 64, 5), ("25c", np.float64, "mwd", 16, 64, 6),
                                  ("25c", np.float32, "naive", 0, 0, 3)],
                         ids=lambda c: "%s-%s-%s-dw%d-T%d" % (c[0], np.dtype(c[1]).name, c[2], c[3], c[5]))
def test_repeated_runs(case):
    """One plan run four times in a row on the same grid, with other device
    work between the calls: after call k the grid holds u_{kT} and
    u_{kT-1}, bit-exact (cur flips with odd T; MWD scratch is reused)."""
    import torch
    import paper_1410_5561_amd as S
    from gpu_util import device_grid, device_coeffs
    kind, dtype, mode, dw, lanes, T = case
    n = (70, 45, 40)
    R = gridgen.RADIUS[kind]
    print("repeated runs", case, flush=True)
    u0, co = _inputs(kind, n, dtype, seed=41)
    g, keep = device_grid(u0, R, 0)
    c, ckeep = device_coeffs(kind, co, dtype)
    plan = S.Plan(kind, "f64" if dtype == np.float64 else "f32", *n, mode=mode, dw=dw, lanes=lanes)
    other = torch.rand(1 << 20, device="cuda")
    try:
        for k in range(1, 5):
            plan.run(g, c, T)
            other.mul_(0.5).add_(1.0)          # other work on the stream between the calls
            S.stencil_norms(g, 0)              # a synchronising library call
            torch.cuda.synchronize()
            got = keep[g.cur].cpu().numpy()
            gotm1 = keep[g.cur ^ 1].cpu().numpy()
            uT, uTm1 = oracle.run(kind, u0, co, k * T)
            assert np.array_equal(got, uT), "call %d" % k
            assert np.array_equal(gotm1, uTm1), "call %d u_{T-1}" % k
    finally:
        plan.close()


# Rows longer than the padded x extent (sy > nx + 2h), the grid starting at a
# column `lead` of each row, the rest of every row NaN: nothing outside the
# padded grid is read (a NaN would reach the results) or written (checked).
# (kind, dtype, mode, dw, lanes, n, row, lead)
PADDED_ROW_CASES = [
    ("7v", np.float64, "mwd", 8, 64, (90, 37, 21), 112, 6),
    ("7v", np.float64, "mwd", 8, 64, (140, 40, 70), 160, 11),   # steady-state step body
    ("7v", np.float32, "mwd", 8, 64, (140, 40, 21), 160, 3),
    ("25c", np.float64, "mwd", 16, 64, (60, 40, 30), 80, 8),
    ("7c", np.float64, "mwd", 4, 128, (200, 30, 20), 224, 1),
    ("25c", np.float32, "naive", 0, 0, (70, 75, 140), 96, 5),
    ("7v", np.float64, "naive", 0, 0, (70, 37, 70), 80, 7),
]


@pytest.mark.parametrize("case", PADDED_ROW_CASES,
                         ids=lambda c: "%s-%s-%s-dw%d-lx%d-%s-row%d-lead%d" % (
                             c[0], np.dtype(c[1]).name, c[2], c[3], c[4], "x".join(map(str, c[5])), c[6], c[7]))
def test_padded_rows(case):
    kind, dtype, mode, dw, lanes, n, row, lead = case
    T = 5
    print("padded rows", case, flush=True)
    u0, co = _inputs(kind, n, dtype, seed=29)
    got = run_gpu(kind, u0, co, T, mode=mode, dw=dw, lanes=lanes, row=row, lead=lead)
    _check(kind, u0, co, T, *got)


@pytest.mark.parametrize("case", [("7v", np.float64, 8, 64, (512, 200, 24), 12),
                                  ("7c", np.float32, 8, 64, (512, 400, 16), 10),
                                  ("25c", np.float64, 16, 64, (512, 400, 20), 8)],
                         ids=lambda c: "%s-%s-dw%d-%s" % (c[0], np.dtype(c[1]).name, c[2], "x".join(map(str, c[4]))))
def test_mwd_rows_larger_than_the_gpu(case):
    """Diamond rows with more tiles than the GPU holds at once (several
    rounds of workgroups per row launch)."""
    kind, dtype, dw, lanes, n, T = case
    print("mwd large rows", kind, np.dtype(dtype).name, dw, lanes, n, T, flush=True)
    u0, co = _inputs(kind, n, dtype, seed=31)
    got = run_gpu(kind, u0, co, T, mode="mwd", dw=dw, lanes=lanes)
    _check(kind, u0, co, T, *got)


@pytest.mark.parametrize("T", [0, 1, 2, 3, 4, 5, 8, 9])
@pytest.mark.parametrize("cur", [0, 1])
def test_mwd_step_counts_and_cur(T, cur):
    """Clipping at t = T for every T mod h, and a run starting from buffer 1."""
    n = (77, 30, 12)
    print("mwd T", T, "cur", cur, flush=True)
    u0, co = _inputs("7c", n, np.float64, seed=T + 3)
    got = run_gpu("7c", u0, co, T, mode="mwd", dw=8, lanes=64, cur=cur)
    uT, uTm1 = oracle.run("7c", u0, co, T)
    assert np.array_equal(got[0], uT)
    if T > 0:
        assert np.array_equal(got[1], uTm1)


@pytest.mark.parametrize("n", [(1, 1, 1), (3, 2, 1), (1, 9, 4), (64, 1, 3), (200, 5, 2)])
def test_mwd_degenerate_extents(n):
    print("mwd degenerate", n, flush=True)
    for kind in ("7c", "25c"):
        u0, co = _inputs(kind, n, np.float64)
        dw = 8 if kind == "7c" else 16
        got = run_gpu(kind, u0, co, 6, mode="mwd", dw=dw, lanes=64)
        _check(kind, u0, co, 6, *got)
        got = run_gpu(kind, u0, co, 6, mode="naive")
        _check(kind, u0, co, 6, *got)


def test_wider_halo_than_radius():
    n = (40, 20, 10)
    print("halo 3 for 7v", flush=True)
    u0 = gridgen.field(2, *n, 3, 0.0, 1.0)
    u0[0:3, :, :] = 0.25   # non-zero boundary values
    u0[:, :, -3:] = -0.5
    co = gridgen.coeffs_7v(2, *n, 3)
    for mode in ("naive", "mwd"):
        got = run_gpu("7v", u0, co, 9, mode=mode, dw=8, lanes=64, halo=3)
        uT, uTm1 = oracle.run("7v", u0, co, 9, halo=3)
        assert np.array_equal(got[0], uT) and np.array_equal(got[1], uTm1)


def test_workload1_7c_64cube_both_modes():
    """The small 7-point workload: 64^3, T = 8, c0 = 0.4, c1 = 0.1, U[0,1)."""
    w = gridgen.workloads()[1]
    print("workload 1", flush=True)
    u0 = gridgen.field(gridgen.seed_for_config(1), *w["n"], 1, *w["field"])
    for mode, dw, lanes in (("naive", 0, 0), ("mwd", 8, 64), ("mwd", 8, 128), ("mwd", 4, 128)):
        got = run_gpu("7c", u0, w["coeffs"], w["T"], mode=mode, dw=dw, lanes=lanes)
        _check("7c", u0, w["coeffs"], w["T"], *got)


def test_f32_against_f64_oracle_bound():
    """FP32 form vs the FP64 oracle on the same (FP32-rounded) inputs:
    ||e_T|| <= T (m + 1) u32 ||u_0|| for non-negative weights summing to <= 1."""
    n = (96, 64, 32)
    T = 20
    print("f32 bound", flush=True)
    u0 = gridgen.field(4, *n, 1, 0.0, 1.0).astype(np.float32)
    C = [c.astype(np.float32) for c in gridgen.coeffs_7v(4, *n, 1)]
    got, _ = run_gpu("7v", u0, C, T, mode="mwd", dw=8, lanes=128)
    ref, _ = oracle.run("7v", u0.astype(np.float64), [c.astype(np.float64) for c in C], T)
    err = np.max(np.abs(got.astype(np.float64) - ref))
    assert err <= T * 14 * 2.0 ** -24 * float(np.max(u0))


@pytest.mark.parametrize("case", [("7c", (1, 2, 70000), 5), ("25c", (3, 1, 66000), 3),
                                  ("7c", (2, 270000, 2), 4)],
                         ids=["7c-nz70000", "25c-nz66000", "7c-ny270000"])
def test_extents_beyond_the_launch_grid_limit(case):
    """z or y extents above 65535 (the y/z limit of a launch grid): the MWD
    gather and boundary fill stride over their launch, the naive sweep uses a
    one-dimensional grid."""
    kind, n, T = case
    print("large extent", kind, n, T, flush=True)
    u0, co = _inputs(kind, n, np.float64, seed=41)
    dw = 8 if kind == "7c" else 16
    got = run_gpu(kind, u0, co, T, mode="mwd", dw=dw, lanes=64)
    _check(kind, u0, co, T, *got)
    got = run_gpu(kind, u0, co, T, mode="naive")
    _check(kind, u0, co, T, *got)


def _random_cases(count=24, seed=1410):
    """Seeded random draws over the whole parameter space: kind, dtype,
    schedule (naive or any compiled MWD shape), extents (1..150 in x, 1..90
    in y, 1..80 in z), T (0..15), halo (R or R + 1..3), starting buffer, and
    rows padded beyond the grid.  Sizes stay small enough for the oracle."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = KINDS[rng.integers(len(KINDS))]
        dts = ("f64", "f32")[rng.integers(2)]
        shapes = [(0, 0)] + MWD_SHAPES[(kind, dts)]
        dw, lanes = shapes[rng.integers(len(shapes))]
        n = (int(rng.integers(1, 151)), int(rng.integers(1, 91)), int(rng.integers(1, 81)))
        if lanes == 256:
            n = (int(rng.integers(200, 600)),) + n[1:]
        T = int(rng.integers(0, 16))
        R = gridgen.RADIUS[kind]
        halo = R + (int(rng.integers(1, 4)) if rng.random() < 0.3 else 0)
        cur = int(rng.integers(2))
        pad = int(rng.integers(0, 20)) if rng.random() < 0.3 else 0
        out.append((i, kind, dts, dw, lanes, n, T, halo, cur, pad))
    return out


@pytest.mark.parametrize("case", _random_cases(), ids=lambda c: "r%d-%s-%s-dw%d-lx%d-%s-T%d-h%d-c%d-p%d" % (
    c[0], c[1], c[2], c[3], c[4], "x".join(map(str, c[5])), c[6], c[7], c[8], c[9]))
def test_random_cases(case):
    i, kind, dts, dw, lanes, n, T, halo, cur, pad = case
    dtype = np.float64 if dts == "f64" else np.float32
    print("random case", case, flush=True)
    R = gridgen.RADIUS[kind]
    u0 = gridgen.field(500 + i, *n, halo, -1.0, 1.0, dtype)
    if kind == "7c":
        co = gridgen.C7
    elif kind == "25c":
        co = gridgen.C25
    elif kind == "7v":
        co = [c.astype(dtype) for c in gridgen.coeffs_7v(500 + i, *n, halo)]
    else:
        co = [c.astype(dtype) for c in gridgen.coeffs_25v(500 + i, *n, halo)]
    mode = "naive" if dw == 0 else "mwd"
    row = u0.shape[2] + pad if pad else None
    got = run_gpu(kind, u0, co, T, mode=mode, dw=dw, lanes=lanes, halo=halo, cur=cur, row=row, lead=pad // 2)
    uT, uTm1 = oracle.run(kind, u0, co, T, halo=halo)
    assert np.array_equal(got[0], uT), "u_T differs"
    if T > 0:
        assert np.array_equal(got[1], uTm1), "u_{T-1} differs"
