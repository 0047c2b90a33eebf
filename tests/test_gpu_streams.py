"""GPU: every call runs in order on the caller's stream.

The inputs reach the grid buffers on a side stream, behind a block of busy
work on that stream.  A run, a batched run or a norm that were not ordered on
that stream would read the buffers before the inputs arrive (or read the
result before it is written) and differ from the oracle.  The first run of
an autotuned plan also tunes (synchronously, on a stream of its own) before
it enqueues the run.
"""
from __future__ import annotations

import numpy as np
import pytest

import gridgen
import oracle
import paper_1410_5561_amd as S
from oracle import norms as onorms

pytestmark = pytest.mark.gpu


def _inputs(kind, n, seed):
    R = gridgen.RADIUS[kind]
    u0 = gridgen.field(seed, *n, R, -1.0, 1.0, np.float64)
    if kind == "7v":
        co = gridgen.coeffs_7v(seed, *n, R)
    else:
        co = gridgen.C7 if kind == "7c" else gridgen.C25
    return u0, co


class _Staged:
    """A grid whose buffers are filled on `stream` only after busy work there:
    buf[0] gets u0 late, buf[1] holds NaN in its interior (and u0's halo)."""

    def __init__(self, kind, u0, co):
        import torch
        R = gridgen.RADIUS[kind]
        self.src = torch.from_numpy(u0).cuda()
        self.a = torch.zeros_like(self.src)
        self.b = self.src.clone()
        self.b[R:-R, R:-R, R:-R] = float("nan")
        if kind == "7v":
            self.cdev = [torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in co]
            self.coeffs = S.make_coeffs(kind, arrays=self.cdev)
        else:
            self.cdev = []
            self.coeffs = S.make_coeffs(kind, consts=list(co))
        self.grid = S.make_grid(self.a, self.b, R, 0)

    def stage(self):
        self.a.copy_(self.src)   # on the current (side) stream


def _busy(big, rounds=24):
    for _ in range(rounds):
        big.mul_(1.0)


@pytest.mark.parametrize("mode,dw,lanes", [("naive", 0, 0), ("mwd", 8, 64), (None, 0, 0)],
                         ids=["naive", "mwd-dw8", "autotuned"])
def test_run_and_norms_on_a_side_stream(mode, dw, lanes):
    import torch
    kind, n, T = "7v", (70, 37, 21), 7
    print("side stream", kind, n, T, mode, flush=True)
    u0, co = _inputs(kind, n, seed=5)
    st = _Staged(kind, u0, co)
    big = torch.ones(1 << 28, device="cuda")   # 1 GiB of busy work per pass
    plan = S.Plan(kind, "f64", *n, mode=mode, dw=dw, lanes=lanes)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        _busy(big)
        st.stage()
        plan.run(st.grid, st.coeffs, T, stream=s)
        l2, mx = S.stencil_norms(st.grid, 1, stream=s)   # residual u_T - u_{T-1}
        got = (st.a, st.b)[st.grid.cur].clone()
        gotm1 = (st.a, st.b)[st.grid.cur ^ 1].clone()
    s.synchronize()
    uT, uTm1 = oracle.run(kind, u0, co, T)
    assert np.array_equal(got.cpu().numpy(), uT)
    assert np.array_equal(gotm1.cpu().numpy(), uTm1)
    rl2, rmx = onorms.residual_norms(uT, uTm1, 1)
    assert abs(l2 - rl2) <= 1e-13 * rl2 and mx == rmx
    plan.close()


def test_batched_run_on_a_side_stream():
    """Two calls with the same grids: the graph is built, captured and
    launched, then replayed; u0 reaches every grid late on the side stream
    before each call (T even: cur stays 0, so the second call replays)."""
    import torch
    specs = [("7c", (40, 33, 20)), ("25c", (50, 37, 18)), ("7v", (45, 20, 13))]
    T = 6
    print("side stream batched", specs, T, flush=True)
    inputs = [_inputs(k, n, seed=60 + i) for i, (k, n) in enumerate(specs)]
    staged = [_Staged(k, u0, co) for (k, _), (u0, co) in zip(specs, inputs)]
    big = torch.ones(1 << 28, device="cuda")
    plan = S.Plan("mixed", "f64")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    for call in (1, 2):
        with torch.cuda.stream(s):
            _busy(big)
            for st in staged:
                st.stage()
            plan.run_batched([st.grid for st in staged], [st.coeffs for st in staged], T, stream=s)
            got = [(st.a, st.b)[st.grid.cur].clone() for st in staged]
        s.synchronize()
        for i, ((kind, n), (u0, co)) in enumerate(zip(specs, inputs)):
            assert staged[i].grid.cur == 0
            uT, _ = oracle.run(kind, u0, co, T)
            assert np.array_equal(got[i].cpu().numpy(), uT), "grid %d (%s %s), call %d" % (i, kind, n, call)
    plan.close()


def test_two_plans_in_flight_on_two_streams():
    """Distinct plans run concurrently on distinct streams: an MWD 7v run and
    an MWD 25c run enqueued on two side streams without synchronizing in
    between, each bit-exact."""
    import torch
    cases = [("7v", (90, 41, 30), 9, 8, 64), ("25c", (60, 48, 36), 5, 16, 64)]
    print("two streams", cases, flush=True)
    work = []
    for i, (kind, n, T, dw, lanes) in enumerate(cases):
        u0, co = _inputs(kind, n, seed=80 + i)
        st = _Staged(kind, u0, co)
        plan = S.Plan(kind, "f64", *n, mode="mwd", dw=dw, lanes=lanes)
        work.append((kind, n, T, u0, co, st, plan, torch.cuda.Stream()))
    big = torch.ones(1 << 28, device="cuda")
    torch.cuda.synchronize()
    for kind, n, T, u0, co, st, plan, s in work:
        with torch.cuda.stream(s):
            _busy(big, rounds=8)
            st.stage()
            plan.run(st.grid, st.coeffs, T, stream=s)
    torch.cuda.synchronize()
    for kind, n, T, u0, co, st, plan, s in work:
        uT, uTm1 = oracle.run(kind, u0, co, T)
        assert np.array_equal((st.a, st.b)[st.grid.cur].cpu().numpy(), uT), kind
        assert np.array_equal((st.a, st.b)[st.grid.cur ^ 1].cpu().numpy(), uTm1), kind
        plan.close()


def test_norms_from_two_host_threads():
    """stencil_norms called from two host threads at once, each on its own
    stream and grid (the library's partials buffer is shared per device and
    held under a lock): every result equals the oracle's."""
    import threading
    import torch
    grids = []
    for i, n in enumerate([(70, 37, 21), (33, 64, 40)]):
        u0, co = _inputs("7c", n, seed=90 + i)
        st = _Staged("7c", u0, co)
        st.stage()
        grids.append((st, onorms.grid_norms(u0, 1)))
    torch.cuda.synchronize()
    errors = []

    def worker(st, ref):
        s = torch.cuda.Stream()
        for _ in range(50):
            l2, mx = S.stencil_norms(st.grid, 0, stream=s)
            if not (abs(l2 - ref[0]) <= 1e-13 * ref[0] and mx == ref[1]):
                errors.append((l2, mx, ref))

    threads = [threading.Thread(target=worker, args=g) for g in grids]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors[:3]
