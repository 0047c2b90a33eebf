"""Helpers for GPU tests: move seeded NumPy inputs to the device, call the
library through its C ABI binding, bring results back."""
from __future__ import annotations

import numpy as np

import paper_1410_5561_amd as S

DT = {np.dtype(np.float64): "f64", np.dtype(np.float32): "f32"}


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def device_grid(u0: np.ndarray, halo: int, cur: int = 0):
    """Two device buffers holding u0 (same halo); buf[cur] is the current level."""
    import torch
    cur_buf = to_dev(u0)
    other = cur_buf.clone()
    # the other buffer gets a NaN interior, so a read of a level that was
    # never written shows up in the result
    h = halo
    other[h:other.shape[0] - h, h:other.shape[1] - h, h:other.shape[2] - h] = float("nan")
    a, b = (cur_buf, other) if cur == 0 else (other, cur_buf)
    g = S.make_grid(a, b, halo, cur)
    return g, (a, b)


def device_coeffs(kind: str, co, dtype):
    if kind in ("7c", "25c"):
        return S.make_coeffs(kind, consts=list(co)), []
    arrs = [to_dev(np.asarray(c, dtype=dtype)) for c in co]
    return S.make_coeffs(kind, arrays=arrs), arrs


def run_gpu(kind, u0, co, T, mode="mwd", dw=0, lanes=0, halo=None, cur=0, plan=None):
    """Run T steps on the GPU; returns (u_T, u_{T-1}) as NumPy arrays."""
    import torch
    R = S.radius(kind)
    h = R if halo is None else halo
    g, keep = device_grid(u0, h, cur)
    c, ckeep = device_coeffs(kind, co, u0.dtype)
    nzp, nyp, nxp = u0.shape
    own = plan is None
    if own:
        plan = S.Plan(kind, DT[np.dtype(u0.dtype)], nxp - 2 * h, nyp - 2 * h, nzp - 2 * h,
                      mode=mode, dw=dw, lanes=lanes)
    plan.run(g, c, T)
    torch.cuda.synchronize()
    bufs = [keep[0].cpu().numpy(), keep[1].cpu().numpy()]
    if own:
        plan.close()
    return bufs[g.cur], bufs[g.cur ^ 1]
