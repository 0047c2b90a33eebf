"""Helpers for GPU tests: move seeded NumPy inputs to the device, call the
library through its C ABI binding, bring results back."""
from __future__ import annotations

import numpy as np

import paper_1410_5561_amd as S

DT = {np.dtype(np.float64): "f64", np.dtype(np.float32): "f32"}


def to_dev(a, row=None, lead=0):
    """u (padded, plain rows) on the device; with `row`, in rows of `row`
    elements holding u's rows from column `lead`, the rest of each row NaN."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if row is None:
        return t.cuda()
    out = torch.full(a.shape[:2] + (row,), float("nan"), dtype=t.dtype)
    out[:, :, lead:lead + a.shape[2]] = t
    return out.cuda()


def from_dev(t, nxp, row=None, lead=0):
    """The plain padded array back from to_dev's layout; with `row`, checks
    that the padding around each row is still NaN (never written)."""
    h = t.cpu().numpy()
    if row is None:
        return h
    pad = np.concatenate([h[:, :, :lead], h[:, :, lead + nxp:]], axis=2)
    assert np.isnan(pad).all(), "the row padding was written"
    return np.ascontiguousarray(h[:, :, lead:lead + nxp])


def device_grid(u0: np.ndarray, halo: int, cur: int = 0, row=None, lead=0):
    """Two device buffers holding u0 (same halo); buf[cur] is the current level."""
    cur_buf = to_dev(u0, row, lead)
    other = cur_buf.clone()
    # the other buffer gets a NaN interior, so a read of a level that was
    # never written shows up in the result
    h = halo
    nzp, nyp, nxp = u0.shape
    other[h:nzp - h, h:nyp - h, lead + h:lead + nxp - h] = float("nan")
    a, b = (cur_buf, other) if cur == 0 else (other, cur_buf)
    g = S.make_grid(a, b, halo, cur, nx=nxp - 2 * h, lead=lead)
    return g, (a, b)


def device_coeffs(kind: str, co, dtype, row=None, lead=0):
    if kind in ("7c", "25c"):
        return S.make_coeffs(kind, consts=list(co)), []
    arrs = [to_dev(np.asarray(c, dtype=dtype), row, lead) for c in co]
    return S.make_coeffs(kind, arrays=arrs, lead=lead), arrs


def run_gpu(kind, u0, co, T, mode="mwd", dw=0, lanes=0, halo=None, cur=0, plan=None, row=None, lead=0):
    """Run T steps on the GPU; returns (u_T, u_{T-1}) as NumPy arrays.  With
    `row`, the arrays live in rows of `row` elements from column `lead`."""
    import torch
    R = S.radius(kind)
    h = R if halo is None else halo
    g, keep = device_grid(u0, h, cur, row, lead)
    c, ckeep = device_coeffs(kind, co, u0.dtype, row, lead)
    nzp, nyp, nxp = u0.shape
    own = plan is None
    if own:
        plan = S.Plan(kind, DT[np.dtype(u0.dtype)], nxp - 2 * h, nyp - 2 * h, nzp - 2 * h,
                      mode=mode, dw=dw, lanes=lanes)
    plan.run(g, c, T)
    torch.cuda.synchronize()
    bufs = [from_dev(keep[0], nxp, row, lead), from_dev(keep[1], nxp, row, lead)]
    if own:
        plan.close()
    return bufs[g.cur], bufs[g.cur ^ 1]
