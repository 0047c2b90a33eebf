"""GPU: the allocation-free norms entry point (partials in the library's
static device array) against stencil_norms, through the C ABI.  Two calls in
a row, the second on a smaller grid; FP64 and FP32 grids; norms of u and of
the residual."""
from __future__ import annotations

import numpy as np
import pytest

import gridgen
import paper_1410_5561_amd as S
from gpu_util import device_grid

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dts", ["f64", "f32"])
def test_noalloc_norms_match_allocating_norms(dts):
    import torch
    dtype = np.float64 if dts == "f64" else np.float32
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    for n, seed in (((300, 97, 61), 1), ((17, 5, 3), 2)):     # the second call is smaller
        u0 = gridgen.field(seed, *n, 1, -1.0, 1.0, dtype)
        g, bufs = device_grid(u0, 1, 0)
        # a finite u_{T-1} for the residual norms
        bufs[1].copy_(bufs[0] * 0.5)
        for which in (0, 1):
            print("noalloc", dts, n, "which", which, flush=True)
            S.stencil_norms_noalloc(g, which, out.data_ptr())
            torch.cuda.synchronize()
            got = tuple(out.cpu().tolist())
            ref = S.stencil_norms(g, which)
            assert got == ref, "%s %s which=%d: %r vs %r" % (dts, n, which, got, ref)
            assert np.isfinite(got[0]) and got[0] > 0


def test_noalloc_rejects_bad_arguments():
    import ctypes
    g = S.StencilGrid()
    L = S.lib()
    assert L.stencil_norms_noalloc(None, 0, None, None) == -1
    u0 = gridgen.field(3, 8, 8, 8, 1, 0.0, 1.0)
    g, bufs = device_grid(u0, 1, 0)
    assert L.stencil_norms_noalloc(ctypes.byref(g), 0, None, None) == -1
    assert L.stencil_norms_noalloc(ctypes.byref(g), 2, ctypes.c_void_p(bufs[0].data_ptr()), None) == -1
