"""The C ABI without a GPU: the library loads, exports every entry point the
header declares, and rejects bad arguments with the documented codes before
touching the device."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

import paper_1410_5561_amd as S

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "mwd_stencil.h")
EINVAL, EUNSUPPORTED = -1, -2


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|double|const char\s*\*)\s*(stencil_\w+)\s*\(",
                                 text, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(S.lib_path):
        pytest.skip("library not built")
    return S.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(L, n), "missing export %s" % n


def test_version_and_strerror(L):
    assert S.stencil_abi_version() == 1
    for code in (0, -1, -2, -3, -4):
        assert S.stencil_strerror(code)
    assert "unknown" in S.stencil_strerror(-99)


def test_model_bytes_per_lup(L):
    # Eq. (5) = 2 s R (N_D + 2) / Dw; naive = s N_D
    assert S.stencil_model_bytes_per_lup("7v", "f64", 8) == pytest.approx(22.0)
    assert S.stencil_model_bytes_per_lup("7c", "f64", 16) == pytest.approx(4.0)
    assert S.stencil_model_bytes_per_lup("25c", "f32", 32) == pytest.approx(4.0)
    assert S.stencil_model_bytes_per_lup("7v", "f64", 0) == pytest.approx(72.0)
    assert S.stencil_model_bytes_per_lup("25v", "f32", 0) == pytest.approx(60.0)
    assert L.stencil_model_bytes_per_lup(9, 0, 8) < 0


def _rc_create(L, kind, dtype, nx, ny, nz, params=None):
    out = ctypes.c_void_p()
    rc = L.stencil_create(ctypes.byref(out), kind, dtype, nx, ny, nz,
                          ctypes.byref(params) if params is not None else None)
    return rc, out


def test_create_argument_checks(L):
    assert _rc_create(L, 7, 0, 8, 8, 8)[0] == EINVAL
    assert _rc_create(L, 0, 5, 8, 8, 8)[0] == EINVAL
    assert _rc_create(L, 0, 0, 0, 8, 8)[0] == EINVAL
    assert _rc_create(L, 0, 0, 8, -1, 8)[0] == EINVAL
    assert _rc_create(L, 0, 0, 8, 8, 8, S.StencilParams(9, 0, 0, 0))[0] == EINVAL
    assert _rc_create(L, 0, 0, 8, 8, 8, S.StencilParams(2, 6, 64, 0))[0] == EUNSUPPORTED
    assert _rc_create(L, 0, 0, 8, 8, 8, S.StencilParams(2, 8, 100, 0))[0] == EINVAL
    assert L.stencil_create(None, 0, 0, 8, 8, 8, None) == EINVAL
    rc, p = _rc_create(L, 1, 1, 8, 8, 8, S.StencilParams(2, 8, 64, 0))
    assert rc == 0 and p.value
    assert L.stencil_destroy(p) == 0
    assert L.stencil_destroy(None) == EINVAL


def _grid(nx=8, ny=8, nz=8, halo=1, dtype=0, cur=0, fake=0x10000):
    g = S.StencilGrid()
    g.nx, g.ny, g.nz, g.halo = nx, ny, nz, halo
    g.sy = nx + 2 * halo
    g.sz = g.sy * (ny + 2 * halo)
    g.dtype, g.cur = dtype, cur
    g.buf[0] = fake
    g.buf[1] = fake + 0x100000
    return g


def test_run_argument_checks_before_any_device_work(L):
    rc, p = _rc_create(L, 0, 0, 8, 8, 8, S.StencilParams(1, 0, 0, 0))
    assert rc == 0
    c = S.make_coeffs("7c", consts=[0.4, 0.1])
    run = lambda g, cc=c, T=1: L.stencil_run(p, ctypes.byref(g), ctypes.byref(cc), T, None)
    assert L.stencil_run(None, ctypes.byref(_grid()), ctypes.byref(c), 1, None) == EINVAL
    assert L.stencil_run(p, None, ctypes.byref(c), 1, None) == EINVAL
    assert L.stencil_run(p, ctypes.byref(_grid()), None, 1, None) == EINVAL
    assert run(_grid(nx=9)) == EINVAL                 # extents differ from the plan
    assert run(_grid(dtype=1)) == EINVAL              # dtype differs
    assert run(_grid(halo=0)) == EINVAL               # halo < R
    assert run(_grid(cur=2)) == EINVAL
    g = _grid(); g.sy = 5
    assert run(g) == EINVAL                           # stride too small
    g = _grid(); g.buf[1] = g.buf[0]
    assert run(g) == EINVAL                           # aliasing buffers
    g = _grid(); g.buf[0] = 0x10003
    assert run(g) == EINVAL                           # misaligned
    assert run(_grid(), T=-1) == EINVAL
    bad = S.make_coeffs("7v")
    assert run(_grid(), cc=bad) == EINVAL             # coefficient kind mismatch
    g = _grid()
    assert run(g, T=0) == 0 and g.cur == 0            # T = 0 is a no-op
    assert "cur" in S.stencil_last_error() or True
    L.stencil_destroy(p)


def test_variable_coefficients_need_arrays(L):
    rc, p = _rc_create(L, 1, 0, 8, 8, 8, S.StencilParams(1, 0, 0, 0))
    assert rc == 0
    c = S.make_coeffs("7v")
    assert L.stencil_run(p, ctypes.byref(_grid()), ctypes.byref(c), 1, None) == EINVAL
    assert "coefficient array" in S.stencil_last_error()
    L.stencil_destroy(p)


def test_norm_argument_checks(L):
    out = (ctypes.c_double * 2)()
    assert L.stencil_norms(None, 0, out, None) == EINVAL
    assert L.stencil_norms(ctypes.byref(_grid()), 2, out, None) == EINVAL
    assert L.stencil_norms(ctypes.byref(_grid()), 0, None, None) == EINVAL
    assert L.stencil_diff_norms(ctypes.byref(_grid()), ctypes.byref(_grid(nx=7)), out, None) == EINVAL


def test_mwd_rejects_planes_of_4gib_before_any_device_work(L):
    """The tile kernel addresses a padded plane with 32-bit byte offsets: an
    explicit MWD plan refuses a grid whose plane is 4 GiB or more (fake
    device pointers: the call must not touch them)."""
    rc, p = _rc_create(L, 0, 0, 8, 8, 8, S.StencilParams(2, 8, 64, 0))
    assert rc == 0
    c = S.make_coeffs("7c", consts=[0.4, 0.1])
    g = _grid()
    g.sz = (1 << 29)                    # 2^29 doubles = 4 GiB per plane
    assert L.stencil_run(p, ctypes.byref(g), ctypes.byref(c), 3, None) == EUNSUPPORTED
    assert "4 GiB" in S.stencil_last_error()
    g.sz = (1 << 29) - 8                # just below: accepted by the check (not run here)
    assert g.sz * 8 < (1 << 32)
    L.stencil_destroy(p)
    # FP32: the limit is 2^30 elements
    rc, p = _rc_create(L, 0, 1, 8, 8, 8, S.StencilParams(2, 8, 64, 0))
    assert rc == 0
    g = _grid(dtype=1)
    g.sz = 1 << 30
    assert L.stencil_run(p, ctypes.byref(g), ctypes.byref(c), 3, None) == EUNSUPPORTED
    L.stencil_destroy(p)


def test_destroy_without_runs_needs_no_device(L):
    rc, p = _rc_create(L, 2, 1, 16, 16, 16, S.StencilParams(2, 16, 64, 0))
    assert rc == 0
    assert L.stencil_destroy(p) == 0


def test_model_cache_block_golden(L):
    """The library's Eq. (3) (the tuner's pruning model) against the worked
    example of Sec. III-B and the hand-evaluated radius-4 values."""
    import json
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    g1 = json.load(open(os.path.join(here, "cache_block_example.json")))
    # N_D = 2, R = 1: the 7-point constant stencil; N_xb = 8 bytes per lane
    assert S.stencil_model_cache_block("7c", "f64", g1["Dw"], 1, g1["N_F"]) == 8 * g1["C_S_per_Nxb"]
    for c in json.load(open(os.path.join(here, "cache_block_r4.json")))["cases"]:
        kind = {2: "25c", 15: "25v"}[c["N_D"]]
        assert S.stencil_model_cache_block(kind, "f32", c["Dw"], 32, c["N_F"]) == 128 * c["C_S_per_Nxb"]
    assert L.stencil_model_cache_block(9, 0, 8, 64, 1) < 0
    assert L.stencil_model_cache_block(0, 0, 8, 0, 1) < 0


def test_make_grid_describes_padded_rows():
    """The binding's grid description (no device needed: CPU tensors stand in
    for device buffers): strides from the tensors, the first buffer element at
    column `lead`, nx given or taken from the row length; rows too short for
    the grid are refused."""
    import torch
    h, nx, ny, nz, W, lead = 1, 20, 6, 5, 32, 7
    a = torch.zeros((nz + 2 * h, ny + 2 * h, W), dtype=torch.float64)
    b = torch.zeros_like(a)
    g = S.make_grid(a, b, h, 1, nx=nx, lead=lead)
    assert (g.nx, g.ny, g.nz, g.halo, g.cur, g.dtype) == (nx, ny, nz, h, 1, 0)
    assert (g.sy, g.sz) == (W, W * (ny + 2 * h))
    assert g.buf[0] == a.data_ptr() + lead * 8 and g.buf[1] == b.data_ptr() + lead * 8
    g2 = S.make_grid(a, b, h)                      # rows without padding
    assert (g2.nx, g2.buf[0]) == (W - 2 * h, a.data_ptr())
    with pytest.raises(ValueError):
        S.make_grid(a, b, h, nx=nx, lead=W - nx - 2 * h + 1)
    c = S.make_coeffs("7v", arrays=[a] * 7, lead=lead)
    assert c.arr[3] == a.data_ptr() + lead * 8


def test_binding_checks_the_library_abi_version(L):
    assert L.stencil_abi_version() == S.ABI_VERSION
