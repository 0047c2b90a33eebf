"""Python binding of the gfx950 MWD stencil library (argument marshalling only).

Every function here forwards to the C ABI declared in ``include/mwd_stencil.h``
(same names, same semantics) in ``libmwdstencil.so``; the stencil sweeps, the
MWD tiles and the FP64 reductions all run in the library's HIP kernels.
PyTorch provides device memory and streams.  There is no fallback: if the
library is missing, importing the binding's entry points raises.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "KIND", "DTYPE", "MODE", "StencilError", "lib", "lib_path",
    "stencil_create", "stencil_run", "stencil_destroy", "stencil_run_batched",
    "stencil_norms", "stencil_norms_noalloc", "stencil_diff_norms", "stencil_plan_describe",
    "stencil_model_bytes_per_lup", "stencil_model_cache_block", "stencil_strerror", "stencil_last_error",
    "stencil_abi_version", "stencil_profile_enable", "stencil_profile_read",
    "stencil_stream_copy", "stencil_kernel_resources", "Plan", "make_grid", "make_coeffs", "padded_empty", "radius",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libmwdstencil.so")

KIND = {"7c": 0, "7v": 1, "25c": 2, "25v": 3, "mixed": 15}
DTYPE = {"f64": 0, "f32": 1}
MODE = {"auto": 0, "naive": 1, "mwd": 2}
_RADIUS = {"7c": 1, "7v": 1, "25c": 4, "25v": 4}
_NARR = {"7c": 0, "7v": 7, "25c": 0, "25v": 13}


def radius(kind: str) -> int:
    return _RADIUS[kind]


class StencilGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("halo", ctypes.c_int32), ("sy", ctypes.c_int64), ("sz", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("cur", ctypes.c_int32),
                ("buf", ctypes.c_void_p * 2)]


class StencilCoeffs(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("c", ctypes.c_double * 13), ("arr", ctypes.c_void_p * 13)]


class StencilParams(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("dw", ctypes.c_int32), ("lanes", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class StencilPlanDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dtype", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("dw", ctypes.c_int32), ("lanes", ctypes.c_int32), ("xtile", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("rows_per_T", ctypes.c_int32),
                ("model_bytes_per_lup", ctypes.c_double)]


class StencilError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__("%s failed: %s (%d): %s" % (where, _strerror(code), code, detail))
        self.code = code


_lib = None
ABI_VERSION = 1  # the structs below match this version of include/mwd_stencil.h
_SIGS = {
    "stencil_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.POINTER(StencilParams)]),
    "stencil_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(StencilGrid),
                                   ctypes.POINTER(StencilCoeffs), ctypes.c_int32, ctypes.c_void_p]),
    "stencil_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "stencil_run_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(StencilGrid),
                                           ctypes.POINTER(StencilCoeffs), ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_void_p]),
    "stencil_norms": (ctypes.c_int, [ctypes.POINTER(StencilGrid), ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "stencil_diff_norms": (ctypes.c_int, [ctypes.POINTER(StencilGrid), ctypes.POINTER(StencilGrid),
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "stencil_norms_noalloc": (ctypes.c_int, [ctypes.POINTER(StencilGrid), ctypes.c_int32, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "stencil_kernel_resources": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_int32)]),
    "stencil_plan_describe": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(StencilPlanDesc)]),
    "stencil_model_bytes_per_lup": (ctypes.c_double, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "stencil_model_cache_block": (ctypes.c_double, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                    ctypes.c_int32, ctypes.c_int32]),
    "stencil_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "stencil_last_error": (ctypes.c_char_p, []),
    "stencil_abi_version": (ctypes.c_int, []),
    "stencil_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "stencil_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "stencil_stream_copy": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_void_p]),
}


def lib():
    """Load libmwdstencil.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            raise RuntimeError("libmwdstencil.so is missing: build it with "
                               "`python -m paper_1410_5561_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(lib_path)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        if L.stencil_abi_version() != ABI_VERSION:
            raise RuntimeError("libmwdstencil.so has ABI %d, this binding needs %d: rebuild it"
                               % (L.stencil_abi_version(), ABI_VERSION))
        _lib = L
    return _lib


def _strerror(code: int) -> str:
    try:
        return lib().stencil_strerror(code).decode()
    except Exception:
        return "error"


def _check(rc: int, where: str):
    if rc != 0:
        raise StencilError(rc, where, lib().stencil_last_error().decode())


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ---- the C ABI, one Python function per entry point -------------------------

def stencil_abi_version() -> int:
    return lib().stencil_abi_version()


def stencil_strerror(code: int) -> str:
    return lib().stencil_strerror(code).decode()


def stencil_last_error() -> str:
    return lib().stencil_last_error().decode()


def stencil_model_bytes_per_lup(kind: str, dtype: str, dw: int) -> float:
    return lib().stencil_model_bytes_per_lup(KIND[kind], DTYPE[dtype], int(dw))


def stencil_model_cache_block(kind: str, dtype: str, dw: int, lanes: int, nf: int = 1) -> float:
    return lib().stencil_model_cache_block(KIND[kind], DTYPE[dtype], int(dw), int(lanes), int(nf))


def stencil_create(kind: str, dtype: str, nx: int, ny: int, nz: int, mode: str | None = None,
                   dw: int = 0, lanes: int = 0) -> ctypes.c_void_p:
    out = ctypes.c_void_p()
    if mode is None:
        pp = None
    else:
        pp = ctypes.byref(StencilParams(MODE[mode], int(dw), int(lanes), 0))
    _check(lib().stencil_create(ctypes.byref(out), KIND[kind], DTYPE[dtype], nx, ny, nz, pp),
           "stencil_create")
    return out


def stencil_run(plan, grid: StencilGrid, coeffs: StencilCoeffs, T: int, stream=None):
    _check(lib().stencil_run(plan, ctypes.byref(grid), ctypes.byref(coeffs), int(T),
                             _stream_ptr(stream)), "stencil_run")


def stencil_destroy(plan):
    _check(lib().stencil_destroy(plan), "stencil_destroy")


def stencil_run_batched(plan, grids, coeffs, T: int, stream=None):
    n = len(grids)
    ga = (StencilGrid * n)(*grids)
    ca = (StencilCoeffs * n)(*coeffs)
    _check(lib().stencil_run_batched(plan, ga, ca, n, int(T), _stream_ptr(stream)),
           "stencil_run_batched")
    for i in range(n):
        grids[i].cur = ga[i].cur


def stencil_norms(grid: StencilGrid, which: int = 0, stream=None) -> tuple[float, float]:
    out = (ctypes.c_double * 2)()
    _check(lib().stencil_norms(ctypes.byref(grid), int(which), out, _stream_ptr(stream)),
           "stencil_norms")
    return out[0], out[1]


def stencil_norms_noalloc(grid: StencilGrid, which: int, out_dev_ptr: int, stream=None):
    """Asynchronous, allocation-free norms into two doubles of device memory."""
    _check(lib().stencil_norms_noalloc(ctypes.byref(grid), int(which), ctypes.c_void_p(out_dev_ptr),
                                       _stream_ptr(stream)), "stencil_norms_noalloc")


def stencil_diff_norms(a: StencilGrid, b: StencilGrid, stream=None) -> tuple[float, float]:
    out = (ctypes.c_double * 2)()
    _check(lib().stencil_diff_norms(ctypes.byref(a), ctypes.byref(b), out, _stream_ptr(stream)),
           "stencil_diff_norms")
    return out[0], out[1]


def stencil_profile_enable(plan, enable: bool = True):
    _check(lib().stencil_profile_enable(plan, 1 if enable else 0), "stencil_profile_enable")


def stencil_profile_read(plan) -> dict:
    out = (ctypes.c_double * 4)()
    _check(lib().stencil_profile_read(plan, out), "stencil_profile_read")
    return {"main_ms": out[0], "main_launches": int(out[1]),
            "other_ms": out[2], "other_launches": int(out[3])}


def stencil_stream_copy(dst, src, nbytes: int, stream=None):
    _check(lib().stencil_stream_copy(ctypes.c_void_p(dst), ctypes.c_void_p(src), int(nbytes),
                                     _stream_ptr(stream)), "stencil_stream_copy")


def stencil_kernel_resources(kind: str, dtype: str, dw: int, lanes: int) -> dict:
    out = (ctypes.c_int32 * 5)()
    _check(lib().stencil_kernel_resources(KIND[kind], DTYPE[dtype], int(dw), int(lanes), out),
           "stencil_kernel_resources")
    return {"vgprs": out[0], "lds_bytes": out[1], "scratch_bytes_per_lane": out[2],
            "threads": out[3], "workgroups_per_cu": out[4]}


def stencil_plan_describe(plan) -> dict:
    d = StencilPlanDesc()
    _check(lib().stencil_plan_describe(plan, ctypes.byref(d)), "stencil_plan_describe")
    return {f: getattr(d, f) for f, _ in StencilPlanDesc._fields_}


# ---- marshalling helpers ----------------------------------------------------

class Plan:
    """Owning wrapper of a stencil_plan*."""

    def __init__(self, kind: str, dtype: str, nx: int = 0, ny: int = 0, nz: int = 0,
                 mode: str | None = None, dw: int = 0, lanes: int = 0):
        self.kind, self.dtype = kind, dtype
        self.ptr = stencil_create(kind, dtype, nx, ny, nz, mode, dw, lanes)

    def run(self, grid, coeffs, T, stream=None):
        stencil_run(self.ptr, grid, coeffs, T, stream)

    def run_batched(self, grids, coeffs, T, stream=None):
        stencil_run_batched(self.ptr, grids, coeffs, T, stream)

    def describe(self) -> dict:
        return stencil_plan_describe(self.ptr)

    def profile(self, enable: bool = True):
        stencil_profile_enable(self.ptr, enable)

    def profile_read(self) -> dict:
        return stencil_profile_read(self.ptr)

    def close(self):
        if self.ptr:
            stencil_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def padded_empty(nx, ny, nz, halo, dtype, device="cuda"):
    import torch
    td = torch.float64 if dtype in ("f64", torch.float64) else torch.float32
    return torch.empty((nz + 2 * halo, ny + 2 * halo, nx + 2 * halo), dtype=td, device=device)


def make_grid(a, b, halo: int, cur: int = 0, nx: int | None = None, lead: int = 0) -> StencilGrid:
    """Describe two contiguous CUDA tensors of shape (nz + 2h, ny + 2h, W) as a
    stencil_grid (buf[0] = a, buf[1] = b).  Each row holds the padded x extent
    nx + 2h starting at column `lead`; by default nx = W - 2h - lead (rows
    without padding).  sy = W and sz = W (ny + 2h) are the tensors' strides."""
    import torch
    if a.shape != b.shape or a.dtype != b.dtype:
        raise ValueError("both buffers need the same shape and dtype")
    if not (a.is_contiguous() and b.is_contiguous()):
        raise ValueError("buffers must be contiguous")
    if a.dtype not in (torch.float64, torch.float32):
        raise ValueError("dtype must be float64 or float32")
    nzp, nyp, width = a.shape
    if nx is None:
        nx = width - 2 * halo - lead
    if lead < 0 or nx < 1 or lead + nx + 2 * halo > width:
        raise ValueError("rows of %d elements cannot hold %d + 2 x %d from column %d" % (width, nx, halo, lead))
    g = StencilGrid()
    g.nx, g.ny, g.nz, g.halo = nx, nyp - 2 * halo, nzp - 2 * halo, halo
    g.sy, g.sz = a.stride(1), a.stride(0)
    g.dtype = 0 if a.dtype == torch.float64 else 1
    g.cur = cur
    es = a.element_size()
    g.buf[0] = a.data_ptr() + lead * es
    g.buf[1] = b.data_ptr() + lead * es
    return g


def make_coeffs(kind: str, consts=None, arrays=None, lead: int = 0) -> StencilCoeffs:
    """Weights: constants, or CUDA tensors laid out like the grid (rows from
    column `lead`, as in make_grid)."""
    c = StencilCoeffs()
    c.kind = KIND[kind]
    if consts is not None:
        for i, v in enumerate(consts):
            c.c[i] = float(v)
    if arrays is not None:
        if len(arrays) != _NARR[kind]:
            raise ValueError("%s needs %d coefficient arrays" % (kind, _NARR[kind]))
        for i, t in enumerate(arrays):
            c.arr[i] = t.data_ptr() + lead * t.element_size()
    return c
