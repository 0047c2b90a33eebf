"""CPU oracle for the repeated stencil sweeps of Sec. I (Listings 1-3).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library and never imports it.

``run`` wraps the plain C two-array sweep in ``stencil_oracle.c``;
``models`` restates the cache-block and code-balance models (Eqs. 2-5);
``norms`` gives the FP64 reductions the GPU reports.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "stencil_oracle.c"), os.path.join(HERE, "oracle_body.h")]

KINDS = {"7c": 0, "7v": 1, "25c": 2, "25v": 3}
RADIUS = {"7c": 1, "7v": 1, "25c": 4, "25v": 4}
N_COEF_ARRAYS = {"7v": 7, "25v": 13}
N_CONST = {"7c": 2, "25c": 13}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc: -O2, OpenMP, no FP contraction."""
    newest_src = max(os.path.getmtime(s) for s in SOURCES)
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= newest_src:
        return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", SOURCES[0], "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_libs: dict = {}


def _load(path: str | None = None):
    """Load the oracle library (default: the one built from this directory).

    Tests that plant mistakes in a copy of the oracle pass that copy's path."""
    key = path or LIB_PATH
    if key not in _libs:
        if path is None:
            build()
        lib = ctypes.CDLL(key)
        for name in ("oracle_run_f64", "oracle_run_f32"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                           ctypes.c_longlong, ctypes.c_longlong,
                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_int, ctypes.c_int]
        _libs[key] = lib
    return _libs[key]


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


def run(kind: str, u0: np.ndarray, coeffs, T: int, halo: int | None = None,
        threads: int | None = None, lib_path: str | None = None):
    """Apply T sweeps of stencil ``kind`` to the padded grid ``u0``.

    ``u0`` is a C-contiguous float64 or float32 array of shape
    (nz+2h, ny+2h, nx+2h) whose halo holds the fixed (Dirichlet) boundary
    values.  ``coeffs`` is a sequence of constants (7c: c0, c1; 25c: C00..C12)
    or a list of padded coefficient arrays of the same dtype (7v: C0..C6;
    25v: C00..C12).  Returns (u_T, u_{T-1}); for T == 0 both are u_0.
    """
    lib = _load(lib_path)
    if kind not in KINDS:
        raise ValueError("unknown stencil kind %r" % kind)
    dt = np.dtype(u0.dtype)
    if dt not in (np.float64, np.float32):
        raise TypeError("oracle works in float64 or float32")
    R = RADIUS[kind]
    h = R if halo is None else int(halo)
    nzp, nyp, nxp = u0.shape
    nx, ny, nz = nxp - 2 * h, nyp - 2 * h, nzp - 2 * h
    a = np.ascontiguousarray(u0).copy()
    b = a.copy()
    keep = []
    cptr = None
    Cptr = None
    if kind in N_CONST:
        cs = np.ascontiguousarray(np.asarray(coeffs, dtype=dt))
        if cs.shape != (N_CONST[kind],):
            raise ValueError("%s needs %d constants" % (kind, N_CONST[kind]))
        keep.append(cs)
        cptr = cs.ctypes.data
    else:
        arrs = [np.ascontiguousarray(c, dtype=dt) for c in coeffs]
        if len(arrs) != N_COEF_ARRAYS[kind] or any(c.shape != a.shape for c in arrs):
            raise ValueError("%s needs %d coefficient arrays shaped like the grid"
                             % (kind, N_COEF_ARRAYS[kind]))
        keep.extend(arrs)
        table = (ctypes.c_void_p * len(arrs))(*[c.ctypes.data for c in arrs])
        keep.append(table)
        Cptr = ctypes.addressof(table)
    fn = lib.oracle_run_f64 if dt == np.float64 else lib.oracle_run_f32
    nt = default_threads() if threads is None else int(threads)
    r = fn(KINDS[kind], nx, ny, nz, h, nxp, nxp * nyp, a.ctypes.data, b.ctypes.data,
           cptr, Cptr, int(T), nt)
    if r < 0:
        raise ValueError("oracle rejected the arguments")
    if T == 0:
        return a, a.copy()
    return (a, b) if r == 0 else (b, a)
