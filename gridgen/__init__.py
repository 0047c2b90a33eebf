"""Seeded synthetic inputs, shared by the GPU path, the oracle and the benchmark.

This module draws random numbers and lays them out in padded grids; it holds
none of the stencil arithmetic.  Both sides consume the arrays it returns, so
neither re-generates inputs.

Recipe (the paper's workloads are synthetic grids; there is no dataset):
  * generator: numpy PCG64; the k-th float64 of a stream is the k-th draw of
    ``Generator(PCG64(seed)).random()``; U[a, b) = a + (b - a) * draw;
  * layout: padded row-major [z][y][x], x contiguous, halo of width h >= R on
    every side holding zeros (the fixed Dirichlet boundary);
  * draw order: the field over the interior in C order (z, y, x), then the
    coefficient arrays C0..C6 one after another, each over the interior in C
    order; stream offsets make slab-by-slab generation identical to one pass;
  * 7-point variable weights: c_m ~ U[0.05, 1) for m = 0..6, then per point
    S = ((((((c0+c1)+c2)+c3)+c4)+c5)+c6) and w_m = (0.999 * c_m) / S in FP64;
    25-point variable weights the same way with m = 0..12 (the 25-point
    variable workload: workload 3's grid and field with these 13 arrays);
  * FP32 inputs are round-to-nearest casts of the FP64 values.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 14105561

# Constant weights used by the workloads.
C7 = (0.4, 0.1)  # c0 on the centre, c1 on each of the six neighbours
# 25-point star, radius 4: C00 on the centre, then per radius r = 1..4 one
# weight per axis (x, y, z), applied to both +r and -r neighbours.
C25_RADIAL = (0.04, 0.02, 0.01, 0.00333)
C25 = (0.5,) + tuple(w for w in C25_RADIAL for _axis in range(3))

RADIUS = {"7c": 1, "7v": 1, "25c": 4, "25v": 4}


def padded_shape(nx: int, ny: int, nz: int, halo: int) -> tuple[int, int, int]:
    return (nz + 2 * halo, ny + 2 * halo, nx + 2 * halo)


def zeros(nx: int, ny: int, nz: int, halo: int, dtype=np.float64) -> np.ndarray:
    return np.zeros(padded_shape(nx, ny, nz, halo), dtype=dtype)


def interior(a: np.ndarray, halo: int) -> np.ndarray:
    h = int(halo)
    return a[h:a.shape[0] - h, h:a.shape[1] - h, h:a.shape[2] - h]


def _stream(seed: int, offset: int) -> np.random.Generator:
    bg = np.random.PCG64(seed)
    if offset:
        bg.advance(int(offset))
    return np.random.Generator(bg)


def _workers() -> int:
    import os
    n = len(os.sched_getaffinity(0))
    return max(1, min(16, n))


def _slabs(nz: int, slab: int):
    return [(z0, min(nz, z0 + slab)) for z0 in range(0, nz, slab)]


def _parallel(fn, items):
    """Run fn over items in threads (NumPy's generators release the GIL);
    each slab draws from its own offset of the stream, so the result does
    not depend on the thread count."""
    if len(items) <= 1:
        for it in items:
            fn(it)
        return
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=_workers()) as ex:
        list(ex.map(fn, items))


def uniform_into(out: np.ndarray, seed: int, offset: int, lo: float, hi: float,
                 slab: int = 16) -> None:
    """Fill ``out`` (shape (nz, ny, nx), any float dtype) with U[lo, hi) draws
    number offset, offset+1, ... of stream ``seed`` in C order, slab by slab."""
    nz, ny, nx = out.shape
    plane = ny * nx

    def one(zz):
        z0, z1 = zz
        g = _stream(seed, offset + z0 * plane)
        d = g.random((z1 - z0) * plane).reshape(z1 - z0, ny, nx)
        out[z0:z1] = lo + (hi - lo) * d

    _parallel(one, _slabs(nz, slab))


def field(seed: int, nx: int, ny: int, nz: int, halo: int, lo: float, hi: float,
          dtype=np.float64, out: np.ndarray | None = None) -> np.ndarray:
    """Padded grid: zero halo, interior U[lo, hi) from stream ``seed`` at offset 0."""
    a = zeros(nx, ny, nz, halo, dtype) if out is None else out
    if out is not None:
        a[...] = 0
    uniform_into(interior(a, halo), seed, 0, lo, hi)
    return a


def coeffs_var(seed: int, nx: int, ny: int, nz: int, halo: int, count: int, dtype=np.float64,
               total: float = 0.999, outs=None, slab: int = 8) -> list[np.ndarray]:
    """``count`` padded weight arrays C0..C{count-1} of a variable stencil.

    Raw weights come after the field in the same stream (C_m at offset
    (1 + m) * n_interior); each point's weights are scaled to sum to
    ``total`` (up to rounding) as described in the module docstring.
    """
    n = nx * ny * nz
    plane = nx * ny
    arrs = outs if outs is not None else [zeros(nx, ny, nz, halo, dtype) for _ in range(count)]
    for a in arrs:
        a[...] = 0
    views = [interior(a, halo) for a in arrs]

    def one(zz):
        z0, z1 = zz
        cnt = (z1 - z0) * plane
        raw = []
        for m in range(count):
            g = _stream(seed, (1 + m) * n + z0 * plane)
            raw.append((0.05 + 0.95 * g.random(cnt)).reshape(z1 - z0, ny, nx))
        s = raw[0] + raw[1]
        for m in range(2, count):
            s = s + raw[m]
        for m in range(count):
            views[m][z0:z1] = (total * raw[m]) / s

    _parallel(one, _slabs(nz, slab))
    return arrs


def coeffs_7v(seed: int, nx: int, ny: int, nz: int, halo: int, dtype=np.float64,
              total: float = 0.999, outs=None, slab: int = 8) -> list[np.ndarray]:
    """Seven padded weight arrays C0..C6 of the 7-point variable stencil."""
    return coeffs_var(seed, nx, ny, nz, halo, 7, dtype, total, outs, slab)


def coeffs_25v(seed: int, nx: int, ny: int, nz: int, halo: int, dtype=np.float64,
               total: float = 0.999, outs=None, slab: int = 8) -> list[np.ndarray]:
    """Thirteen padded weight arrays C00, C01..C12 of the 25-point variable
    stencil (Listing 3's order), drawn and scaled like the 7-point ones."""
    return coeffs_var(seed, nx, ny, nz, halo, 13, dtype, total, outs, slab)


def seed_for_config(index: int) -> int:
    """Seed of workload ``index`` (1-based, in the order listed by ``workloads``)."""
    return SEED_BASE + int(index)


def workloads() -> dict:
    """The five workloads: sizes are interior extents (nx, ny, nz)."""
    return {
        1: dict(name="7c-f64-64^3-T8", kind="7c", dtype="f64", n=(64, 64, 64), T=8,
                field=(0.0, 1.0), coeffs=C7),
        2: dict(name="7v-f64-512^3-T64", kind="7v", dtype="f64", n=(512, 512, 512), T=64,
                field=(0.0, 1.0), coeffs="7v"),
        3: dict(name="25c-512^3-T32", kind="25c", dtype=("f64", "f32"), n=(512, 512, 512),
                T=32, field=(-1.0, 1.0), coeffs=C25),
        4: dict(name="7v-f32-1024x1024x512-T100", kind="7v", dtype="f32",
                n=(1024, 1024, 512), T=100, field=(0.0, 1.0), coeffs="7v",
                error_subrun=(256, 256, 256)),
        5: dict(name="batch-256-mixed-f32-T16", kind="batch", dtype="f32", T=16,
                count=256, sides=tuple(range(32, 257, 16))),
    }


def batch_specs(seed: int | None = None, count: int = 256, sides=None) -> list[dict]:
    """Grid list of the batched workload.

    Sides are drawn per axis, uniformly from {32, 48, ..., 256}, as one
    (count, 3) integer draw of stream ``seed``; even-indexed grids are
    7-point constant (field U[0,1), halo 1), odd-indexed grids are 25-point
    constant (field U[-1,1), halo 4).  Grid g's field comes from its own
    stream seeded with SeedSequence([seed, g]).
    """
    seed = seed_for_config(5) if seed is None else seed
    sides = tuple(range(32, 257, 16)) if sides is None else tuple(sides)
    g = np.random.Generator(np.random.PCG64(seed))
    idx = g.integers(0, len(sides), size=(count, 3))
    out = []
    for k in range(count):
        nx, ny, nz = (sides[i] for i in idx[k])
        kind = "7c" if k % 2 == 0 else "25c"
        out.append(dict(index=k, kind=kind, n=(int(nx), int(ny), int(nz)),
                        halo=RADIUS[kind], field=(0.0, 1.0) if kind == "7c" else (-1.0, 1.0),
                        coeffs=C7 if kind == "7c" else C25,
                        seed=np.random.SeedSequence([seed, k])))
    return out


def batch_field(spec: dict, dtype=np.float32) -> np.ndarray:
    nx, ny, nz = spec["n"]
    h = spec["halo"]
    a = zeros(nx, ny, nz, h, dtype)
    g = np.random.Generator(np.random.PCG64(spec["seed"]))
    lo, hi = spec["field"]
    interior(a, h)[...] = lo + (hi - lo) * g.random((nz, ny, nx))
    return a
