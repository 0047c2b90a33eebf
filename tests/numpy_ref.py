"""Whole-array NumPy re-evaluation of the sweep, in the listings' operation order.

Used by tests only, as a cross-check of the C oracle's evaluation order: NumPy
ufuncs round every operation and never fuse, so equal order means equal bits.
"""
from __future__ import annotations

import numpy as np

AXES = ((1, 0, 0), (0, 1, 0), (0, 0, 1))


def _sl(h, n, off):
    return slice(h + off, h + off + n)


def sweep(kind, V, coeffs, h):
    nzp, nyp, nxp = V.shape
    nx, ny, nz = nxp - 2 * h, nyp - 2 * h, nzp - 2 * h
    dt = V.dtype

    def nb(dx, dy, dz):
        return V[_sl(h, nz, dz), _sl(h, ny, dy), _sl(h, nx, dx)]

    inner = (slice(h, h + nz), slice(h, h + ny), slice(h, h + nx))
    U = V.copy()
    if kind == "7c":
        c0, c1 = (dt.type(c) for c in coeffs)
        u = c0 * nb(0, 0, 0)
        for (a, b, c) in AXES:
            u = u + c1 * (nb(a, b, c) + nb(-a, -b, -c))
    elif kind == "7v":
        C = [c[inner] for c in coeffs]
        order = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
        u = C[0] * nb(*order[0])
        for m in range(1, 7):
            u = u + C[m] * nb(*order[m])
    else:
        if kind == "25c":
            W = [dt.type(c) for c in coeffs]
        else:
            W = [c[inner] for c in coeffs]
        u = W[0] * nb(0, 0, 0)
        q = 1
        for r in (1, 2, 3, 4):
            for (a, b, c) in AXES:
                u = u + W[q] * (nb(r * a, r * b, r * c) + nb(-r * a, -r * b, -r * c))
                q += 1
    U[inner] = u
    return U


def run(kind, u0, coeffs, T, halo):
    a = u0.copy()
    prev = u0.copy()
    for _ in range(T):
        prev, a = a, sweep(kind, a, coeffs, halo)
    return a, prev
