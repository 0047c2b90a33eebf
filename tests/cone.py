"""Sampled parity for full-size runs: the oracle recomputes single outputs.

u_T at a point depends only on the inputs within R*T (per axis) of it.  The
oracle therefore runs on the sub-box that reaches R*T + R beyond the point
(clipped to the true halo, which is fixed), whose outer R layers act as a
fixed boundary: a fixed layer perturbs a neighbour within R per step, so
after T steps the point, R*T away from every artificial face, is exact.
"""
from __future__ import annotations

import numpy as np

import oracle

RADIUS = {"7c": 1, "7v": 1, "25c": 4, "25v": 4}


def subbox_value(kind, u0, coeffs, T, halo, p):
    """Oracle u_T at interior point p = (x, y, z) of the padded grid u0."""
    R = RADIUS[kind]
    nzp, nyp, nxp = u0.shape
    n = (nxp - 2 * halo, nyp - 2 * halo, nzp - 2 * halo)
    W = R * T + R
    lo = [max(p[a] - W, -R) for a in range(3)]
    hi = [min(p[a] + W + 1, n[a] + R) for a in range(3)]
    sl = tuple(slice(lo[a] + halo, hi[a] + halo) for a in (2, 1, 0))
    sub = np.ascontiguousarray(u0[sl])
    if kind in ("7c", "25c"):
        co = coeffs
    else:
        co = [np.ascontiguousarray(c[sl]) for c in coeffs]
    uT, _ = oracle.run(kind, sub, co, T, halo=R)
    return uT[p[2] - lo[2], p[1] - lo[1], p[0] - lo[0]]


def sample_points(n, count, seed=0):
    """Corners, face centres near the boundary, and random interior points."""
    nx, ny, nz = n
    pts = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (0, ny - 1, nz // 2), (nx // 2, 0, nz - 1),
           (nx - 1, ny // 2, 0), (nx // 2, ny // 2, nz // 2)]
    rng = np.random.default_rng(seed)
    while len(pts) < count:
        pts.append((int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))))
    return pts[:count]
