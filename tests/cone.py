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


def box_values(kind, u0, coeffs, T, halo, lo, hi):
    """Oracle u_T over the interior box [lo, hi) (x, y, z) of the padded grid
    u0, as a (z, y, x) array: one oracle run on the box widened by R*T + R
    per side (clipped to the true halo), as for a single point."""
    R = RADIUS[kind]
    nzp, nyp, nxp = u0.shape
    n = (nxp - 2 * halo, nyp - 2 * halo, nzp - 2 * halo)
    W = R * T + R
    blo = [max(lo[a] - W, -R) for a in range(3)]
    bhi = [min(hi[a] + W, n[a] + R) for a in range(3)]
    sl = tuple(slice(blo[a] + halo, bhi[a] + halo) for a in (2, 1, 0))
    sub = np.ascontiguousarray(u0[sl])
    if kind in ("7c", "25c"):
        co = coeffs
    else:
        co = [np.ascontiguousarray(c[sl]) for c in coeffs]
    uT, _ = oracle.run(kind, sub, co, T, halo=R)
    return uT[lo[2] - blo[2]:hi[2] - blo[2], lo[1] - blo[1]:hi[1] - blo[1], lo[0] - blo[0]:hi[0] - blo[0]]


def line_boxes(n, T, R, seed=0):
    """Boxes of full x rows and full y columns (two points thick in the other
    two axes) at a few positions: every x tile seam and every diamond of the
    rows they cross, near the faces and in the middle."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    ys = [0, ny // 2 - 1, ny - 2, int(rng.integers(2, ny - 4))]
    zs = [0, nz // 2, nz - 2, int(rng.integers(2, nz - 4))]
    xs = [0, nx // 2 + 3, nx - 2]
    boxes = []
    for y0, z0 in zip(ys[:3], zs[:3]):
        boxes.append(((0, y0, z0), (nx, y0 + 2, z0 + 2)))
    for x0, z0 in zip(xs, zs[1:]):
        boxes.append(((x0, 0, z0), (x0 + 2, ny, z0 + 2)))
    return boxes
