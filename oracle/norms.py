"""FP64 reductions over the interior of a padded grid, written plainly.

TEST INFRASTRUCTURE ONLY.  Sums use math.fsum, i.e. the exactly rounded sum
of the (individually rounded) FP64 squares, so the only rounding left is in
the squares and the final square root.
"""
from __future__ import annotations

import math

import numpy as np


def interior(a: np.ndarray, halo: int) -> np.ndarray:
    h = int(halo)
    return a[h:a.shape[0] - h, h:a.shape[1] - h, h:a.shape[2] - h]


def l2_max(x: np.ndarray) -> tuple[float, float]:
    """(sqrt(sum x^2), max |x|) with x taken in float64."""
    v = np.asarray(x, dtype=np.float64).ravel()
    if v.size == 0:
        return 0.0, 0.0
    return math.sqrt(math.fsum(v * v)), float(np.max(np.abs(v)))


def grid_norms(u: np.ndarray, halo: int) -> tuple[float, float]:
    return l2_max(interior(u, halo))


def residual_norms(uT: np.ndarray, uTm1: np.ndarray, halo: int) -> tuple[float, float]:
    """Norms of u_T - u_{T-1}, the difference formed in float64."""
    d = interior(uT, halo).astype(np.float64) - interior(uTm1, halo).astype(np.float64)
    return l2_max(d)


def diff_norms(a: np.ndarray, b: np.ndarray, halo_a: int, halo_b: int) -> tuple[float, float]:
    d = interior(a, halo_a).astype(np.float64) - interior(b, halo_b).astype(np.float64)
    return l2_max(d)
