"""Checks that pin the oracle's FP64 reductions (oracle/norms.py) to closed forms.

Each ``pin_*`` takes a module ``N`` with the functions of oracle/norms.py
(``interior``, ``l2_max``, ``grid_norms``, ``residual_norms``, ``diff_norms``)
and raises AssertionError when a result departs from what the check fixes.
They run on the real module (test_norms_oracle.py) and on copies with planted
mistakes, every one of which some pin must catch.

What fixes the expected values:
  * a constant interior of n points: L2 = |c| sqrt(n), max = |c|, whatever
    the (different) halo values are;
  * a discrete sine mode on an n-point axis: sum_{i=1..n} sin^2(p pi i/(n+1))
    = (n+1)/2 for 0 < p < n+1, so over a box L2 = sqrt(prod_a (n_a+1)/2); its
    peak is sin(pi/2) = 1 at the centre of an odd axis for p = 1;
  * exact rational arithmetic on values whose squares and sums are exact in
    FP64 (a few bits each), where the only rounding left is the final sqrt.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def _padded(n, halo, interior_value, halo_value, dtype=np.float64):
    nx, ny, nz = n
    u = np.full((nz + 2 * halo, ny + 2 * halo, nx + 2 * halo), halo_value, dtype=dtype)
    u[halo:halo + nz, halo:halo + ny, halo:halo + nx] = interior_value
    return u


def pin_constant_interior(N):
    """L2 = |c| sqrt(n) and max = |c| over the interior only (the halo holds
    larger values of the other sign, so counting it changes both norms)."""
    for n, halo, c, hv in (((4, 4, 4), 2, 1.0, 7.0), ((4, 4, 4), 1, -1.0, 3.0),
                           ((5, 3, 7), 4, -0.5, 9.0), ((1, 1, 1), 1, 2.0, -5.0)):
        u = _padded(n, halo, c, hv)
        npts = n[0] * n[1] * n[2]
        l2, mx = N.grid_norms(u, halo)
        assert mx == abs(c), "max of a constant interior: %r" % mx
        exp = abs(c) * math.sqrt(npts)
        assert abs(l2 - exp) <= 2 * 2.0 ** -53 * exp, "L2 of a constant interior: %r vs %r" % (l2, exp)
        # perfect squares come out exact
        if int(math.isqrt(npts)) ** 2 == npts:
            assert l2 == exp


def pin_sine_mode(N):
    """Sum of squares of a sine mode is prod (n_a + 1)/2 (discrete orthogonality)."""
    n, halo = (9, 11, 13), 1
    for modes in ((1, 1, 1), (2, 3, 5), (9, 1, 12)):
        ax = [np.sin(m * np.pi * np.arange(1, k + 1) / (k + 1)) for m, k in zip(modes, n)]
        u = _padded(n, halo, 0.0, 4.0)
        u[halo:-halo, halo:-halo, halo:-halo] = ax[2][:, None, None] * ax[1][None, :, None] * ax[0][None, None, :]
        l2, mx = N.grid_norms(u, halo)
        exp = math.sqrt(math.prod((k + 1) / 2 for k in n))
        assert abs(l2 - exp) <= 1e-14 * exp, "sine mode %s: L2 %r vs %r" % (modes, l2, exp)
        if modes == (1, 1, 1):
            # odd axes: the centre point is sin(pi/2)^3 = 1, the peak
            assert mx == 1.0, "sine mode peak %r" % mx
        # a negated mode has the same norms
        l2n, mxn = N.grid_norms(-u, halo)
        assert l2n == l2 and mxn == mx


def pin_exact_sum(N):
    """Values k/256 with |k| < 2^10: squares have at most 20 significant bits
    and the sum over a few thousand points is exact in FP64, so
    L2 = sqrt(exact sum) rounded once, and max is the exact max |v|."""
    rng = np.random.default_rng(5)
    n, halo = (17, 13, 11), 3
    k = rng.integers(-1023, 1024, size=(n[2], n[1], n[0]))
    u = _padded(n, halo, 0.0, 1e6)
    u[halo:-halo, halo:-halo, halo:-halo] = k / 256.0
    tot = sum(Fraction(int(v) * int(v), 65536) for v in k.ravel())
    assert tot.denominator <= 65536
    exp = math.sqrt(float(tot))   # float(tot) is exact here
    l2, mx = N.grid_norms(u, halo)
    assert l2 == exp, "exact-sum L2 %r vs %r" % (l2, exp)
    assert mx == float(np.max(np.abs(k))) / 256.0


def pin_residual_constant_step(N):
    """u_T = u_{T-1} + d with dyadic values: the residual is d at every
    interior point, so its norms are (|d| sqrt(n), |d|); the halos differ
    between the two arrays (they must not enter)."""
    rng = np.random.default_rng(8)
    n, halo = (6, 5, 4), 2
    for dtype in (np.float64, np.float32):
        base = rng.integers(-512, 512, size=(n[2], n[1], n[0])) / 1024.0
        um1 = _padded(n, halo, 0.0, -2.0, dtype)
        uT = _padded(n, halo, 0.0, 6.0, dtype)
        um1[halo:-halo, halo:-halo, halo:-halo] = base
        uT[halo:-halo, halo:-halo, halo:-halo] = base - 0.375
        l2, mx = N.residual_norms(uT, um1, halo)
        npts = n[0] * n[1] * n[2]
        assert mx == 0.375, "residual max %r" % mx
        assert abs(l2 - 0.375 * math.sqrt(npts)) <= 2 * 2.0 ** -53 * l2
    # FP32 inputs whose difference needs 31 significant bits: exact only if
    # the difference is formed in FP64 (rounded to 1 + 2^-23 in FP32)
    a = _padded(n, halo, np.float32(1.0 + 2.0 ** -23), 1.0, np.float32)
    b = _padded(n, halo, np.float32(2.0 ** -30), 1.0, np.float32)
    l2, mx = N.residual_norms(a, b, halo)
    assert mx == 1.0 + 2.0 ** -23 - 2.0 ** -30, "FP32 residual not formed in FP64: %r" % mx


def pin_diff_across_halos(N):
    """Two grids with the same interior extents and different halo widths:
    the interiors are aligned, and only they enter."""
    rng = np.random.default_rng(9)
    n = (7, 6, 5)
    base = rng.integers(-100, 100, size=(n[2], n[1], n[0])) / 64.0
    a = _padded(n, 1, 0.0, 11.0)
    b = _padded(n, 3, 0.0, -13.0, np.float32)
    a[1:-1, 1:-1, 1:-1] = base
    b[3:-3, 3:-3, 3:-3] = base + 0.25
    b[3, 3, 3] += 1.0                      # one point differs by 1.25
    l2, mx = N.diff_norms(a, b, 1, 3)
    npts = n[0] * n[1] * n[2]
    exp = math.sqrt((npts - 1) * 0.0625 + 1.5625)
    assert mx == 1.25, "diff max %r" % mx
    assert abs(l2 - exp) <= 2 * 2.0 ** -53 * exp, "diff L2 %r vs %r" % (l2, exp)
    # argument order does not matter for norms of a difference
    assert N.diff_norms(b, a, 3, 1) == (l2, mx)


def pin_l2_max_plain(N):
    """l2_max on a flat vector: (5, 4) for (3, -4); an empty input gives (0, 0)."""
    assert N.l2_max(np.array([3.0, -4.0])) == (5.0, 4.0)
    assert N.l2_max(np.array([-4.0, 0.0, 3.0], dtype=np.float32)) == (5.0, 4.0)
    assert N.l2_max(np.zeros(0)) == (0.0, 0.0)


EVERY_NORM_PIN = (pin_constant_interior, pin_sine_mode, pin_exact_sum, pin_residual_constant_step,
                  pin_diff_across_halos, pin_l2_max_plain)
