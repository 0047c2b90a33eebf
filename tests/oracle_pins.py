"""Checks that pin the CPU oracle to facts fixed by the paper and by mathematics.

Each ``pin_*`` function takes a ``run(kind, u0, coeffs, T, halo=...)`` callable
with the oracle's signature and raises AssertionError when the result departs
from what the check fixes.  They are used on the real oracle
(test_oracle.py) and on copies of it with planted mistakes
(test_oracle_mutants.py), which every pin set must catch.

What fixes the expected values:
  * lattice-walk counts (combinatorics) for the 7-point operator applied to a
    unit impulse;
  * pure shifts for one-hot 7-point variable weights (each weight of
    Listing 2 multiplies exactly one neighbour);
  * binomial spreading for one-hot 25-point weights (each weight of
    Listing 3 multiplies the +r and -r neighbour pair along one axis);
  * the closed-form eigenvalue of discrete sine modes on a Dirichlet box;
  * exact integer brute force on tiny grids.
"""
from __future__ import annotations

import math
from math import comb

import numpy as np

import gridgen

U64 = 2.0 ** -53
U32 = 2.0 ** -24

# Offsets (dx, dy, dz) of the 12 radius/axis weights C01..C12 of Listing 3.
AXES = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
C25_OFFSETS = [(r, AXES[a]) for r in (1, 2, 3, 4) for a in range(3)]


def _b(k: int, d: int) -> int:
    """Number of +-1 walks of k steps along one axis ending at d."""
    if abs(d) > k or (k + d) % 2:
        return 0
    return comb(k, (k + d) // 2)


def walk_count(T: int, d: tuple[int, int, int], c0: int) -> int:
    """Weighted count of T-step lattice walks with steps 0 (weight c0) or +-e_axis
    (weight 1) from the origin to d: the impulse response of Listing 1 with
    c1 = 1 on an unbounded grid."""
    tot = 0
    for k0 in range(T + 1):
        for kx in range(T - k0 + 1):
            for ky in range(T - k0 - kx + 1):
                kz = T - k0 - kx - ky
                m = math.factorial(T) // (math.factorial(k0) * math.factorial(kx)
                                          * math.factorial(ky) * math.factorial(kz))
                tot += m * c0 ** k0 * _b(kx, d[0]) * _b(ky, d[1]) * _b(kz, d[2])
    return tot


def _impulse(n: tuple[int, int, int], halo: int, at: tuple[int, int, int], dtype=np.float64):
    nx, ny, nz = n
    u = gridgen.zeros(nx, ny, nz, halo, dtype)
    x, y, z = at
    u[z + halo, y + halo, x + halo] = 1.0
    return u


def pin_walks_7c(run, dtype=np.float64):
    n, h, T, c0 = (11, 12, 13), 1, 4, 2
    cx, cy, cz = 5, 6, 6
    u0 = _impulse(n, h, (cx, cy, cz), dtype)
    uT, _ = run("7c", u0, (float(c0), 1.0), T, halo=h)
    got = gridgen.interior(uT, h)
    exp = np.zeros_like(got)
    for dz in range(-T, T + 1):
        for dy in range(-T, T + 1):
            for dx in range(-T, T + 1):
                if abs(dx) + abs(dy) + abs(dz) <= T:
                    exp[cz + dz, cy + dy, cx + dx] = walk_count(T, (dx, dy, dz), c0)
    assert np.array_equal(got, exp), "7c impulse response differs from the walk count"


def _shift_expect(u0i: np.ndarray, axis_xyz: int, step: int, T: int) -> np.ndarray:
    """u_T(p) = u_0(p + T*step*e_axis) if that point is interior, else 0."""
    ax = 2 - axis_xyz  # numpy axis of x, y, z
    out = np.zeros_like(u0i)
    n = u0i.shape[ax]
    s = T * step
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    if s >= 0:
        src[ax] = slice(s, n)
        dst[ax] = slice(0, max(0, n - s))
    else:
        src[ax] = slice(0, max(0, n + s))
        dst[ax] = slice(-s, n)
    out[tuple(dst)] = u0i[tuple(src)]
    return out


def pin_shifts_7v(run, dtype=np.float64):
    """One-hot weights of Listing 2: C1..C6 pick +x,-x,+y,-y,+z,-z; C0 the centre."""
    n, h, T = (9, 10, 11), 1, 3
    rng = np.random.default_rng(7)
    u0 = gridgen.zeros(*n, h, dtype)
    gridgen.interior(u0, h)[...] = rng.uniform(-1, 1, size=(n[2], n[1], n[0]))
    dirs = [None, (0, +1), (0, -1), (1, +1), (1, -1), (2, +1), (2, -1)]
    for m in range(7):
        C = [np.zeros_like(u0) for _ in range(7)]
        C[m][...] = 1.0
        uT, _ = run("7v", u0, C, T, halo=h)
        got = gridgen.interior(uT, h)
        if m == 0:
            exp = gridgen.interior(u0, h)
        else:
            exp = _shift_expect(gridgen.interior(u0, h), dirs[m][0], dirs[m][1], T)
        assert np.array_equal(got, exp), "7v weight C%d does not pick its neighbour" % m


def pin_binomial_25(run, kind="25c", dtype=np.float64):
    """One-hot weights of Listing 3: weight q spreads an impulse binomially
    along its axis with step r; C00 alone is the identity."""
    n, h, T = (21, 23, 25), 4, 2
    at = (10, 11, 12)
    u0 = _impulse(n, h, at, dtype)
    for q in range(13):
        if kind == "25c":
            coeffs = [0.0] * 13
            coeffs[q] = 1.0
        else:
            coeffs = [np.zeros_like(u0) for _ in range(13)]
            coeffs[q][...] = 1.0
        uT, _ = run(kind, u0, coeffs, T, halo=h)
        got = gridgen.interior(uT, h)
        exp = np.zeros_like(got)
        if q == 0:
            exp[at[2], at[1], at[0]] = 1.0
        else:
            r, (ex, ey, ez) = C25_OFFSETS[q - 1]
            for k in range(T + 1):
                o = r * (2 * k - T)
                exp[at[2] + o * ez, at[1] + o * ey, at[0] + o * ex] += comb(T, k)
        assert np.array_equal(got, exp), "%s weight %d misplaced" % (kind, q)


def sine_mode(n, modes, halo, dtype=np.float64):
    """u(i,j,k) = sin(p pi i/(nx+1)) sin(q pi j/(ny+1)) sin(r pi k/(nz+1)), i = 1..n."""
    nx, ny, nz = n
    p, q, r = modes
    sx = np.sin(p * np.pi * np.arange(1, nx + 1) / (nx + 1))
    sy = np.sin(q * np.pi * np.arange(1, ny + 1) / (ny + 1))
    sz = np.sin(r * np.pi * np.arange(1, nz + 1) / (nz + 1))
    u = gridgen.zeros(nx, ny, nz, halo, dtype)
    gridgen.interior(u, halo)[...] = sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    return u


def thetas(n, modes):
    return [m * np.pi / (k + 1) for m, k in zip(modes, n)]


def pin_eigen_7(run, dtype=np.float64):
    """Sine modes are eigenvectors of the radius-1 operators with Dirichlet zero
    halo: u_T = lambda^T u_0, lambda = c0 + sum_axis (w+ + w-) cos(theta_axis)."""
    u = U64 if dtype == np.float64 else U32
    n, h, T = (20, 22, 24), 1, 8
    for modes in ((1, 1, 1), (3, 5, 2), (20, 22, 24), (7, 1, 13)):
        th = thetas(n, modes)
        u0 = sine_mode(n, modes, h, dtype)
        ref = gridgen.interior(u0, h).astype(np.float64)
        # 7c, c0 = 0.4, c1 = 0.1
        lam = 0.4 + 0.2 * sum(math.cos(t) for t in th)
        uT, _ = run("7c", u0, (0.4, 0.1), T, halo=h)
        err = np.max(np.abs(gridgen.interior(uT, h) - lam ** T * ref))
        assert err <= (4 + 12 * T) * u, "7c eigenmode %s: err %g" % (modes, err)
        # 7v, spatially uniform but anisotropic weights summing to 1
        w = (0.3, 0.05, 0.05, 0.1, 0.1, 0.2, 0.2)
        C = [np.full_like(u0, wm) for wm in w]
        lam = w[0] + (w[1] + w[2]) * math.cos(th[0]) + (w[3] + w[4]) * math.cos(th[1]) \
            + (w[5] + w[6]) * math.cos(th[2])
        uT, _ = run("7v", u0, C, T, halo=h)
        err = np.max(np.abs(gridgen.interior(uT, h) - lam ** T * ref))
        assert err <= (4 + 16 * T) * u, "7v eigenmode %s: err %g" % (modes, err)


def pin_eigen_25(run, kind="25c", dtype=np.float64):
    """Radius-4 star on a sine mode: lambda = C00 + 2 sum_{r,axis} C_{r,axis}
    cos(r theta_axis), exact at points farther than R*T from every face (the
    zero halo differs from the mode's odd extension beyond the first layer)."""
    u = U64 if dtype == np.float64 else U32
    n, h, T, R = (30, 32, 34), 4, 2, 4
    rng = np.random.default_rng(11)
    cw = rng.uniform(0.01, 0.06, size=12)
    coeffs = [0.2] + [float(x) for x in cw]
    for modes in ((1, 2, 3), (5, 3, 9), (30, 32, 34)):
        th = thetas(n, modes)
        u0 = sine_mode(n, modes, h, dtype)
        lam = coeffs[0] + 2 * sum(coeffs[1 + i] * math.cos(r * th[a])
                                  for i, (r, e) in enumerate(C25_OFFSETS)
                                  for a in range(3) if e[a])
        cs = coeffs if kind == "25c" else [np.full_like(u0, c) for c in coeffs]
        uT, _ = run(kind, u0, cs, T, halo=h)
        d = R * T
        got = gridgen.interior(uT, h)[d:-d, d:-d, d:-d]
        ref = gridgen.interior(u0, h)[d:-d, d:-d, d:-d].astype(np.float64)
        err = np.max(np.abs(got - lam ** T * ref))
        assert err <= (4 + 40 * T) * u, "%s eigenmode %s: err %g" % (kind, modes, err)


def brute_int(kind, u0i, coeffs, T, R):
    """Exact integer evaluation of T sweeps on the padded Python-int grid u0i
    (nested lists [z][y][x]); halo entries are fixed.  Used only with integer
    fields and weights, where every order of evaluation gives the same sum."""
    nzp, nyp, nxp = len(u0i), len(u0i[0]), len(u0i[0][0])
    V = [[row[:] for row in pl] for pl in u0i]
    for _ in range(T):
        U = [[row[:] for row in pl] for pl in V]
        for k in range(R, nzp - R):
            for j in range(R, nyp - R):
                for i in range(R, nxp - R):
                    if kind == "7c":
                        c0, c1 = coeffs
                        s = c0 * V[k][j][i]
                        for (a, b, c) in AXES:
                            s += c1 * (V[k + c][j + b][i + a] + V[k - c][j - b][i - a])
                    elif kind == "7v":
                        C = coeffs
                        nb = [V[k][j][i], V[k][j][i + 1], V[k][j][i - 1], V[k][j + 1][i],
                              V[k][j - 1][i], V[k + 1][j][i], V[k - 1][j][i]]
                        s = sum(C[m][k][j][i] * nb[m] for m in range(7))
                    else:
                        def w(q):
                            return coeffs[q] if kind == "25c" else coeffs[q][k][j][i]
                        s = w(0) * V[k][j][i]
                        for q, (r, (a, b, c)) in enumerate(C25_OFFSETS, start=1):
                            s += w(q) * (V[k + r * c][j + r * b][i + r * a]
                                         + V[k - r * c][j - r * b][i - r * a])
                    U[k][j][i] = s
        V = U
    return V


def pin_brute_integer(run, dtype=np.float64):
    """Small integer fields and weights make every operation exact, so the
    oracle must equal the exact integer brute force bit for bit."""
    rng = np.random.default_rng(3)
    for kind, n, T in (("7c", (4, 5, 3), 4), ("7v", (3, 4, 5), 3),
                       ("25c", (9, 3, 2), 2), ("25v", (2, 9, 3), 2)):
        R = gridgen.RADIUS[kind]
        u0 = gridgen.zeros(*n, R, dtype)
        u0[...] = rng.integers(-3, 4, size=u0.shape)   # halo values too (fixed boundary)
        if kind == "7c":
            coeffs = (2.0, -1.0)
            cint = (2, -1)
        elif kind == "25c":
            cint = tuple(int(x) for x in rng.integers(-2, 3, size=13))
            coeffs = tuple(float(x) for x in cint)
        else:
            m = 7 if kind == "7v" else 13
            arrs = [rng.integers(-2, 3, size=u0.shape).astype(dtype) for _ in range(m)]
            coeffs = arrs
            cint = [a.astype(np.int64).tolist() for a in arrs]
        exp = brute_int(kind, u0.astype(np.int64).tolist(), cint, T, R)
        uT, _ = run(kind, u0, coeffs, T, halo=R)
        assert np.array_equal(uT, np.array(exp, dtype=np.float64)), "%s brute force" % kind


ALL_PINS = (pin_walks_7c, pin_shifts_7v, pin_binomial_25, pin_eigen_7, pin_eigen_25,
            pin_brute_integer)


def pin_binomial_25v(run):
    return pin_binomial_25(run, kind="25v")


def pin_eigen_25v(run):
    return pin_eigen_25(run, kind="25v")


EVERY_PIN = ALL_PINS + (pin_binomial_25v, pin_eigen_25v)
