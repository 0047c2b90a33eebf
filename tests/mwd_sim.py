"""CPU simulator of the GPU library's MWD tile schedule (a test double, no GPU).

It restates, in NumPy, the tiling rules the HIP tile kernel follows: diamond
rows in y-t, per-row level classification (computed / needed / stored), the
x tiles with their recomputed overlap, the three rotating buffer pairs, the
load sources of values a tile does not compute, and the final gather.  It
then executes every tile, row by row, and

  * records every buffer location each tile reads or writes, and checks that
    within one row no tile reads a location that any tile writes and no two
    tiles write the same location (tiles of a row run concurrently on the
    GPU);
  * poisons all scratch with NaN, so a value the schedule fails to provide
    shows up in the result;
  * returns the caller's two buffers after the gather, to be compared bit for
    bit with the oracle.

Values are combined in the listings' operation order with NumPy (one rounding
per operation), so a correct schedule reproduces the oracle exactly.
"""
from __future__ import annotations

import numpy as np

AXES = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
RADIUS = {"7c": 1, "7v": 1, "25c": 4, "25v": 4}


def floordiv(a, b):
    return a // b


def row_of(y, t, R, DW):
    return floordiv(y + R * t, DW) - floordiv(y - R * t, DW)


def pair_of_row(rho):
    return (rho + 1) % 3


class Buffers:
    """Three pairs of padded buffers; pair 0 holds the caller's arrays."""

    def __init__(self, u0, halo, cur):
        self.h = halo
        self.p = [[None, None] for _ in range(3)]
        self.p[0][cur] = u0.copy()
        self.p[0][cur ^ 1] = u0.copy()  # same halo; interior overwritten
        for k in (1, 2):
            for b in (0, 1):
                a = np.full_like(u0, np.nan)
                self.p[k][b] = a
        self.halo_src = (0, cur)

    def get(self, pair, bi, x, y, z):
        h = self.h
        return self.p[pair][bi][z + h, y + h, x + h]

    def set(self, pair, bi, x, y, z, v):
        h = self.h
        self.p[pair][bi][z + h, y + h, x + h] = v


def _apply(kind, nb, w):
    """One update in the listings' order; nb(dx,dy,dz) and w(m) return arrays."""
    if kind == "7c":
        u = w(0) * nb(0, 0, 0)
        for (a, b, c) in AXES:
            u = u + w(1) * (nb(a, b, c) + nb(-a, -b, -c))
        return u
    if kind == "7v":
        order = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
        u = w(0) * nb(*order[0])
        for m in range(1, 7):
            u = u + w(m) * nb(*order[m])
        return u
    u = w(0) * nb(0, 0, 0)
    q = 1
    for r in (1, 2, 3, 4):
        for (a, b, c) in AXES:
            u = u + w(q) * (nb(r * a, r * b, r * c) + nb(-r * a, -r * b, -r * c))
            q += 1
    return u


def simulate(kind, u0, coeffs, T, DW, LX, halo=None, cur=0, shuffle_seed=None, checks=True):
    """Run the MWD schedule on the CPU; returns (buf0, buf1, new_cur)."""
    R = RADIUS[kind]
    h = R if halo is None else halo
    dt = u0.dtype
    nzp, nyp, nxp = u0.shape
    nx, ny, nz = nxp - 2 * h, nyp - 2 * h, nzp - 2 * h
    H = DW // (2 * R)
    L = 2 * H - 1
    XT = LX - 2 * L * R
    assert DW % (2 * R) == 0 and XT > 0
    bufs = Buffers(u0, h, cur)
    if kind in ("7c", "25c"):
        W = [dt.type(c) for c in coeffs]
        wget = lambda m, xs, y, zs: W[m]
    else:
        carr = [np.ascontiguousarray(c) for c in coeffs]
        wget = lambda m, xs, y, zs: carr[m][zs[:, None] + h, y + h, xs[None, :] + h]
    nxt = -(-nx // XT)
    rho_max = -(-T // H)
    rng = np.random.default_rng(shuffle_seed) if shuffle_seed is not None else None
    zs_all = np.arange(-R, nz + R)  # plane index space of the value arrays

    for rho in range(rho_max + 1):
        t0 = (rho - 1) * H
        yoff = (rho % 2) * (DW // 2)
        ybase = yoff - DW if yoff > 0 else 0
        nB = (ny - 1 - ybase) // DW + 1
        tiles = [(b, j) for b in range(nB) for j in range(nxt)]
        if rng is not None:
            rng.shuffle(tiles)
        reads = [[np.zeros(u0.shape, bool) for _ in range(2)] for _ in range(3)]
        owner = [[np.full(u0.shape, -1, np.int64) for _ in range(2)] for _ in range(3)]
        for (b, j) in tiles:
            yL = ybase + b * DW
            x0 = j * XT
            xs = x0 - L * R + np.arange(LX)

            def computed(yrr, tau):
                if tau < 1 or tau > L or yrr < 0 or yrr >= DW:
                    return False
                t = t0 + tau
                if t < 1 or t > T:
                    return False
                yy = yL + yrr
                if yy < 0 or yy >= ny:
                    return False
                d = DW // 2 - 1 - yrr if yrr < DW // 2 else yrr - DW // 2
                return d < R * min(tau, 2 * H - tau)

            def needed(yrr, tau):
                return tau < L and any(computed(yrr + dy, tau + 1) for dy in range(-R, R + 1))

            def level_src(yy, t):
                if t < 0 or yy < 0 or yy >= ny:
                    return None  # halo
                p = 0 if t == 0 else pair_of_row(row_of(yy, t, R, DW))
                return (p, (cur + t) & 1)

            # value arrays: val[(yr, tau)] -> (planes -R..nz+R-1, lanes)
            val = {}
            xl = np.arange(LX)
            xin = (xs >= 0) & (xs < nx)
            pin = (zs_all >= 0) & (zs_all < nz)
            Z = np.broadcast_to(zs_all[:, None], (nz + 2 * R, LX))
            X = np.broadcast_to(xs[None, :], (nz + 2 * R, LX))
            for tau in range(L + 1):
                for yr in range(-R, DW + R):
                    c = computed(yr, tau)
                    side = yr < 0 or yr >= DW
                    pres = (tau == H - 1 and needed(yr, tau)) if side else (c or needed(yr, tau))
                    if not pres:
                        continue
                    y = yL + yr
                    yin = 0 <= y < ny
                    lact = (xl >= tau * R) & (xl < LX - tau * R) & (xs >= -R) & (xs < nx + R)
                    zrow = pin if side else np.ones_like(pin)
                    act = lact[None, :] & zrow[:, None]
                    comp = (act & xin[None, :] & pin[:, None]) if (c and tau >= 1) else np.zeros_like(act)
                    load = act & ~comp
                    v = np.full((nz + 2 * R, LX), np.nan, dtype=dt)
                    inner = load & xin[None, :] & pin[:, None] & yin
                    halo_ld = load & ~inner
                    if halo_ld.any():
                        hb = bufs.p[0][cur]
                        v[halo_ld] = hb[Z[halo_ld] + h, y + h, X[halo_ld] + h]
                    if inner.any():
                        src = level_src(y, t0 + tau)
                        assert src is not None
                        sb = bufs.p[src[0]][src[1]]
                        v[inner] = sb[Z[inner] + h, y + h, X[inner] + h]
                        rd = reads[src[0]][src[1]]
                        rd[Z[inner] + h, y + h, X[inner] + h] = True
                    if comp.any():
                        zi, ks = np.nonzero(comp)

                        def nb(dx, dy, dz, zi=zi, ks=ks, yr=yr, tau=tau):
                            return val[(yr + dy, tau - 1)][zi + dz, ks + dx]

                        def w(m, zi=zi, ks=ks, y=y):
                            if kind in ("7c", "25c"):
                                return W[m]
                            return carr[m][zs_all[zi] + h, y + h, xs[ks] + h]

                        v[zi, ks] = _apply(kind, nb, w)
                    val[(yr, tau)] = v
            # stores: last two computed levels of each diamond row
            xout = (xl >= L * R) & (xl < L * R + XT) & (xs < nx)
            ko = np.nonzero(xout)[0]
            for yr in range(DW):
                clev = [tau for tau in range(L + 1) if computed(yr, tau)]
                if not clev:
                    continue
                thi = clev[-1]
                y = yL + yr
                pr = pair_of_row(rho)
                for tau in clev:
                    if tau < thi - 1:
                        continue
                    bi = (cur + t0 + tau) & 1
                    vv = val[(yr, tau)][R:R + nz][:, ko]
                    assert not np.isnan(vv).any(), "stored an unset value (row %d tile %s)" % (rho, (b, j))
                    own = owner[pr][bi][h:h + nz, y + h, xs[ko] + h]
                    assert (own < 0).all(), "two tiles write the same points (row %d)" % rho
                    owner[pr][bi][h:h + nz, y + h, xs[ko] + h] = b * 100000 + j
                    bufs.p[pr][bi][h:h + nz, y + h, xs[ko] + h] = vv
        if checks:
            for pp in range(3):
                for bb in range(2):
                    clash = reads[pp][bb] & (owner[pp][bb] >= 0)
                    assert not clash.any(), "row %d reads points it writes (pair %d)" % (rho, pp)
    # gather u_T and u_{T-1} into pair 0
    for k in (0, 1):
        t = T - k
        if t < 1:
            continue
        bi = (cur + t) & 1
        for y in range(ny):
            p = pair_of_row(row_of(y, t, R, DW))
            if p != 0:
                bufs.p[0][bi][h:h + nz, y + h, h:h + nx] = bufs.p[p][bi][h:h + nz, y + h, h:h + nx]
    return bufs.p[0][0], bufs.p[0][1], cur ^ (T & 1)
