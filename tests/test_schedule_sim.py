"""The MWD tile schedule, run on the CPU by the simulator, against the oracle.

Checks the geometry the HIP tile kernel follows (no GPU): diamond rows,
clipping at t = 1, t = T and the y edges, x tiles with recomputed overlap,
the three rotating buffer pairs and the gather; tiles of a row are executed
in a shuffled order and must never read what another tile of the row writes.
"""
from __future__ import annotations

import numpy as np
import pytest

import gridgen
import mwd_sim
import oracle

CASES = [
    # kind, DW, LX, (nx, ny, nz), T, cur
    ("7c", 4, 64, (20, 17, 9), 7, 0),
    ("7c", 8, 64, (23, 29, 7), 9, 1),
    ("7c", 8, 128, (130, 19, 5), 5, 0),
    ("7c", 8, 64, (51, 8, 4), 1, 0),
    ("7c", 8, 64, (37, 3, 6), 2, 1),
    ("7c", 4, 128, (70, 31, 5), 12, 0),
    ("7v", 8, 64, (30, 21, 6), 11, 0),
    ("7v", 4, 64, (61, 13, 5), 6, 1),
    ("7c", 16, 64, (40, 33, 4), 20, 0),
    ("25c", 16, 64, (45, 37, 10), 5, 0),
    ("25c", 8, 64, (29, 23, 9), 3, 1),
    ("25v", 16, 64, (41, 20, 9), 4, 0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-dw%d-lx%d-%s-T%d" % (c[0], c[1], c[2], "x".join(map(str, c[3])), c[4]))
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_schedule_matches_oracle(case, dtype):
    kind, DW, LX, n, T, cur = case
    R = gridgen.RADIUS[kind]
    u0 = gridgen.field(17, *n, R, -1.0, 1.0, dtype)
    rng = np.random.default_rng(5)
    if kind == "7c":
        co = gridgen.C7
    elif kind == "25c":
        co = gridgen.C25
    elif kind == "7v":
        co = [c.astype(dtype) for c in gridgen.coeffs_7v(17, *n, R)]
    else:
        co = [rng.uniform(0, 0.07, size=u0.shape).astype(dtype) for _ in range(13)]
    b0, b1, ncur = mwd_sim.simulate(kind, u0, co, T, DW, LX, cur=cur, shuffle_seed=T)
    uT, uTm1 = oracle.run(kind, u0, co, T)
    bufs = (b0, b1)
    assert ncur == cur ^ (T & 1)
    assert np.array_equal(bufs[ncur], uT)
    if T >= 1:
        assert np.array_equal(bufs[ncur ^ 1], uTm1)


def test_every_point_in_exactly_one_tile():
    """The diamond rows partition space-time: each (y, t), 1 <= t <= T, is
    computed by exactly one (row, diamond) and rows increase with t."""
    for R, DW, ny, T in ((1, 8, 37, 19), (4, 16, 50, 9), (1, 4, 9, 30)):
        H = DW // (2 * R)
        L = 2 * H - 1
        seen = np.zeros((ny, T + 1), int)
        for rho in range(-(-T // H) + 1):
            t0 = (rho - 1) * H
            yoff = (rho % 2) * (DW // 2)
            ybase = yoff - DW if yoff > 0 else 0
            nB = (ny - 1 - ybase) // DW + 1
            for b in range(nB):
                yL = ybase + b * DW
                for tau in range(1, L + 1):
                    t = t0 + tau
                    if not (1 <= t <= T):
                        continue
                    r = R * min(tau, 2 * H - tau)
                    for yr in range(DW):
                        d = DW // 2 - 1 - yr if yr < DW // 2 else yr - DW // 2
                        y = yL + yr
                        if d < r and 0 <= y < ny:
                            seen[y, t] += 1
                            assert mwd_sim.row_of(y, t, R, DW) == rho
        assert (seen[:, 1:] == 1).all()


def _tile_masks(R, DW, ny, T, rho, b):
    """Per diamond row yr of tile (rho, b): the computed and present level
    masks, and the side-row presence, in the HIP tile kernel's terms."""
    H = DW // (2 * R)
    L = 2 * H - 1
    t0 = (rho - 1) * H
    yoff = (rho % 2) * (DW // 2)
    ybase = yoff - DW if yoff > 0 else 0
    yL = ybase + b * DW

    def computed(yrr, tau):
        if tau < 1 or tau > L or yrr < 0 or yrr >= DW:
            return False
        t = t0 + tau
        if t < 1 or t > T:
            return False
        if not 0 <= yL + yrr < ny:
            return False
        d = DW // 2 - 1 - yrr if yrr < DW // 2 else yrr - DW // 2
        return d < R * min(tau, 2 * H - tau)

    def needed(yrr, tau):
        return tau < L and any(computed(yrr + dy, tau + 1) for dy in range(-R, R + 1))

    out = []
    for yr in range(DW):
        c = [computed(yr, tau) for tau in range(L + 1)]
        p = [c[tau] or needed(yr, tau) for tau in range(L + 1)]
        out.append((c, p))
    side = {yrs: any(needed(yrs, tau) for tau in range(L + 1) if tau != H - 1)
            for yrs in list(range(-R, 0)) + list(range(DW, DW + R))}
    return out, side, yL


@pytest.mark.parametrize("R,DW", [(1, 4), (1, 6), (1, 8), (1, 12), (1, 16), (4, 8), (4, 16), (4, 24)])
def test_edge_levels_at_most_two(R, DW):
    """The tile kernel loads, per diamond row, only the (at most two) levels
    below its first computed level that the tile needs, plus the boundary;
    side rows are needed at level h - 1 only.  Checked over every row and
    diamond, with clipping at t = 1, t = T and both y edges."""
    H = DW // (2 * R)
    for ny in (DW // 2 + 1, 3 * DW + 5, 40):
        for T in (1, H, 2 * H + 1, 3 * H + 2):
            for rho in range(-(-T // H) + 1):
                yoff = (rho % 2) * (DW // 2)
                ybase = yoff - DW if yoff > 0 else 0
                for b in range((ny - 1 - ybase) // DW + 1):
                    rows, side, yL = _tile_masks(R, DW, ny, T, rho, b)
                    for yr, (c, p) in enumerate(rows):
                        if not 0 <= yL + yr < ny:
                            # a row outside the domain holds boundary values
                            # at every level it is present at
                            assert not any(c)
                            continue
                        edge = [tau for tau in range(len(c)) if p[tau] and not c[tau]]
                        assert len(edge) <= 2, (R, DW, ny, T, rho, b, yr, edge)
                        if edge and any(c):
                            first = c.index(True)
                            assert all(tau < first for tau in edge)
                    # side rows are never needed at a level other than h - 1
                    assert not any(side.values())


def _xcd_tile(blk, ntiles, c):
    # the tile kernel's workgroup-to-tile map (XCD-aware, see mwd_tile.hpp)
    g = blk // (8 * c)
    if (g + 1) * 8 * c > ntiles:
        return blk
    r = blk - g * 8 * c
    return g * 8 * c + (r % 8) * c + r // 8


@pytest.mark.parametrize("ntiles,c", [(1, 1), (7, 3), (64 * 11, 11), (128 * 9, 9), (100, 13), (8 * 5 * 3 + 4, 5)])
def test_xcd_tile_map_is_bijection_with_runs_per_xcd(ntiles, c):
    t = [_xcd_tile(b, ntiles, c) for b in range(ntiles)]
    assert sorted(t) == list(range(ntiles))
    # inside full groups, consecutive tiles of a run share the XCD (blk mod 8)
    full = (ntiles // (8 * c)) * 8 * c
    inv = {tt: b for b, tt in enumerate(t)}
    for tt in range(full):
        if tt % c != c - 1:
            assert inv[tt] % 8 == inv[tt + 1] % 8
