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
