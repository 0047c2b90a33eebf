"""The sampled-parity helper against full oracle runs (CPU only)."""
import numpy as np
import pytest

import cone
import gridgen
import oracle


@pytest.mark.parametrize("kind,n,T", [("7v", (40, 36, 30), 6), ("25c", (45, 50, 41), 3),
                                      ("7c", (33, 20, 25), 9)])
def test_subbox_value_equals_full_run(kind, n, T):
    R = gridgen.RADIUS[kind]
    h = R + (1 if kind == "7c" else 0)          # a halo wider than the radius too
    u0 = gridgen.field(4, *n, h, -1.0, 1.0)
    co = (gridgen.coeffs_7v(4, *n, h) if kind == "7v" else
          gridgen.C7 if kind == "7c" else gridgen.C25)
    uT, _ = oracle.run(kind, u0, co, T, halo=h)
    for p in cone.sample_points(n, 12, seed=1):
        v = cone.subbox_value(kind, u0, co, T, h, p)
        assert v == uT[p[2] + h, p[1] + h, p[0] + h]


@pytest.mark.parametrize("kind,n,T", [("7v", (60, 50, 40), 5), ("25c", (70, 60, 50), 3),
                                      ("7c", (33, 20, 25), 9)])
def test_box_values_equal_full_run(kind, n, T):
    R = gridgen.RADIUS[kind]
    h = R + (1 if kind == "7c" else 0)
    u0 = gridgen.field(6, *n, h, -1.0, 1.0)
    co = (gridgen.coeffs_7v(6, *n, h) if kind == "7v" else
          gridgen.C7 if kind == "7c" else gridgen.C25)
    uT, _ = oracle.run(kind, u0, co, T, halo=h)
    full = gridgen.interior(uT, h)
    boxes = cone.line_boxes(n, T, R, seed=2) + [((5, 6, 7), (9, 18, 12))]
    for lo, hi in boxes:
        got = cone.box_values(kind, u0, co, T, h, lo, hi)
        assert np.array_equal(got, full[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]), (lo, hi)
