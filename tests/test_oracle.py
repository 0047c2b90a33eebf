"""The CPU oracle against what the paper and mathematics fix (no GPU)."""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

import gridgen
import numpy_ref
import oracle
import oracle_pins as P

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def run(kind, u0, coeffs, T, halo=None):
    return oracle.run(kind, u0, coeffs, T, halo=halo)


@pytest.mark.parametrize("pin", P.EVERY_PIN, ids=lambda f: f.__name__)
def test_pins_f64(pin):
    pin(run)


@pytest.mark.parametrize("pin", [P.pin_walks_7c, P.pin_shifts_7v, P.pin_brute_integer],
                         ids=lambda f: f.__name__)
def test_exact_pins_f32(pin):
    pin(run, dtype=np.float32)


def test_eigen_f32():
    P.pin_eigen_7(run, dtype=np.float32)
    P.pin_eigen_25(run, dtype=np.float32)


@pytest.mark.parametrize("kind", ["7c", "7v", "25c", "25v"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_numpy_order_bitexact(kind, dtype):
    """Same operation order => same bits (the oracle neither fuses nor reorders)."""
    R = gridgen.RADIUS[kind]
    n = (13, 9, 11)
    u0 = gridgen.field(5, *n, R, -1.0, 1.0, dtype)
    rng = np.random.default_rng(1)
    if kind == "7c":
        co = gridgen.C7
    elif kind == "25c":
        co = gridgen.C25
    elif kind == "7v":
        co = [c.astype(dtype) for c in gridgen.coeffs_7v(9, *n, R)]
    else:
        co = [rng.uniform(0, 0.08, size=u0.shape).astype(dtype) for _ in range(13)]
    a, b = run(kind, u0, co, 5, halo=R)
    ra, rb = numpy_ref.run(kind, u0, co, 5, R)
    assert np.array_equal(a, ra) and np.array_equal(b, rb)


def test_constant_field_preserved_exactly():
    """7c with c0 + 6 c1 = 1 maps a constant field (halo included) to itself;
    in the listing's order this holds exactly for the workload's weights."""
    for val in (1.0, 2.0, 0.5):
        u0 = np.full(gridgen.padded_shape(10, 11, 12, 1), val)
        uT, uTm1 = run("7c", u0, gridgen.C7, 17, halo=1)
        assert np.all(uT == val) and np.all(uTm1 == val)


def test_constant_decay_inside_light_cone():
    """7v with weights summing to 0.999 and a zero halo: points farther than t
    from the halo see only the constant, so u_t = 0.999^t c (to rounding)."""
    n, T, c = (20, 20, 20), 6, 0.75
    u0 = gridgen.zeros(*n, 1)
    gridgen.interior(u0, 1)[...] = c
    C = gridgen.coeffs_7v(4, *n, 1)
    uT, _ = run("7v", u0, C, T, halo=1)
    core = gridgen.interior(uT, 1)[T:-T, T:-T, T:-T]
    assert np.max(np.abs(core / (0.999 ** T * c) - 1)) <= T * 10 * P.U64


def test_max_principle_and_positivity():
    n = (16, 14, 12)
    u0 = gridgen.field(21, *n, 1, 0.0, 1.0)
    C = gridgen.coeffs_7v(21, *n, 1)
    prev = np.max(u0)
    u = u0
    for _ in range(6):
        u, _ = run("7v", u, C, 1, halo=1)
        m = np.max(u)
        assert m <= prev * (1 + 8 * P.U64)
        assert np.min(u) >= 0
        prev = m


@pytest.mark.parametrize("kind", ["7c", "7v", "25c"])
def test_dyadic_scaling_bitexact(kind):
    R = gridgen.RADIUS[kind]
    n = (10, 12, 9)
    u0 = gridgen.field(2, *n, R, -1, 1)
    co = gridgen.C7 if kind == "7c" else gridgen.C25 if kind == "25c" else gridgen.coeffs_7v(2, *n, R)
    a, _ = run(kind, u0, co, 6, halo=R)
    b, _ = run(kind, u0 * 8.0, co, 6, halo=R)
    assert np.array_equal(b, a * 8.0)


@pytest.mark.parametrize("kind", ["7c", "7v", "25c", "25v"])
def test_composition_bitexact(kind):
    """run(T1); run(T2) == run(T1 + T2) and the returned u_{T-1} is the level before."""
    R = gridgen.RADIUS[kind]
    n = (9, 10, 11)
    u0 = gridgen.field(8, *n, R, 0, 1)
    rng = np.random.default_rng(0)
    co = (gridgen.C7 if kind == "7c" else gridgen.C25 if kind == "25c"
          else gridgen.coeffs_7v(8, *n, R) if kind == "7v"
          else [rng.uniform(0, 0.07, size=u0.shape) for _ in range(13)])
    a7, a6 = run(kind, u0, co, 7, halo=R)
    b3, _ = run(kind, u0, co, 3, halo=R)
    b7, b6 = run(kind, b3, co, 4, halo=R)
    c6, _ = run(kind, u0, co, 6, halo=R)
    assert np.array_equal(a7, b7) and np.array_equal(a6, b6) and np.array_equal(a6, c6)


def test_linearity_within_rounding():
    n = (12, 12, 12)
    a = gridgen.field(30, *n, 1, -1, 1)
    b = gridgen.field(31, *n, 1, -1, 1)
    C = gridgen.coeffs_7v(30, *n, 1)
    T = 5
    ra, _ = run("7v", a, C, T, halo=1)
    rb, _ = run("7v", b, C, T, halo=1)
    rab, _ = run("7v", a + b, C, T, halo=1)
    assert np.max(np.abs(rab - (ra + rb))) <= 3 * T * 16 * P.U64 * 2


def test_threads_do_not_change_bits():
    n = (20, 18, 17)
    u0 = gridgen.field(6, *n, 1, 0, 1)
    C = gridgen.coeffs_7v(6, *n, 1)
    a, _ = oracle.run("7v", u0, C, 4, threads=1)
    b, _ = oracle.run("7v", u0, C, 4, threads=5)
    assert np.array_equal(a, b)


def test_zero_steps_and_argument_checks():
    u0 = gridgen.field(1, 5, 5, 5, 1, 0, 1)
    a, b = run("7c", u0, gridgen.C7, 0)
    assert np.array_equal(a, u0) and np.array_equal(b, u0)
    with pytest.raises(ValueError):
        run("7c", u0, gridgen.C7, -1)
    with pytest.raises(ValueError):
        run("25c", u0, gridgen.C25, 1, halo=1)   # halo narrower than the radius
    with pytest.raises(ValueError):
        run("7c", u0, (0.4,), 1)


def _exact_sweeps(kind, u0, co, T, R):
    """Exact rational evaluation (every FP64 input is a dyadic rational)."""
    V = [[[Fraction(float(x)) for x in row] for row in pl] for pl in u0]
    if kind == "7c":
        cf = [Fraction(float(c)) for c in co]
    else:
        cf = [[[[Fraction(float(x)) for x in row] for row in pl] for pl in c] for c in co]
    nzp, nyp, nxp = u0.shape
    for _ in range(T):
        U = [[row[:] for row in pl] for pl in V]
        for k in range(R, nzp - R):
            for j in range(R, nyp - R):
                for i in range(R, nxp - R):
                    if kind == "7c":
                        U[k][j][i] = cf[0] * V[k][j][i] + cf[1] * (
                            V[k][j][i + 1] + V[k][j][i - 1] + V[k][j + 1][i] + V[k][j - 1][i]
                            + V[k + 1][j][i] + V[k - 1][j][i])
                    else:
                        nb = [V[k][j][i], V[k][j][i + 1], V[k][j][i - 1], V[k][j + 1][i],
                              V[k][j - 1][i], V[k + 1][j][i], V[k - 1][j][i]]
                        U[k][j][i] = sum(cf[m][k][j][i] * nb[m] for m in range(7))
        V = U
    return V


@pytest.mark.parametrize("kind", ["7c", "7v"])
def test_within_rounding_bound_of_exact(kind):
    """Non-negative weights summing to <= 1: each sweep adds at most
    gamma_m * ||u||_inf (m = terms + adds); errors do not grow under the
    non-expansive operator, so ||e_T|| <= T * gamma_14 * ||u_0||."""
    n, T = (4, 3, 5), 4
    u0 = gridgen.field(12, *n, 1, 0, 1)
    co = gridgen.C7 if kind == "7c" else gridgen.coeffs_7v(12, *n, 1)
    got, _ = run(kind, u0, co, T, halo=1)
    exact = _exact_sweeps(kind, u0, co, T, 1)
    g14 = 14 * P.U64 / (1 - 14 * P.U64)
    bound = T * g14 * float(np.max(u0))
    err = max(abs(Fraction(float(got[k, j, i])) - exact[k][j][i])
              for k in range(u0.shape[0]) for j in range(u0.shape[1]) for i in range(u0.shape[2]))
    assert float(err) <= bound


def test_f32_form_within_stated_bound():
    """FP32 storage and compute against FP64 on the same (FP32-rounded) inputs:
    ||e_T|| <= T (m + 1) u32 ||u_0|| with m = 13 (7v), the weights being
    non-negative with sum <= 1."""
    n, T = (24, 20, 16), 20
    u0 = gridgen.field(40, *n, 1, 0, 1).astype(np.float32)
    C32 = [c.astype(np.float32) for c in gridgen.coeffs_7v(40, *n, 1)]
    a32, _ = run("7v", u0, C32, T, halo=1)
    a64, _ = run("7v", u0.astype(np.float64), [c.astype(np.float64) for c in C32], T, halo=1)
    err = np.max(np.abs(a32.astype(np.float64) - a64))
    assert err <= T * 14 * P.U32 * float(np.max(u0))
    assert err > 0  # it is a different precision


def test_model_worked_example_golden():
    """The cache-block model's worked example (Sec. III-B, after Eq. 2)."""
    import json
    import os
    from oracle import models
    with open(os.path.join(os.path.dirname(__file__), "golden", "cache_block_example.json")) as f:
        g = json.load(f)
    Ww = models.wavefront_width_r1(g["Dw"], g["N_F"])
    assert Ww == g["W_w"]
    assert models.cache_block_r1(g["Dw"], g["N_F"], 1.0, g["N_D"]) == g["C_S_per_Nxb"]
    assert models.cache_block(g["Dw"], g["N_F"], 1.0, g["R"], g["N_D"]) == g["C_S_per_Nxb"]


@pytest.mark.parametrize("Dw", [4, 8, 12, 16, 20, 32, 64])
@pytest.mark.parametrize("ND", [2, 9, 15])
def test_models_consistent(Dw, ND):
    from oracle import models
    # Eq. (5) reduces to Eq. (4) for R = 1, and Eq. (3) to Eq. (2)
    assert math.isclose(models.code_balance(Dw, ND, 1), models.code_balance_r1(Dw, ND))
    for NF in (1, 4, 10):
        assert math.isclose(models.cache_block(Dw, NF, 64, 1, ND),
                            models.cache_block_r1(Dw, NF, 64, ND))
    # the traffic count of Sec. III-C collapses to 2 s R (N_D + 2) / Dw
    for R in (1, 2, 4):
        for s in (4, 8):
            assert math.isclose(models.code_balance(Dw, ND, R, s), 2 * s * R * (ND + 2) / Dw)


def test_model_radius4_golden():
    """Eq. (3) and Eq. (5) at R = 4 against values evaluated by hand
    (tests/golden/cache_block_r4.json): pins the R-dependent terms that the
    R = 1 worked example cannot reach."""
    import json
    import os
    from oracle import models
    with open(os.path.join(os.path.dirname(__file__), "golden", "cache_block_r4.json")) as f:
        g = json.load(f)
    for c in g["cases"]:
        assert models.wavefront_width(c["Dw"], c["N_F"], c["R"]) == c["W_w"]
        assert models.cache_block(c["Dw"], c["N_F"], 1.0, c["R"], c["N_D"]) == c["C_S_per_Nxb"]
        assert models.cache_block(c["Dw"], c["N_F"], 128.0, c["R"], c["N_D"]) == 128 * c["C_S_per_Nxb"]
        assert models.code_balance(c["Dw"], c["N_D"], c["R"]) == c["B_C_f64"]
