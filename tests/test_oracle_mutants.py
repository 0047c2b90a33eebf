"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check that
the pins catch every one of them: a dropped term, a wrong sign, a wrong index
or radius, a transposed axis or weight, a missing buffer swap, a short loop."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

import oracle
import oracle_pins as P

MUTANTS = {
    "7c_wrong_index": ("u = u + c[1] * (v[axis_step[a]] + v[-axis_step[a]]);",
                       "u = u + c[1] * (v[axis_step[a]] + v[axis_step[a]]);"),
    "7c_dropped_z_pair": ("for (int a = 0; a < 3; a++)\n                        u = u + c[1]",
                          "for (int a = 0; a < 2; a++)\n                        u = u + c[1]"),
    "7c_wrong_centre_weight": ("u = c[0] * v[0];", "u = c[1] * v[0];"),
    "7v_transposed_axis": ("const long long nb7[6] = {1, -1, sy, -sy, sz, -sz};",
                           "const long long nb7[6] = {1, -1, sz, -sy, sy, -sz};"),
    "7v_wrong_sign": ("u = u + C[m][o] * v[nb7[m - 1]];",
                      "u = u + (m == 6 ? -C[m][o] : C[m][o]) * v[nb7[m - 1]];"),
    "7v_swapped_weights": ("const long long nb7[6] = {1, -1, sy, -sy, sz, -sz};",
                           "const long long nb7[6] = {-1, 1, sy, -sy, sz, -sz};"),
    "25_wrong_radius": ("u = u + w * (v[r * axis_step[a]] + v[-r * axis_step[a]]);",
                        "u = u + w * (v[r * axis_step[a]] + v[-(r == 3 ? 2 : r) * axis_step[a]]);"),
    "25_transposed_weight": ("const int q = 3 * (r - 1) + a + 1;", "const int q = 4 * a + r;"),
    "25_wrong_offset": ("u = u + w * (v[r * axis_step[a]] + v[-r * axis_step[a]]);",
                        "u = u + w * (v[r * axis_step[a]] + v[r * axis_step[a]]);"),
    "25_dropped_radius": ("for (int r = 1; r <= 4; r++)", "for (int r = 1; r <= 3; r++)"),
    "25v_constant_weight": ("const REAL w = kind == ORACLE_25C ? c[q] : C[q][o];",
                            "const REAL w = kind == ORACLE_25C ? c[q] : C[q][0];"),
    "7v_weight_at_wrong_point": ("u = C[0][o] * v[0];", "u = C[0][o + 1] * v[0];"),
    "no_buffer_swap": ("const REAL *V = (t % 2 == 0) ? buf0 : buf1;",
                       "const REAL *V = buf0;"),
    "short_x_loop": ("for (int i = h; i < h + nx; i++)", "for (int i = h; i < h + nx - 1; i++)"),
}


def _build_mutant(tmp_path, name, old, new):
    d = tmp_path / name
    d.mkdir()
    for f in ("stencil_oracle.c", "oracle_body.h"):
        shutil.copy(os.path.join(oracle.HERE, f), d / f)
    body = (d / "oracle_body.h").read_text()
    assert body.count(old) >= 1, "mutation anchor for %s not found" % name
    (d / "oracle_body.h").write_text(body.replace(old, new, 1))
    so = d / "liboracle_mutant.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                           str(d / "stencil_oracle.c"), "-o", str(so)])
    return str(so)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(tmp_path, name):
    old, new = MUTANTS[name]
    lib = _build_mutant(tmp_path, name, old, new)

    def run(kind, u0, coeffs, T, halo=None):
        return oracle.run(kind, u0, coeffs, T, halo=halo, lib_path=lib)

    caught = []
    for pin in P.EVERY_PIN:
        try:
            pin(run)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, "no pin caught mutant %s" % name
