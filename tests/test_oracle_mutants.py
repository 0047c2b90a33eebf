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
    "7c_wrong_index": ("+ c[1] * (AT(V, k, j, i + 1) + AT(V, k, j, i - 1))",
                       "+ c[1] * (AT(V, k, j, i + 1) + AT(V, k, j, i + 1))"),
    "7c_dropped_z_pair": ("+ c[1] * (AT(V, k + 1, j, i) + AT(V, k - 1, j, i));",
                          ";"),
    "7c_wrong_centre_weight": ("u = c[0] * AT(V, k, j, i)\n                      + c[1]",
                               "u = c[1] * AT(V, k, j, i)\n                      + c[1]"),
    "7v_transposed_axis": ("+ AT(C[3], k, j, i) * AT(V, k, j + 1, i)",
                           "+ AT(C[3], k, j, i) * AT(V, k + 1, j, i)"),
    "7v_wrong_sign": ("+ AT(C[6], k, j, i) * AT(V, k - 1, j, i);",
                      "- AT(C[6], k, j, i) * AT(V, k - 1, j, i);"),
    "7v_swapped_weights": ("+ AT(C[1], k, j, i) * AT(V, k, j, i + 1)\n                      + AT(C[2], k, j, i) * AT(V, k, j, i - 1)",
                           "+ AT(C[2], k, j, i) * AT(V, k, j, i + 1)\n                      + AT(C[1], k, j, i) * AT(V, k, j, i - 1)"),
    "25c_wrong_radius": ("+ c[8] * (AT(V, k, j + 3, i) + AT(V, k, j - 3, i))",
                         "+ c[8] * (AT(V, k, j + 2, i) + AT(V, k, j - 3, i))"),
    "25c_transposed_weight": ("+ c[10] * (AT(V, k, j, i + 4) + AT(V, k, j, i - 4))\n                      + c[11]",
                              "+ c[11] * (AT(V, k, j, i + 4) + AT(V, k, j, i - 4))\n                      + c[10]"),
    "25v_wrong_offset": ("AT(C[12], k, j, i) * (AT(V, k + 4, j, i) + AT(V, k - 4, j, i))",
                         "AT(C[12], k, j, i) * (AT(V, k + 4, j, i) + AT(V, k + 4, j, i))"),
    "25v_dropped_term": ("+ AT(C[5], k, j, i) * (AT(V, k, j + 2, i) + AT(V, k, j - 2, i))",
                         ""),
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
