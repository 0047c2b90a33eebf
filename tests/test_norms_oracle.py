"""The oracle's FP64 reductions against closed forms, and planted mistakes in
copies of oracle/norms.py that the pins must catch (no GPU)."""
from __future__ import annotations

import importlib.util
import os

import pytest

import norms_pins as NP
import oracle
from oracle import norms

NORMS_SRC = os.path.join(oracle.HERE, "norms.py")


@pytest.mark.parametrize("pin", NP.EVERY_NORM_PIN, ids=lambda f: f.__name__)
def test_norm_pins(pin):
    pin(norms)


# (anchor, replacement) in oracle/norms.py
MUTANTS = {
    "interior_includes_halo": ("return a[h:a.shape[0] - h, h:a.shape[1] - h, h:a.shape[2] - h]",
                               "return a"),
    "interior_one_layer_short": ("return a[h:a.shape[0] - h, h:a.shape[1] - h, h:a.shape[2] - h]",
                                 "return a[h:a.shape[0] - h, h:a.shape[1] - h, h:a.shape[2] - h - 1]"),
    "missing_sqrt": ("return math.sqrt(math.fsum(v * v)), float(np.max(np.abs(v)))",
                     "return math.fsum(v * v), float(np.max(np.abs(v)))"),
    "max_without_abs": ("return math.sqrt(math.fsum(v * v)), float(np.max(np.abs(v)))",
                        "return math.sqrt(math.fsum(v * v)), float(np.max(v))"),
    "sum_of_abs": ("return math.sqrt(math.fsum(v * v)), float(np.max(np.abs(v)))",
                   "return math.sqrt(math.fsum(np.abs(v))), float(np.max(np.abs(v)))"),
    "residual_sum": ("d = interior(uT, halo).astype(np.float64) - interior(uTm1, halo).astype(np.float64)",
                     "d = interior(uT, halo).astype(np.float64) + interior(uTm1, halo).astype(np.float64)"),
    "diff_wrong_halo": ("- interior(b, halo_b).astype(np.float64)",
                        "- interior(b, halo_a).astype(np.float64)"),
    "residual_in_input_precision": ("d = interior(uT, halo).astype(np.float64) - interior(uTm1, halo).astype(np.float64)",
                                    "d = (interior(uT, halo) - interior(uTm1, halo)).astype(np.float64)"),
}


def _load_mutant(tmp_path, name, old, new):
    src = open(NORMS_SRC).read()
    assert src.count(old) >= 1, "mutation anchor for %s not found" % name
    path = tmp_path / ("norms_%s.py" % name)
    path.write_text(src.replace(old, new, 1))
    spec = importlib.util.spec_from_file_location("norms_mutant_" + name, str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_norm_pins_catch_planted_mistake(tmp_path, name):
    mod = _load_mutant(tmp_path, name, *MUTANTS[name])
    caught = []
    for pin in NP.EVERY_NORM_PIN:
        try:
            pin(mod)
        except (AssertionError, ValueError, IndexError):
            caught.append(pin.__name__)
    assert caught, "no pin caught mutant %s" % name
