"""Planted mistakes in copies of oracle/models.py (Eqs. 2-5) that the golden
values of tests/golden/ must catch (no GPU)."""
from __future__ import annotations

import importlib.util
import json
import os

import pytest

import oracle

MODELS_SRC = os.path.join(oracle.HERE, "models.py")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

MUTANTS = {
    "ww_radius_once": ("return Dw - 2 * R + NF", "return Dw - R + NF"),
    "ring_without_radius": ("+ 2 * R * (Dw + Ww))", "+ 2 * (Dw + Ww))"),
    "half_width_radius_dropped": ("ND * Dw * (Dw / 2 - R + NF)", "ND * Dw * (Dw / 2 - 1 + NF)"),
    "frontlines_dropped": ("ND * Dw * (Dw / 2 - R + NF)", "ND * Dw * (Dw / 2 - R)"),
    "balance_radius_dropped": ("return 2 * elem_bytes * R * ((2 * Dw - 2 * R)",
                               "return 2 * elem_bytes * ((2 * Dw - 2 * R)"),
    "balance_reads_per_width": ("+ (ND * Dw + 2 * R))", "+ (ND + 2 * R))"),
}


def golden_checks(models):
    with open(os.path.join(GOLDEN, "cache_block_r4.json")) as f:
        g4 = json.load(f)
    with open(os.path.join(GOLDEN, "cache_block_example.json")) as f:
        g1 = json.load(f)
    assert models.cache_block(g1["Dw"], g1["N_F"], 1.0, g1["R"], g1["N_D"]) == g1["C_S_per_Nxb"]
    for c in g4["cases"]:
        assert models.wavefront_width(c["Dw"], c["N_F"], c["R"]) == c["W_w"]
        assert models.cache_block(c["Dw"], c["N_F"], 1.0, c["R"], c["N_D"]) == c["C_S_per_Nxb"]
        assert models.code_balance(c["Dw"], c["N_D"], c["R"]) == c["B_C_f64"]


def test_golden_on_real_models():
    from oracle import models
    golden_checks(models)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_golden_catches_planted_mistake(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(MODELS_SRC).read()
    assert src.count(old) >= 1, "mutation anchor for %s not found" % name
    path = tmp_path / ("models_%s.py" % name)
    path.write_text(src.replace(old, new, 1))
    spec = importlib.util.spec_from_file_location("models_mutant_" + name, str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with pytest.raises(AssertionError):
        golden_checks(mod)
