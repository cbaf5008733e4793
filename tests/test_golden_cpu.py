"""CPU checks of the stored oracle values (tests/golden/oracle_values.json):
the generator still produces the stored inputs, every entry carries what the
GPU tests need, and the FP64 and extended-precision references of the same
matrix differ by no more than the FP64 floor -- the error model the GPU
tolerances (tests/bounds.py) rest on, pinned without the GPU."""
import json
import math
import os

import pytest

import bounds
from paper_2109_04528_amd import inputs as gen

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "oracle_values.json")))


@pytest.mark.parametrize("name", sorted(GOLD))
def test_entry_is_complete_and_reproducible(name):
    g = GOLD[name]
    for key in ("n", "seed", "r_lo", "r_hi", "eta", "oracle_mode", "sha256", "tor_hi", "tor_lo", "sum_abs",
                "sum_sq", "subsets"):
        assert key in g, key
    assert g["subsets"] == 1 << g["n"]
    assert g["oracle_mode"] in bounds.UNIT_OF_MODE
    # sum t^2 <= (sum |t|)^2 and sum t^2 >= (sum |t|)^2 / 2^n (Cauchy-Schwarz)
    assert g["sum_sq"] <= g["sum_abs"] ** 2 * (1 + 1e-12)
    assert g["sum_sq"] >= g["sum_abs"] ** 2 / 2.0 ** g["n"] * (1 - 1e-12)
    if g["n"] <= 24:  # the larger input's generator is checked by the GPU tests
        O = gen.random_O(g["n"], g["seed"], g["r_lo"], g["r_hi"], g["eta"])
        assert gen.sha256(O) == g["sha256"]


def test_fp64_oracle_within_its_floor_of_extended():
    pairs = [n for n in sorted(GOLD) if n.endswith("_ld") and n[:-3] in GOLD]
    assert len(pairs) >= 8
    worst = 0.0
    for name in pairs:
        e, f = GOLD[name], GOLD[name[:-3]]
        assert e["sha256"] == f["sha256"]
        ve, vf = e["tor_hi"] + e["tor_lo"], f["tor_hi"] + f["tor_lo"]
        scale = bounds.U64 * math.sqrt(e["sum_sq"])
        tol = bounds.sum_bound(e["sum_sq"], bounds.U64, bounds.ULD)
        worst = max(worst, abs(vf - ve) / scale)
        assert abs(vf - ve) <= tol, (name, vf, ve, tol)
        assert abs(e["sum_abs"] - f["sum_abs"]) <= 1e-12 * e["sum_abs"]
    # and the model is not vacuous: the FP64 oracle does carry an error of
    # the order of u sqrt(sum t^2)
    assert worst > 0.3


def test_extended_oracle_within_its_floor_of_quad():
    """The x87 extended reference of an n = 24 matrix against the __float128
    one of the same matrix: they differ by about the extended rounding of
    each term, 2^-64 sqrt(sum t^2), which is the floor the n = 24 and n = 30
    extended references carry."""
    pairs = [n for n in sorted(GOLD) if n.endswith("_q") and n[:-2] + "_ld" in GOLD]
    assert pairs
    for name in pairs:
        q, e = GOLD[name], GOLD[name[:-2] + "_ld"]
        assert q["sha256"] == e["sha256"] and q["oracle_mode"] == "quad" and e["oracle_mode"] == "ld"
        vq, ve = q["tor_hi"] + q["tor_lo"], e["tor_hi"] + e["tor_lo"]
        tol = bounds.sum_bound(q["sum_sq"], bounds.ULD, bounds.UQ)
        assert abs(ve - vq) <= tol, (name, ve, vq, tol)
        # not vacuous: the extended value does carry its own rounding
        assert abs(ve - vq) >= 0.05 * bounds.ULD * math.sqrt(q["sum_sq"])
        assert abs(q["sum_abs"] - e["sum_abs"]) <= 1e-15 * q["sum_abs"]
