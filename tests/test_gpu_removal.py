"""The paper's removal-order kernel (tor_eval_removal, Algorithm 2) against
the oracle: both sides round every term once and sum exactly, so the
tolerance of tests/bounds.py applies (FP64 on the GPU, the oracle's own
precision on the other side)."""
import json
import os
import sys

import numpy as np
import pytest

import bounds
from oracle import oracle as orc
from paper_2109_04528_amd import inputs as gen

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "oracle_values.json")))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2109_04528_amd import Context
    c = Context(device=0)
    yield c
    c.close()


@pytest.mark.parametrize("label,O", [
    ("n1", gen.random_O(1, 2, 0.5, 1.0, 0.7)),
    ("n5", gen.random_O(5, 3, 0.5, 1.0, 0.7)),
    ("n11", gen.random_O(11, 4, 0.3, 1.2, 0.9)),
    ("hpd_n9", gen.random_hpd_O(9, 6)),
    ("hpd_n13", gen.random_hpd_O(13, 7)),
    ("vacuum_n7", gen.vacuum_O(7)),
])
def test_removal_vs_oracle(ctx, label, O):
    say(f"case removal {label}")
    r = ctx.eval_removal(O)
    q = orc.tor(O, mode=orc.QUAD)
    b = bounds.sum_bound(q.sum_sq, bounds.U64, bounds.UQ)
    say(f"  gpu={r.value!r} oracle={q.value!r} diff={abs(r.value - q.value):.3e} bound={b:.3e} ms={r.device_ms:.2f}")
    assert r.status == 0
    assert abs(r.value - q.value) <= b
    assert abs(r.sum_abs - q.sum_abs) <= 1e-12 * q.sum_abs


@pytest.mark.parametrize("name", ["first_n10_s0", "prec_n16_s0", "prec_n20_s0", "pair_n24_s0"])
def test_removal_golden(ctx, name):
    g = GOLD[name]
    O = gen.random_O(g["n"], g["seed"], g["r_lo"], g["r_hi"], g["eta"])
    assert gen.sha256(O) == g["sha256"]
    say(f"case removal golden {name}")
    r = ctx.eval_removal(O)
    want = g["tor_hi"] + g["tor_lo"]
    b = bounds.sum_bound(g["sum_sq"], bounds.U64, bounds.UNIT_OF_MODE[g["oracle_mode"]])
    say(f"  gpu={r.value!r} oracle={want!r} rel={abs(r.value - want) / abs(want):.3e} "
        f"bound_rel={b / abs(want):.3e} ms={r.device_ms:.2f}")
    assert r.status == 0
    assert b <= 1e-2 * abs(want)
    assert abs(r.value - want) <= b


def test_removal_empty_and_errors(ctx):
    from paper_2109_04528_amd import TOR_E_INVAL, TOR_E_NOT_PD, TorError
    assert ctx.eval_removal(gen.vacuum_O(0)).value == 1.0
    with pytest.raises(TorError) as ei:
        ctx.eval_removal(np.eye(12, dtype=np.complex128) * 1.5)
    assert ei.value.code == TOR_E_NOT_PD
    with pytest.raises(TorError) as ei:
        ctx.eval_removal(gen.vacuum_O(35))
    assert ei.value.code == TOR_E_INVAL
