"""GPU results against stored oracle values (tests/golden/oracle_values.json,
written by tests/golden/make_golden.py from the CPU oracle only).

The inputs are regenerated from their seeds and checked byte-for-byte against
the stored SHA-256 first, so a generator change cannot pass silently.  The
tolerance is the FP64 term bound of test_gpu_parity (every term rounded once
by each side, sums exact), and the precision report prints the measured
relative error next to the cancellation R = sum|t| / |Tor|.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_2109_04528_amd import inputs as gen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "oracle_values.json")))
U = 2.0 ** -53


def kappa(O):
    C = np.eye(O.shape[0]) - O
    C = np.tril(C) + np.tril(C, -1).conj().T
    w = np.linalg.eigvalsh(C)
    return float(w[-1] / w[0])


@pytest.fixture(scope="module")
def ctx():
    from paper_2109_04528_amd import Context
    c = Context(device=0)
    yield c
    c.close()


@pytest.mark.parametrize("name", sorted(GOLD))
def test_against_golden(ctx, name):
    g = GOLD[name]
    O = gen.random_O(g["n"], g["seed"], g["r_lo"], g["r_hi"], g["eta"])
    assert gen.sha256(O) == g["sha256"], "generator output changed"
    print(f"case golden {name}", flush=True)
    r = ctx.eval(O)
    want = g["tor_hi"] + g["tor_lo"]
    err = abs(r.value - want)
    bound = 8.0 * max(g["n"], 10) * kappa(O) * U * g["sum_abs"]
    rel = err / abs(want)
    R = g["sum_abs"] / abs(want)
    print(f"  {name}: gpu={r.value!r} oracle({g['oracle_mode']})={want!r} rel={rel:.3e} R={R:.3e} "
          f"u*R/sqrt(2^n)={U * R / np.sqrt(2.0 ** g['n']):.2e} ms={r.device_ms:.2f}", flush=True)
    assert abs(r.sum_abs - g["sum_abs"]) <= 1e-9 * g["sum_abs"]
    assert err <= bound
    if g["n"] <= 10:
        assert rel <= 1e-10  # the target precision, reachable at this R


def test_dd_beats_plain_fp64_sum():
    """Double-double vs plain FP64 accumulation of the same terms, against
    __float128 at n = 20 (R ~ 1e10): the plain sum adds its own rounding on
    top of the per-term floor."""
    from paper_2109_04528_amd import Context
    errs = {}
    for accum in ("dd", "fp64"):
        with Context(device=0, accum=accum) as c:
            e = []
            for s in range(4):
                g = GOLD[f"prec_n20_s{s}"]
                O = gen.random_O(20, s, 0.3, 1.2, 0.9)
                want = g["tor_hi"] + g["tor_lo"]
                e.append(abs(c.eval(O).value - want) / abs(want))
            errs[accum] = e
    print("  rel errors dd:", ["%.2e" % v for v in errs["dd"]], "fp64 sum:", ["%.2e" % v for v in errs["fp64"]],
          flush=True)
    assert np.median(errs["dd"]) <= np.median(errs["fp64"])
