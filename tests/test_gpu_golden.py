"""GPU results against stored oracle values (tests/golden/oracle_values.json,
written by tests/golden/make_golden.py from the CPU oracle only).

The inputs are regenerated from their seeds and checked byte for byte
against the stored SHA-256 first, so a generator change cannot pass
silently.  Full sums are compared at the tolerance of tests/bounds.py: a
few standard deviations of the independent per-term roundings of both
sides, RHO sqrt(u_gpu^2 + u_oracle^2) sqrt(sum t^2) each.  Every test also
asserts that its bound is at most 1 % of |Tor|, so a wrong sign, a zero or a
missing term cannot pass.  The stored references: __float128 at n <= 20, and
at n = 24 and 30 both the FP64 oracle and the x87 extended one (64-bit
significands), which is accurate enough to pin the double-double factor.
"""
import json
import os
import sys

import numpy as np
import pytest

import bounds
from paper_2109_04528_amd import inputs as gen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "oracle_values.json")))
ACCURATE = sorted(k for k, g in GOLD.items() if g["oracle_mode"] in ("quad", "ld"))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def load(name):
    g = GOLD[name]
    O = gen.random_O(g["n"], g["seed"], g["r_lo"], g["r_hi"], g["eta"])
    assert gen.sha256(O) == g["sha256"], "generator output changed"
    return O, g, g["tor_hi"] + g["tor_lo"]


@pytest.fixture(scope="module")
def ctx():
    from paper_2109_04528_amd import Context
    c = Context(device=0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def qctx():
    from paper_2109_04528_amd import Context, TOR_FACTOR_DD
    c = Context(device=0, flags=TOR_FACTOR_DD)
    yield c
    c.close()


@pytest.mark.parametrize("name", sorted(GOLD))
def test_fp64_path_against_golden(ctx, name):
    O, g, want = load(name)
    say(f"case golden {name} (FP64 factor)")
    r = ctx.eval(O)
    err = abs(r.value - want)
    tol = bounds.sum_bound(g["sum_sq"], bounds.U64, bounds.UNIT_OF_MODE[g["oracle_mode"]])
    R = g["sum_abs"] / abs(want)
    say(f"  {name}: gpu={r.value!r} oracle({g['oracle_mode']})={want!r} rel={err / abs(want):.3e} "
        f"bound_rel={tol / abs(want):.3e} R={R:.3e} err_est={r.err_est:.2e} ms={r.device_ms:.2f}")
    assert r.status == 0
    assert tol <= 1e-2 * abs(want)
    assert err <= tol
    assert abs(r.sum_abs - g["sum_abs"]) <= 1e-9 * g["sum_abs"]
    if g["n"] <= 10:
        assert err <= 1e-10 * abs(want)  # the target precision, reachable at this R


@pytest.mark.parametrize("name", ACCURATE)
def test_double_double_factor_against_golden(qctx, name):
    """TOR_FACTOR_DD against the __float128 and extended references: at
    n = 30 the bound is set by the extended oracle's own rounding, about
    1e-8 relative, where the FP64 floor is about 1e-6."""
    O, g, want = load(name)
    say(f"case golden {name} (double-double factor)")
    r = qctx.eval(O)
    d = (r.tor - g["tor_hi"]) + (r.tor_lo - g["tor_lo"])
    tol = bounds.sum_bound(g["sum_sq"], bounds.UDD, bounds.UNIT_OF_MODE[g["oracle_mode"]])
    say(f"  {name}: rel={abs(d) / abs(want):.3e} bound_rel={tol / abs(want):.3e} "
        f"err_est={r.err_est:.2e} ms={r.device_ms:.2f}")
    assert r.status == 0 and r.path == 3
    assert tol <= 1e-6 * abs(want)
    assert abs(d) <= tol


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
                O, g, want = load(f"prec_n20_s{s}")
                e.append(abs(c.eval(O).value - want) / abs(want))
            errs[accum] = e
    say("  rel errors dd:", ["%.2e" % v for v in errs["dd"]], "fp64 sum:", ["%.2e" % v for v in errs["fp64"]])
    assert np.median(errs["dd"]) <= np.median(errs["fp64"])
