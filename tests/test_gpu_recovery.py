"""Recovery from numeric failures of single subtree roots (GPU).

Every root writes its partial sum to a slot of its own, which a later run
of the same root overwrites.  A root that reports a numeric failure (a
non-finite partial with every tested pivot positive) is run once more and
the slots are reduced again in the same fixed order, so a recovered result
must equal a clean one bit for bit.  The failure is forced from the host
(tor_debug_fail_root): root r of the next evaluation's first matrix reports
it in its first `runs` launches.  No kernel faults or waits: the forced root
only writes a NaN and a flag into its own slot.
"""
import sys

import numpy as np
import pytest

from paper_2109_04528_amd import inputs as gen

pytestmark = pytest.mark.gpu

TOR_E_NUMERIC = -3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2109_04528_amd import Context
    c = Context(device=0)
    yield c
    c.close()


@pytest.mark.parametrize("n,root", [(20, 0), (24, 5), (30, 4095)])
def test_recovered_root_equals_clean_run(ctx, n, root):
    O = gen.random_O(n, 3, 0.3, 1.2, 0.9)
    say(f"case recovery n={n} root={root}")
    clean = ctx.eval(O)
    assert clean.launches == 1
    ctx.debug_fail_root(root, runs=1)
    r = ctx.eval(O)
    say(f"  clean={clean.value!r} recovered={r.value!r} launches={r.launches}")
    assert r.status == 0 and r.launches == 2
    assert (r.tor, r.tor_lo, r.sum_abs) == (clean.tor, clean.tor_lo, clean.sum_abs)
    again = ctx.eval(O)  # the request was used up
    assert again.launches == 1 and (again.tor, again.tor_lo) == (clean.tor, clean.tor_lo)


def test_failure_that_persists_is_reported(ctx):
    O = gen.random_O(22, 4, 0.3, 1.2, 0.9)
    say("case recovery persisting failure n=22")
    ctx.debug_fail_root(3, runs=2)
    r = ctx.eval(O, check=False)
    assert r.status == TOR_E_NUMERIC and r.launches == 2
    assert ctx.eval(O).status == 0


def test_partials_after_recovery_equal_clean_partials(ctx):
    O = gen.random_O(24, 5, 0.5, 1.0, 0.7)
    say("case recovery partials n=24")
    k, clean, rc = ctx.eval_partials(O, 8)
    ctx.debug_fail_root(77, runs=1)
    k2, parts, r = ctx.eval_partials(O, 8)
    assert k2 == k and r.status == 0 and r.launches == 2
    assert np.array_equal(parts, clean)


def test_batch_recovers_only_the_failing_matrix(ctx):
    Os = [gen.random_O(n, 10 + n, 0.5, 1.0, 0.7) for n in (18, 26, 21)]
    say("case recovery batch n=18,26,21")
    clean = ctx.eval_batch(Os)
    ctx.debug_fail_root(2, runs=1)  # root 2 of the first matrix (n = 18)
    rs = ctx.eval_batch(Os)
    assert [r.launches for r in rs] == [2, 1, 1]
    for a, b in zip(rs, clean):
        assert a.status == 0 and (a.tor, a.tor_lo, a.sum_abs) == (b.tor, b.tor_lo, b.sum_abs)


def test_root_beyond_the_split_is_ignored(ctx):
    O = gen.random_O(16, 6, 0.5, 1.0, 0.7)
    say("case recovery root out of range n=16")
    ctx.debug_fail_root(1 << 40, runs=1)
    r = ctx.eval(O)
    assert r.status == 0 and r.launches == 1


def test_debug_hook_rejects_bad_runs(ctx):
    from paper_2109_04528_amd import TorError
    with pytest.raises(TorError):
        ctx.debug_fail_root(0, runs=3)
    ctx.debug_fail_root(-1)  # clears
