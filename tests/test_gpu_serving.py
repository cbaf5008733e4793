"""Serving (tor_submit / tor_poll): chunked continuous batching on the GPU.

A request larger than one launch's budget is split into root ranges over
several persistent launches, and requests that arrive while it runs join
the next launch.  Each served result must equal the same matrix evaluated
alone (tor_eval) bit for bit: every term is a double of magnitude >= 1 and
the double-double sums are exact, so the value does not depend on how the
subsets were split over roots and launches (only the FP64 sum of |t| may
differ in its last bits).  One large request is also checked against the
stored oracle value of the same matrix (Eq. 2) at the tolerance of
tests/bounds.py.
"""
import json
import os
import sys
import time

import numpy as np
import pytest

from paper_2109_04528_amd import inputs as gen
import bounds

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "oracle_values.json")))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def collect(ctx, tickets, limit_s=120.0):
    got = {}
    t0 = time.time()
    while len(got) < len(tickets) and time.time() - t0 < limit_s:
        for t in tickets:
            if t not in got:
                r = ctx.poll(t)
                if r is not None:
                    got[t] = r
        time.sleep(0.0005)
    assert len(got) == len(tickets), f"{len(tickets) - len(got)} requests unfinished after {limit_s} s"
    return got


def same_value(a, b):
    return (a.tor, a.tor_lo, a.path, a.status) == (b.tor, b.tor_lo, b.path, b.status)


def reference_n30():
    """The n = 30 precision workload and its most accurate stored oracle value."""
    name = "prec_n30_s0_ld" if "prec_n30_s0_ld" in GOLD else "prec_n30_s0"
    g = GOLD[name]
    O = gen.random_O(g["n"], g["seed"], g["r_lo"], g["r_hi"], g["eta"])
    assert gen.sha256(O) == g["sha256"]
    return O, g


def test_chunked_large_requests_with_a_second_wave():
    """Requests of n = 25..30 split over many launches (chunks of 2^23
    subsets, no express launches), small ones among them, and a second wave
    submitted while the first is still pending."""
    from paper_2109_04528_amd import Context
    O30, g30 = reference_n30()
    state = gen.random_O(40, 7001, 0.5, 1.0, 0.8)
    rng = np.random.default_rng(17)

    def click(n):
        return gen.click_submatrix(state, sorted(rng.choice(40, size=n, replace=False).tolist()))

    big1 = [O30, click(26)]
    big2 = [click(25), click(27)]
    small1 = [click(int(rng.integers(8, 21))) for _ in range(10)]
    small2 = [click(int(rng.integers(8, 21))) for _ in range(10)]
    with Context(device=0) as ctx:
        ctx.serve_config(chunk_subsets=1 << 23, oldest_share=0.5, express_subsets=0)
        say("case serving chunked: wave 1 (n=30, 26 and 10 small)")
        w1 = big1 + small1
        t1 = [ctx.submit(O) for O in w1]
        # the n = 30 request takes 2^30 / 2^23 launches at least: it is
        # still running when the second wave arrives
        assert ctx.poll(t1[0]) is None
        say("case serving chunked: wave 2 (n=25, 27 and 10 small) while wave 1 is pending")
        w2 = big2 + small2
        t2 = [ctx.submit(O) for O in w2]
        got = collect(ctx, t1 + t2)
        say("case serving chunked: comparing with tor_eval alone")
        for O, t in zip(w1 + w2, t1 + t2):
            n = O.shape[0] // 2
            alone = ctx.eval(O)
            r = got[t]
            assert r.status == 0
            assert same_value(r, alone), (n, r, alone)
            if n >= 25:
                say(f"  n={n}: launches={r.launches} tor={r.value!r}")
                assert r.launches >= 2
            assert abs(r.sum_abs - alone.sum_abs) <= 1e-12 * alone.sum_abs
        r30 = got[t1[0]]
        want = g30["tor_hi"] + g30["tor_lo"]
        unit = bounds.UNIT_OF_MODE[g30["oracle_mode"]]
        tol = bounds.sum_bound(g30["sum_sq"], bounds.U64, unit)
        say(f"  n=30 served vs oracle ({g30['oracle_mode']}): diff={abs(r30.value - want):.3e} "
            f"bound={tol:.3e} ({tol / abs(want):.2e} relative)")
        assert tol <= 1e-2 * abs(want)
        assert abs(r30.value - want) <= tol


def test_chunking_forced_at_small_n():
    """The same policy at n <= 20: chunks of 2^12 subsets and no express
    launches split every request with more than two roots over several
    launches, in two waves."""
    from paper_2109_04528_amd import Context
    ns = [12, 16, 20, 14, 18, 13, 19, 15]
    mats = [gen.random_O(n, 900 + i, 0.5, 1.0, 0.7) for i, n in enumerate(ns)]
    with Context(device=0) as ctx:
        ctx.serve_config(chunk_subsets=1 << 12, oldest_share=0.25, express_subsets=0)
        say("case serving forced chunking, n in [12, 20]")
        ta = [ctx.submit(O) for O in mats[:4]]
        tb = [ctx.submit(O) for O in mats[4:]]
        got = collect(ctx, ta + tb)
        for O, t in zip(mats, ta + tb):
            alone = ctx.eval(O)
            r = got[t]
            say(f"  n={O.shape[0] // 2}: launches={r.launches}")
            assert same_value(r, alone)
            if O.shape[0] // 2 >= 14:
                assert r.launches >= 2


def test_express_and_chunked_in_one_stream():
    """Default express threshold with a small chunk: small requests run whole
    in express launches (beside the chunked ones), large ones are chunked;
    all equal alone."""
    from paper_2109_04528_amd import Context
    state = gen.random_O(40, 7002, 0.5, 1.0, 0.6)
    rng = np.random.default_rng(23)
    ns = [26, 9, 12, 25, 17, 22, 10, 24, 11, 26]
    mats = [gen.click_submatrix(state, sorted(rng.choice(40, size=n, replace=False).tolist())) for n in ns]
    with Context(device=0) as ctx:
        ctx.serve_config(chunk_subsets=1 << 22, oldest_share=0.5, express_subsets=1 << 20)
        say("case serving express + chunked")
        ts = [ctx.submit(O) for O in mats]
        got = collect(ctx, ts)
        for O, t in zip(mats, ts):
            n = O.shape[0] // 2
            r = got[t]
            assert same_value(r, ctx.eval(O))
            if n <= 20:
                assert r.launches == 1  # whole, in an express launch
            elif n >= 24:
                assert r.launches >= 2  # 2^24 subsets or more, in chunks of 2^22


def test_serve_config_rejects_bad_values():
    from paper_2109_04528_amd import Context, TorError
    with Context(device=0) as ctx:
        for kw in ({"chunk_subsets": 100}, {"express_subsets": -1}, {"oldest_share": 1.5},
                   {"max_queue": 0}):
            with pytest.raises(TorError):
                ctx.serve_config(**kw)


def test_destroy_with_requests_in_flight():
    """Closing a context while its scheduler has work: the launch on the GPU
    finishes, the requests still waiting are dropped, and the call returns
    after that scheduler round, not after the 9 s of work that was queued.
    The device stays usable (a new context evaluates as before)."""
    from paper_2109_04528_amd import Context
    big = [gen.random_O(n, 700 + n, 0.5, 1.0, 0.7) for n in (32, 32, 31, 31, 30, 30)]
    small = [gen.random_O(n, 720 + n, 0.5, 1.0, 0.7) for n in range(8, 20)]
    probe = gen.random_O(16, 740, 0.5, 1.0, 0.7)
    with Context(device=0) as ref:
        want = ref.eval(probe)
    say("case destroy with requests in flight")
    c = Context(device=0)
    for O in big * 250 + small:
        c.submit(O)
    time.sleep(0.05)  # the scheduler is inside its first launches
    t0 = time.perf_counter()
    c.close()
    dt = time.perf_counter() - t0
    say(f"  close took {1e3 * dt:.1f} ms with about 9 s of queued work")
    assert dt < 1.0
    with Context(device=0) as again:
        got = again.eval(probe)
    assert same_value(got, want)


def test_both_paths_and_the_double_double_factor_served():
    """Requests of both arithmetic paths in one stream (Gaussian-state
    matrices on the real quadrature form, general Hermitian ones on the
    complex form), chunked: every result equals the same matrix evaluated
    alone, bit for bit.  A double-double context serving its own: its terms
    are double-doubles, whose sums are not exact, and serving splits a
    request into finer roots than a lone evaluation, so the two results
    agree to the double-double rounding of the sum (2^-90 of sum |t|)."""
    from paper_2109_04528_amd import TOR_FACTOR_DD, Context
    real = [gen.random_O(n, 950 + n, 0.5, 1.0, 0.7) for n in (22, 13, 25)]
    herm = [gen.random_hpd_O(n, 960 + n, 0.05, 0.9) for n in (21, 11, 24)]
    mats = [real[0], herm[0], real[1], herm[1], real[2], herm[2]]
    with Context(device=0) as ctx:
        ctx.serve_config(chunk_subsets=1 << 21, oldest_share=0.5, express_subsets=1 << 14)
        say("case serving both paths")
        ts = [ctx.submit(O) for O in mats]
        got = collect(ctx, ts)
        paths = []
        for O, t in zip(mats, ts):
            r = got[t]
            paths.append(r.path)
            assert same_value(r, ctx.eval(O))
        assert paths == [1, 2, 1, 2, 1, 2]
        assert got[ts[4]].launches >= 2 and got[ts[5]].launches >= 2
    dd = [gen.random_O(n, 970 + n, 0.5, 1.0, 0.7) for n in (18, 10, 22)]
    with Context(device=0, flags=TOR_FACTOR_DD) as qctx:
        qctx.serve_config(chunk_subsets=1 << 19, oldest_share=0.5, express_subsets=1 << 12)
        say("case serving, double-double factor")
        ts = [qctx.submit(O) for O in dd]
        got = collect(qctx, ts)
        for O, t in zip(dd, ts):
            r, alone = got[t], qctx.eval(O)
            assert r.path == 3 and r.status == 0
            d = abs((r.tor - alone.tor) + (r.tor_lo - alone.tor_lo))
            assert d <= 2.0 ** -90 * alone.sum_abs, (d, alone.sum_abs)
        assert got[ts[2]].launches >= 2
