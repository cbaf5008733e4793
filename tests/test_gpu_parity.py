"""GPU parity: the recursive HIP path (through the C ABI) against the CPU oracle.

Tolerances.  Every term t_Z = (-1)^(n-|Z|)/sqrt(det) is formed by both
sides through different but backward-stable factorisation orders, so each
term carries a small relative rounding error of either sign, independent
between subsets and sides.  The sums themselves add no error (double-double
on the GPU, __float128 in the oracle), so the difference of two full or
subtree sums is bounded statistically by tests/bounds.py: SIGMAS standard
deviations of RHO sqrt(u_gpu^2 + u_oracle^2) sqrt(sum t^2).  Only the plain
FP64 accumulation mode, which adds its own summation error, keeps the
worst-case bound c N kappa u sum|t|.  Where the result allows it, the tests
ask for the target precision of 1e-10.
"""
import math
import sys

import numpy as np
import pytest

import bounds
from oracle import oracle as orc
from paper_2109_04528_amd import inputs as gen

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2109_04528_amd import Context
    c = Context(device=0)
    yield c
    c.close()


def kappa(O):
    n2 = O.shape[0]
    C = np.eye(n2) - O
    C = np.tril(C) + np.tril(C, -1).conj().T
    w = np.linalg.eigvalsh(C)
    return float(w[-1] / w[0])


def term_bound(O, sum_abs):
    """Worst case c N kappa u sum|t|: for the plain FP64 accumulation only."""
    n = O.shape[0] // 2
    return 8.0 * max(n, 9) * kappa(O) * U * sum_abs


def tol(q, mode):
    """FP64 GPU sum against an oracle sum q computed in `mode`."""
    return bounds.sum_bound(q.sum_sq, bounds.U64, bounds.UQ if mode == orc.QUAD else bounds.U64)


def tol_terms(ts):
    """FP64 GPU sum against the exact sum of the FP64 oracle terms ts."""
    return bounds.sum_bound(sum(t * t for t in ts), bounds.U64, bounds.U64)


def check(ctx, O, mode=orc.QUAD, label=""):
    say(f"case {label}: n={O.shape[0] // 2}")
    r = ctx.eval(O)
    q = orc.tor(O, mode=mode)
    err = abs(r.value - q.value)
    bound = tol(q, mode)
    rel = err / abs(q.value) if q.value else err
    say(f"  gpu={r.value!r} oracle={q.value!r} rel={rel:.3e} R={q.cancellation:.3e} "
        f"bound_rel={bound / max(abs(q.value), 1e-300):.3e} ms={r.device_ms:.3f}")
    assert r.status == 0
    assert err <= bound, (label, r.value, q.value, err, bound)
    # sum of |t| over the input's own subsets (padding modes scale it by 3
    # each on the device; the library divides that back out)
    n = O.shape[0] // 2
    assert abs(r.sum_abs - q.sum_abs) <= max(1e-9, 8.0 * max(n, 9) * kappa(O) * U) * q.sum_abs
    return r, q


def test_math_probe(ctx):
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(1e-6, 1.0, 4000), 10.0 ** rng.uniform(-60, 0, 4000),
                        np.array([1.0, 0.25, 0.5, 2.0 ** -40])])
    say("case math_probe")
    out = ctx.debug_math(x)
    xl = x.astype(np.longdouble)
    rs = (1 / np.sqrt(xl)).astype(np.float64)
    rc = (1 / xl).astype(np.float64)

    def ulps(a, b):
        return np.abs(a.view(np.int64) - b.view(np.int64))

    say(f"  raw seed error (ulps): rsq max {ulps(out[:, 2], rs).max()}, rcp max {ulps(out[:, 3], rc).max()}")
    assert ulps(out[:, 0], rs).max() <= 1
    assert ulps(out[:, 1], rc).max() <= 1


def test_fma_peak_probe(ctx):
    """The FP64 FMA probe reaches a throughput of the order of the published
    vector peak (78.6 TFLOP/s): more than half of it, and not above it by
    more than the clock's headroom."""
    tf, ms = ctx.fma_peak(2048)
    say(f"case fma peak: {tf:.1f} TFLOP/s in {ms:.3f} ms")
    assert 39.3 < tf < 100.0


@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 8, 9, 10, 11, 12, 13])
def test_small_n_against_quad(ctx, n):
    O = gen.random_O(n, 100 + n, 0.5, 1.0, 0.7) if n else gen.vacuum_O(0)
    if n == 0:
        r = ctx.eval(O)
        assert r.value == 1.0
        return
    check(ctx, O, label=f"small n={n}")


def test_first_workload_meets_1e10(ctx):
    # n = 10, r ~ U[.5, 1], Haar U, eta = .5, seed 0: 1024 subsets
    O = gen.random_O(10, 0, 0.5, 1.0, 0.5)
    r, q = check(ctx, O, label="n=10 seed 0")
    assert abs(r.value - q.value) <= 1e-10 * abs(q.value)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_precision_workload_n16_against_quad(ctx, seed):
    # r ~ U[.3, 1.2], eta = .9: strong cancellation
    O = gen.random_O(16, seed, 0.3, 1.2, 0.9)
    check(ctx, O, label=f"n=16 eta=.9 seed {seed}")


@pytest.mark.parametrize("n", [10, 12, 14])
def test_generic_hermitian_input(ctx, n):
    # no Gaussian-state structure: the general complex path
    O = gen.random_hpd_O(n, 7 + n, 0.05, 0.9)
    check(ctx, O, label=f"generic HPD n={n}")


def test_vacuum_is_exactly_zero(ctx):
    for n in (4, 9, 17, 30):
        say(f"case vacuum n={n}")
        assert ctx.eval(gen.vacuum_O(n)).value == 0.0


def product_closed_form(O):
    """Exact Tor, sum |t| and sum t^2 of a product-state input (a direct sum
    of single-mode 2x2 blocks of I - O), from the input's own FP64 entries in
    50-digit arithmetic: t_Z = (-1)^(n-|Z|) prod_{i in Z} a_i with
    a_i = 1/sqrt(det (I - O)_i), so Tor = prod (a_i - 1),
    sum |t| = prod (1 + a_i) and sum t^2 = prod (1 + a_i^2)."""
    import mpmath as mp
    mp.mp.dps = 50
    n = O.shape[0] // 2
    blocks = np.zeros_like(O, dtype=bool)
    for i in range(n):
        for x in (i, i + n):
            for y in (i, i + n):
                blocks[x, y] = True
    assert np.all(O[~blocks] == 0)  # a direct sum of the modes, exactly
    tor, sabs, ssq = mp.mpf(1), mp.mpf(1), mp.mpf(1)
    for i in range(n):
        c11 = 1 - mp.mpf(float(O[i, i].real))
        c22 = 1 - mp.mpf(float(O[i + n, i + n].real))
        c21 = mp.mpc(-float(O[i + n, i].real), -float(O[i + n, i].imag))  # lower triangle
        a = 1 / mp.sqrt(c11 * c22 - abs(c21) ** 2)
        tor *= a - 1
        sabs *= 1 + a
        ssq *= 1 + a * a
    return tor, sabs, ssq


def test_product_state_n30_closed_form(ctx):
    """n = 30 product state, R = 1.4e28: far beyond what an FP64 factor can
    resolve (its floor u sqrt(sum t^2) / |Tor| is 7e7), so the value is
    checked on the double-double factor against the exact closed form of the
    input, at a tolerance from 2^-100 sqrt(sum t^2) (1e-5 relative); the FP64
    path's sum |t| is checked against its closed form."""
    import mpmath as mp
    from paper_2109_04528_amd import Context, TOR_FACTOR_DD
    rng = np.random.default_rng(30)
    r = rng.uniform(0.3, 1.2, 30)
    eta = 0.9
    O = gen.structured_O(gen.product_state_O(r, eta, rng.uniform(0, 2 * np.pi, 30)))
    tor, sabs, ssq = product_closed_form(O)
    say("case product state n=30")
    with Context(device=0, flags=TOR_FACTOR_DD) as qc:
        rq = qc.eval(O)
    d = float(mp.mpf(rq.tor) + mp.mpf(rq.tor_lo) - tor)
    b = bounds.sum_bound(float(ssq), bounds.UDD) + 4 * bounds.UDD * abs(float(tor))
    rf = ctx.eval(O)
    say(f"  dd={rq.value!r} closed={float(tor)!r} rel={abs(d) / abs(float(tor)):.3e} "
        f"bound_rel={b / abs(float(tor)):.3e} R={float(sabs / abs(tor)):.3e} ms={rq.device_ms:.2f}; "
        f"FP64 path {rf.value!r} (err_est {rf.err_est:.1e})")
    assert rq.status == 0 and rq.path == 3
    assert b <= 1e-2 * abs(float(tor))
    assert abs(d) <= b
    assert abs(rq.sum_abs - float(sabs)) <= 1e-12 * float(sabs)
    assert rf.status == 0
    assert abs(rf.sum_abs - float(sabs)) <= 1e-9 * float(sabs)


def test_n30_partials_sampled_against_oracle(ctx):
    # full-size precision workload: n = 30, r ~ U[.3, 1.2], eta = .9, seed 0
    O = gen.random_O(30, 0, 0.3, 1.2, 0.9)
    say("case n=30 partials")
    k, parts, res = ctx.eval_partials(O, 12)
    say(f"  k={k} tor={res.value!r} R={res.cancellation:.3e} ms={res.device_ms:.2f}")
    assert k == 12 and res.status == 0
    # the partials are the exact pieces of the total
    hi = 0.0
    lo = 0.0
    for h, l_, _ in parts:
        s = hi + h
        bb = s - hi
        e = (hi - (s - bb)) + (h - bb)
        hi = s
        lo += e + l_
    assert abs((hi + lo) - res.value) <= 1e-12 * res.sum_abs
    rng = np.random.default_rng(1)
    for root in [0, (1 << k) - 1] + [int(v) for v in rng.integers(1, (1 << k) - 1, 2)]:
        q = orc.tor(O, mode=orc.F64, fix_mask=(1 << k) - 1, fix_val=root)
        got = parts[root, 0] + parts[root, 1]
        bound = tol(q, orc.F64)
        say(f"  root {root}: gpu={got!r} oracle={q.value!r} diff={abs(got - q.value):.3e} bound={bound:.3e}")
        assert q.count == 1 << (30 - k)
        assert abs(got - q.value) <= bound
        assert abs(parts[root, 2] - q.sum_abs) <= 1e-12 * q.sum_abs


@pytest.mark.parametrize("label,n,gen_fn", [
    ("complex path, precision workload", 30, lambda: gen.random_O(30, 0, 0.3, 1.2, 0.9)),
    ("complex path, generic HPD", 26, lambda: gen.random_hpd_O(26, 77, 0.05, 0.9)),
])
def test_complex_path_partials_sampled_against_oracle(label, n, gen_fn):
    # the general Hermitian path at full size: subtrees against the oracle
    # restricted to the same roots
    from paper_2109_04528_amd import Context, TOR_FORCE_COMPLEX
    O = gen_fn()
    say(f"case {label} n={n} partials")
    with Context(device=0, flags=TOR_FORCE_COMPLEX) as c:
        k, parts, res = c.eval_partials(O, 12)
    say(f"  k={k} tor={res.value!r} R={res.cancellation:.3e} ms={res.device_ms:.2f} path={res.path}")
    assert k == 12 and res.status == 0 and res.path == 2
    rng = np.random.default_rng(2)
    for root in [0, (1 << k) - 1] + [int(v) for v in rng.integers(1, (1 << k) - 1, 2)]:
        q = orc.tor(O, mode=orc.F64, fix_mask=(1 << k) - 1, fix_val=root)
        got = parts[root, 0] + parts[root, 1]
        bound = tol(q, orc.F64)
        say(f"  root {root}: gpu={got!r} oracle={q.value!r} diff={abs(got - q.value):.3e} bound={bound:.3e}")
        assert q.count == 1 << (n - k)
        assert abs(got - q.value) <= bound
        assert abs(parts[root, 2] - q.sum_abs) <= 1e-12 * q.sum_abs


def test_batch_is_bitwise_equal_to_single(ctx):
    ns = [12, 9, 15, 3, 11, 0, 14]
    Os = [gen.random_O(n, 200 + i, 0.5, 1.0, 0.3 + 0.1 * i) if n else gen.vacuum_O(0) for i, n in enumerate(ns)]
    say("case batch vs single")
    batch = ctx.eval_batch(Os)
    for O, b in zip(Os, batch):
        s = ctx.eval(O)
        assert (b.tor, b.tor_lo, b.status) == (s.tor, s.tor_lo, s.status)


def test_repeat_is_bitwise_identical(ctx):
    O = gen.random_O(18, 5, 0.5, 1.0, 0.7)
    say("case repeat n=18")
    a, b = ctx.eval(O), ctx.eval(O)
    assert (a.tor, a.tor_lo, a.sum_abs) == (b.tor, b.tor_lo, b.sum_abs)


@pytest.mark.parametrize("n", [6, 10])
def test_plain_kernel_against_oracle(ctx, n):
    O = gen.random_O(n, 300 + n, 0.5, 1.0, 0.7)
    say(f"case plain n={n}")
    p = ctx.eval_plain(O)
    q = orc.tor(O, mode=orc.QUAD)
    assert p.subsets == 1 << n
    assert abs(p.value - q.value) <= tol(q, orc.QUAD)
    # a sub-range of masks is a plain restricted sum
    lo_, hi_ = 5, (1 << n) - 7
    pr = ctx.eval_plain(O, lo_, hi_)
    ts = [orc.det(O, Z)[1] for Z in range(lo_, hi_)]
    assert abs(pr.value - math.fsum(ts)) <= tol_terms(ts)


@pytest.mark.parametrize("n", [6, 12])
def test_plain_kernel_real_and_complex_forms(ctx, n):
    # a Gaussian-state matrix runs on the real quadrature form (padded to the
    # recursive kernel's 11 modes when n is smaller); the forced complex form
    # must give the same sum, and both the oracle's
    from paper_2109_04528_amd import Context, TOR_FORCE_COMPLEX
    O = gen.random_O(n, 310 + n, 0.4, 1.1, 0.8)
    say(f"case plain real/complex n={n}")
    pr = ctx.eval_plain(O)
    with Context(device=0, flags=TOR_FORCE_COMPLEX) as cc:
        pc = cc.eval_plain(O)
        lo_, hi_ = 3, (1 << n) - 5
        pcr = cc.eval_plain(O, lo_, hi_)
    prr = ctx.eval_plain(O, lo_, hi_)
    assert pr.path == 1 and pc.path == 2
    q = orc.tor(O, mode=orc.QUAD)
    b = tol(q, orc.QUAD)
    assert abs(pr.value - q.value) <= b and abs(pc.value - q.value) <= b
    ts = [orc.det(O, Z)[1] for Z in range(lo_, hi_)]
    want = math.fsum(ts)
    tol_r = tol_terms(ts)
    assert abs(prr.value - want) <= tol_r and abs(pcr.value - want) <= tol_r


def test_error_codes(ctx):
    from paper_2109_04528_amd import TorError, TOR_E_INVAL, TOR_E_NOT_PD
    say("case error codes")
    O = gen.random_O(6, 1) + 2.0 * np.eye(12)
    with pytest.raises(TorError) as ei:
        ctx.eval(O)
    assert ei.value.code == TOR_E_NOT_PD
    O = gen.random_O(6, 1)
    O[3, 1] = np.nan
    with pytest.raises(TorError) as ei:
        ctx.eval(O)
    assert ei.value.code == TOR_E_INVAL
    with pytest.raises(TorError) as ei:
        ctx.eval(gen.vacuum_O(41))
    assert ei.value.code == TOR_E_INVAL


def test_fp64_accumulation_mode():
    from paper_2109_04528_amd import Context
    O = gen.random_O(16, 0, 0.3, 1.2, 0.9)
    say("case fp64 accumulation n=16")
    with Context(device=0, accum="fp64") as c:
        f = c.eval(O)
    q = orc.tor(O, mode=orc.QUAD)
    assert f.tor_lo == 0.0
    assert abs(f.value - q.value) <= 2 * term_bound(O, q.sum_abs)


def test_serving_results_equal_eval(ctx):
    ns = [8, 13, 10, 16, 9]
    Os = [gen.random_O(n, 400 + n, 0.5, 1.0, 0.6) for n in ns]
    say("case serving submit/poll")
    tickets = [ctx.submit(O) for O in Os]
    ctx.drain(60000)
    for O, t in zip(Os, tickets):
        r = ctx.poll(t)
        assert r is not None
        s = ctx.eval(O)
        assert (r.tor, r.tor_lo) == (s.tor, s.tor_lo)


def test_path_choice_and_real_vs_complex(ctx):
    from paper_2109_04528_amd import Context, TOR_FORCE_COMPLEX
    O = gen.random_O(14, 9, 0.3, 1.2, 0.9)
    G = gen.random_hpd_O(11, 3)
    say("case path choice n=14 / generic n=11")
    r_real = ctx.eval(O)
    assert r_real.path == 1
    assert ctx.eval(G).path == 2
    with Context(device=0, flags=TOR_FORCE_COMPLEX) as c:
        r_cplx = c.eval(O)
    assert r_cplx.path == 2
    q = orc.tor(O, mode=orc.QUAD)
    b = tol(q, orc.QUAD)
    assert abs(r_real.value - q.value) <= b
    assert abs(r_cplx.value - q.value) <= b
    say(f"  real={r_real.value!r} complex={r_cplx.value!r} quad={q.value!r}")


def test_click_submatrices_of_a_40_mode_state(ctx):
    # serving workload inputs: principal submatrices O_S of an M = 40 state
    big = gen.random_O(40, 5000, 0.5, 1.0, 0.6)
    rng = np.random.default_rng(11)
    for n in (8, 12, 15):
        S = sorted(rng.choice(40, size=n, replace=False).tolist())
        O = gen.click_submatrix(big, S)
        r, q = check(ctx, O, label=f"click pattern n={n}")
        assert r.path == 1


def test_autotune_and_cache_roundtrip(tmp_path):
    from paper_2109_04528_amd import Context, TOR_TUNE_REAL, TorError
    say("case autotune n=12..16")
    with Context(device=0) as c:
        c.autotune(12, 16, TOR_TUNE_REAL)
        p = str(tmp_path / "tune.json")
        c.save_tuning(p)
        import json
        d = json.load(open(p))
        assert d["arch"].startswith("gfx") and len(d["entries"]) == 5
        O = gen.random_O(15, 1, 0.5, 1.0, 0.6)
        a = c.eval(O)
    with Context(device=0) as c2:
        c2.load_tuning(p)
        b = c2.eval(O)
        bad = tmp_path / "bad.json"
        bad.write_text('{"arch": "gfx000", "cus": 1, "entries": []}')
        with pytest.raises(TorError):
            c2.load_tuning(str(bad))
    q = orc.tor(O, mode=orc.QUAD)
    assert abs(a.value - q.value) <= tol(q, orc.QUAD)
    assert (a.tor, a.tor_lo) == (b.tor, b.tor_lo)


def test_batch_of_64_mixed_sizes_bitwise(ctx):
    ns, Os = gen.batch_mix(64, 12, 20, seed=4)
    say("case batch of 64, n in [12, 20]")
    batch = ctx.eval_batch(Os)
    for O, b in zip(Os[::7], batch[::7]):
        s = ctx.eval(O)
        assert (b.tor, b.tor_lo) == (s.tor, s.tor_lo)
    O = Os[3]
    q = orc.tor(O, mode=orc.F64)
    assert abs(batch[3].value - q.value) <= tol(q, orc.F64)


def test_serving_alone_equals_in_mix(ctx):
    big = gen.random_O(40, 5001, 0.5, 1.0, 0.8)
    rng = np.random.default_rng(3)
    reqs = []
    for i in range(40):
        n = int(rng.integers(8, 23))
        S = sorted(rng.choice(40, size=n, replace=False).tolist())
        reqs.append(gen.click_submatrix(big, S))
    say("case serving: 40 mixed requests in one stream")
    tickets = [ctx.submit(O) for O in reqs]
    got = {}
    import time
    t0 = time.time()
    while len(got) < len(tickets) and time.time() - t0 < 120:
        for t in tickets:
            if t not in got:
                r = ctx.poll(t)
                if r is not None:
                    got[t] = r
        time.sleep(0.001)
    assert len(got) == len(tickets)
    for O, t in zip(reqs, tickets):
        alone = ctx.eval(O)
        assert got[t].status == 0
        assert (got[t].tor, got[t].tor_lo) == (alone.tor, alone.tor_lo)


def test_serving_errors(ctx):
    from paper_2109_04528_amd import TorError, TOR_E_UNKNOWN, TOR_E_INVAL
    say("case serving errors")
    with pytest.raises(TorError) as ei:
        ctx.poll(10 ** 12)
    assert ei.value.code == TOR_E_UNKNOWN
    with pytest.raises(TorError) as ei:
        ctx.submit(gen.vacuum_O(41))
    assert ei.value.code == TOR_E_INVAL
    t = ctx.submit(gen.random_O(9, 1))
    ctx.drain(60000)
    assert ctx.poll(t) is not None
    with pytest.raises(TorError):
        ctx.poll(t)  # released after the first successful poll


@pytest.mark.parametrize("n", [12, 14, 17])
def test_split_depth_does_not_change_the_result(n):
    """Each term is the same sequence of pivots whichever tier takes a level,
    and the sums are exact for Gaussian-state input, so every split depth --
    down to one tier-A leaf per root (k = n - 11 on the real path, and k = 0
    with no root decisions) -- gives the same Torontonian bit for bit, on the
    real and the complex path (the sum of |t|, a plain FP64 sum grouped by
    root, to its rounding)."""
    from paper_2109_04528_amd import TOR_FORCE_COMPLEX, Context
    O = gen.random_O(n, 60 + n, 0.5, 1.0, 0.7)
    for flags, R in ((0, 11), (TOR_FORCE_COMPLEX, 9)):
        vals = {}
        for k in sorted({0, 1, max(n - R - 1, 0), n - R}):
            with Context(device=0, split_k=k, flags=flags) as c:
                r = c.eval(O)
            assert r.status == 0
            vals[k] = (r.tor, r.tor_lo, r.sum_abs)
        say(f"case split depths n={n} flags={flags}: {sorted(vals)} -> {set(vals.values())}")
        assert len({v[:2] for v in vals.values()}) == 1
        # the sum of |t| is a plain FP64 sum, grouped by root
        sa = [v[2] for v in vals.values()]
        assert max(sa) - min(sa) <= 1e-13 * max(sa)
