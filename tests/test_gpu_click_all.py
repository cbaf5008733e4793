"""Click probabilities of every pattern at once (tor_click_all), GPU.

One launch of the recursive kernel stores the signed term of every subset of
the state's modes; an exact double-double subset-sum transform then gives
Tor(O_S) for every pattern S.  Pins:
  * the transform alone against exact integer arithmetic (every term a
    multiple of 2^-52, so the sums are exact);
  * the whole state's Tor bit for bit against tor_eval: each term is the same
    sequence of pivots in both (the same arithmetic whichever tier takes a
    level), and both sums are exact;
  * every pattern against tor_click_probs, which stages each O_S on its own
    (its terms differ in the last mode's 2x2 determinant, which the last level
    of a tree forms directly; so at the statistical bound);
  * a product state's closed form p(S) = prod_{i in S} (1 - 1/a_i)
    prod_{i not in S} 1/a_i, a_i = 1/sqrt(det (I - O)_i), in 50-digit
    arithmetic from the input's own entries;
  * the __float128 oracle per pattern, and the normalisation sum_S p(S) = 1.
"""
import math
import sys

import numpy as np
import pytest

import bounds
from oracle import oracle as orc
from paper_2109_04528_amd import inputs as gen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2109_04528_amd import Context
    c = Context(device=0)
    yield c
    c.close()


def state(M, seed):
    return gen.random_O(M, seed, 0.5, 1.0, 0.7)


def sqrt_det(O):
    return math.sqrt(np.linalg.det(np.eye(O.shape[0]) - O).real)


def exact_zeta(t):
    """Subset sums in integers of 2^-52 (object arrays of Python ints)."""
    a = np.array([int(x * 2.0 ** 52) for x in t], dtype=object)
    nb = a.size.bit_length() - 1
    for b in range(nb):
        v = a.reshape(-1, 2, 1 << b)
        v[:, 1, :] += v[:, 0, :]
    return a


@pytest.mark.parametrize("nbits", [1, 4, 10, 12, 13, 16, 17, 20])
def test_subset_sum_transform_is_exact(ctx, nbits):
    rng = np.random.default_rng(nbits)
    n = 1 << nbits
    # doubles of magnitude 1 .. 2^20 with full significands, both signs
    t = rng.choice([-1.0, 1.0], n) * np.ldexp(1.0 + rng.random(n), rng.integers(0, 20, n))
    say(f"case zeta nbits={nbits}")
    gh, gl = ctx.debug_zeta(t)
    want = exact_zeta(t)
    got = np.array([int(h * 2.0 ** 52) + int(l * 2.0 ** 52) for h, l in zip(gh, gl)], dtype=object)
    assert np.all(got == want)
    assert np.all(np.abs(gl) <= np.spacing(np.abs(gh)) / 2)


@pytest.mark.parametrize("M", [8, 12, 20])
def test_whole_state_equals_eval_bitwise(ctx, M):
    O = state(M, 40 + M)
    say(f"case click_all whole state M={M}")
    probs, (th, tl), r = ctx.click_all(O, tor=True)
    e = ctx.eval(O)
    full = (1 << M) - 1
    say(f"  click_all={r.tor!r},{r.tor_lo!r} eval={e.tor!r},{e.tor_lo!r} ms={r.device_ms:.2f}")
    assert r.status == 0 and r.path == 1
    assert (r.tor, r.tor_lo) == (e.tor, e.tor_lo)
    assert (th[full], tl[full]) == (e.tor, e.tor_lo)
    assert r.sum_abs == e.sum_abs


@pytest.mark.parametrize("M", [12, 13])
def test_every_pattern_against_click_probs(ctx, M):
    """M = 12 takes the transform in LDS alone, M = 13 a register pass after
    it."""
    O = state(M, 52)
    say(f"case click_all vs click_probs M={M} ({1 << M} patterns)")
    probs, (th, tl), _ = ctx.click_all(O, tor=True)
    p2, res = ctx.click_probs(O, range(1 << M))
    assert all(r.status == 0 for r in res)
    same, worst = 0, 0.0
    for S, r in enumerate(res):
        d = abs((th[S] - r.tor) + (tl[S] - r.tor_lo))
        same += d == 0.0
        modes = [i for i in range(M) if (S >> i) & 1]
        q = orc.tor(gen.click_submatrix(O, modes), mode=orc.F64)
        tol = bounds.sum_bound(q.sum_sq, bounds.U64, bounds.U64)
        worst = max(worst, d / tol)
        assert d <= tol
    say(f"  patterns bit-identical: {same} of {1 << M}; worst difference / bound = {worst:.3f}")
    # the patterns without the last mode share every term with the whole state
    assert same >= 1 << (M - 1)


def test_product_state_closed_form(ctx):
    """p(S) = prod_{i in S} (a_i - 1) / prod_i a_i; the terms t_Z = prod_{i in Z}
    a_i of pattern S have sum t^2 = prod_{i in S} (1 + a_i^2), which sets the
    FP64 floor of each Tor(O_S)."""
    import mpmath as mp
    mp.mp.dps = 50
    M = 10
    rng = np.random.default_rng(8)
    O = gen.product_state_O(rng.uniform(0.3, 1.2, M), 0.8, rng.uniform(0, 2 * np.pi, M))
    say("case click_all product state M=10")
    probs, (th, tl), _ = ctx.click_all(O, tor=True)
    a = []
    for i in range(M):
        c11 = 1 - mp.mpf(float(O[i, i].real))
        c22 = 1 - mp.mpf(float(O[i + M, i + M].real))
        c21 = mp.mpc(-float(O[i + M, i].real), -float(O[i + M, i].imag))
        a.append(1 / mp.sqrt(c11 * c22 - abs(c21) ** 2))
    vac = mp.mpf(1)
    for ai in a:
        vac /= ai  # p(no click) = sqrt(det(I - O))
    worst, rels = 0.0, []
    for S in range(1 << M):
        tor, ssq = mp.mpf(1), mp.mpf(1)
        for i in range(M):
            if (S >> i) & 1:
                tor *= a[i] - 1
                ssq *= 1 + a[i] ** 2
        tol = bounds.sum_bound(float(ssq), bounds.U64, 0.0)
        d = float(abs((mp.mpf(th[S]) + mp.mpf(tl[S])) - tor))
        worst = max(worst, d / tol)
        rels.append(d / float(abs(tor)))
        assert d <= tol
        assert abs(probs[S] - float(tor * vac)) <= tol * float(vac) + 4e-16 * float(abs(tor * vac))
    say(f"  worst difference / bound = {worst:.3f}; median relative error {np.median(rels):.2e}")
    assert np.median(rels) <= 1e-12


def test_patterns_against_oracle(ctx):
    M = 8
    O = state(M, 53)
    say("case click_all vs __float128 oracle M=8 (256 patterns)")
    probs, (th, tl), _ = ctx.click_all(O, tor=True)
    sq = sqrt_det(O)
    worst = 0.0
    for S in range(1 << M):
        modes = [i for i in range(M) if (S >> i) & 1]
        q = orc.tor(gen.click_submatrix(O, modes), mode=orc.QUAD)
        tol = bounds.sum_bound(q.sum_sq, bounds.U64, bounds.UQ)
        d = abs((th[S] - q.hi) + (tl[S] - q.lo))
        worst = max(worst, d / tol)
        assert d <= tol
        assert abs(probs[S] - q.value * sq) <= tol * sq + 4e-16 * abs(q.value * sq)
    say(f"  worst difference / bound = {worst:.3f}")


def test_probabilities_sum_to_one(ctx):
    M = 16
    O = state(M, 54)
    say("case click_all sum rule M=16")
    probs, _, r = ctx.click_all(O)
    s = math.fsum(probs)
    say(f"  sum={s!r} min={probs.min():.3e} ms={r.device_ms:.2f}")
    assert abs(s - 1.0) <= 1e-12
    assert probs.min() >= -1e-12


def test_click_all_errors(ctx):
    from paper_2109_04528_amd import (TOR_E_INVAL, TOR_E_NOT_PD, TOR_FACTOR_DD, TOR_FORCE_COMPLEX, Context,
                                      TorError)
    bad = np.eye(12, dtype=np.complex128) * 1.5
    with pytest.raises(TorError) as ei:
        ctx.click_all(bad)
    assert ei.value.code == TOR_E_NOT_PD
    rng = np.random.default_rng(3)
    A = rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16))
    H = A @ A.conj().T
    herm = 0.5 * H / np.linalg.eigvalsh(H).max()  # Hermitian, no Gaussian-state structure
    with pytest.raises(TorError) as ei:
        ctx.click_all(herm)
    assert ei.value.code == TOR_E_INVAL
    from paper_2109_04528_amd import TOR_CLICK_ALL_MAX_M
    with pytest.raises(TorError) as ei:  # refused before anything is read or allocated
        ctx.click_all(np.zeros((2 * TOR_CLICK_ALL_MAX_M + 2,) * 2, dtype=np.complex128))
    assert ei.value.code == TOR_E_INVAL
    for flags in (TOR_FORCE_COMPLEX, TOR_FACTOR_DD):
        with Context(device=0, flags=flags) as c:
            with pytest.raises(TorError) as ei:
                c.click_all(state(6, 1))
            assert ei.value.code == TOR_E_INVAL
    probs, (th, tl), r = ctx.click_all(np.zeros((0, 0), dtype=np.complex128), tor=True)
    assert probs.tolist() == [1.0] and th.tolist() == [1.0] and r.tor == 1.0


def test_device_outputs_equal_host_outputs(ctx):
    import torch
    from paper_2109_04528_amd import TOR_INPUT_DEVICE, TOR_OUTPUT_DEVICE, Context
    M = 14
    O = state(M, 55)
    say("case click_all device input and outputs M=14")
    probs, (th, tl), r = ctx.click_all(O, tor=True)
    Od = torch.from_numpy(O).to("cuda:0")
    with Context(device=0, flags=TOR_INPUT_DEVICE | TOR_OUTPUT_DEVICE) as c:
        pd, (hd, ld), rd = c.click_all(Od, tor=True)
        assert pd.is_cuda and hd.is_cuda
        assert np.array_equal(pd.cpu().numpy(), probs)
        assert np.array_equal(hd.cpu().numpy(), th) and np.array_equal(ld.cpu().numpy(), tl)
        assert (rd.tor, rd.tor_lo) == (r.tor, r.tor_lo)
        p0, _, _ = c.click_all(torch.zeros((0, 0), dtype=torch.complex128, device="cuda:0"))
        assert p0.cpu().tolist() == [1.0]


def test_largest_state(ctx):
    """The largest state the call takes (M = 32: 2^32 terms, 96 GiB of
    workspace and 96 GiB of outputs left on the device).  A pattern that holds the last
    mode, and has enough modes that its own staged form needs no padding
    modes (11 on the real path), forms every term exactly as a call for that
    pattern alone does (the same include steps, the same last-level
    determinant, exact sums), so the two agree bit for bit; small patterns
    are checked against the FP64 oracle at the statistical bound; the
    probabilities sum to one."""
    import torch
    from paper_2109_04528_amd import TOR_CLICK_ALL_MAX_M, TOR_OUTPUT_DEVICE, Context
    M = TOR_CLICK_ALL_MAX_M
    O = state(M, 56)
    say(f"case click_all largest state M={M}")
    with Context(device=0, flags=TOR_OUTPUT_DEVICE) as c:
        pd, (hd, ld), r = c.click_all(O, tor=True)
        torch.cuda.synchronize(0)
        e = ctx.eval(O)
        full = (1 << M) - 1
        say(f"  whole state {r.tor!r},{r.tor_lo!r} eval {e.tor!r},{e.tor_lo!r} ms={r.device_ms:.1f}")
        assert r.status == 0 and (r.tor, r.tor_lo) == (e.tor, e.tor_lo)
        assert (hd[full].item(), ld[full].item()) == (e.tor, e.tor_lo)
        s = torch.sum(pd).item()
        say(f"  sum of 2^{M} probabilities - 1 = {s - 1.0:.3e}; min {torch.min(pd).item():.3e}")
        assert abs(s - 1.0) <= 1e-10
        rng = np.random.default_rng(56)
        last = 1 << (M - 1)
        pats = [last, full] + [int(x) | last for x in rng.integers(0, last, 10)]
        pats += [int(x) for x in rng.integers(0, last, 6)]
        pats = [S for S in pats if S != full]
        idx = torch.tensor(pats, dtype=torch.int64, device=pd.device)
        gh, gl, gp = hd[idx].cpu().numpy(), ld[idx].cpu().numpy(), pd[idx].cpu().numpy()
    p1, res = ctx.click_probs(O, pats)
    sq = sqrt_det(O)
    bitwise = 0
    for j, S in enumerate(pats):
        rr = res[j]
        assert rr.status == 0
        if S & last and bin(S).count("1") >= 11:
            assert (gh[j], gl[j]) == (rr.tor, rr.tor_lo), S
            assert gp[j] == p1[j]
            bitwise += 1
        elif bin(S).count("1") <= 16:
            modes = [i for i in range(M) if (S >> i) & 1]
            q = orc.tor(gen.click_submatrix(O, modes), mode=orc.F64)
            tol = bounds.sum_bound(q.sum_sq, bounds.U64, bounds.U64)
            assert abs((gh[j] - q.hi) + (gl[j] - q.lo)) <= tol
            assert abs(gp[j] - q.value * sq) <= tol * sq + 4e-16 * abs(q.value * sq)
    say(f"  {len(pats)} sampled patterns checked, {bitwise} of them bit for bit")
    assert bitwise >= 8


def mobius_units(g):
    """Inverse of the subset-sum transform, in exact integers: the terms t[Z]
    from the sums g[S] = sum over Z subset of S of t[Z]."""
    a = np.array(g, dtype=object)
    nb = a.size.bit_length() - 1
    for b in range(nb):
        v = a.reshape(-1, 2, 1 << b)
        v[:, 1, :] -= v[:, 0, :]
    return a


@pytest.mark.parametrize("M,sample", [(12, None), (20, 768)])
def test_every_term_against_oracle(ctx, M, sample):
    """The hot path's sum, term by term.  The every-pattern call returns each
    pattern's Torontonian as an exact double-double sum of the stored terms,
    so inverting the subset-sum transform in integers recovers every term
    the recursive kernel formed, t[Z] = (-1)^(M-|Z|) / sqrt(det (I - O)_Z),
    bit for bit.  Each is compared with the __float128 oracle's term for the
    same subset (all 4096 at M = 12; the empty and full sets and a sample at
    M = 20, where the walk takes every tier).  The bound is the FP64
    elimination's: (2|Z| + 2)^2 u cond(I - O) relative error per term (a
    principal submatrix is no worse conditioned than I - O)."""
    O = state(M, 57 + M)
    say(f"case every term M={M}")
    _, (th, tl), r = ctx.click_all(O, tor=True)
    assert r.status == 0
    n = 1 << M
    pop = np.array([bin(S).count("1") for S in range(n)])
    g = [(-1 if (M - pop[S]) & 1 else 1) * (int(th[S] * 2.0 ** 52) + int(tl[S] * 2.0 ** 52)) for S in range(n)]
    t = mobius_units(g)
    ev = np.linalg.eigvalsh(np.eye(2 * M) - O)
    cond = ev.max() / ev.min()
    Zs = range(n) if sample is None else [0, n - 1] + [int(z) for z in np.random.default_rng(M).integers(0, n, sample)]
    worst = 0.0
    for Z in Zs:
        d, tq = orc.det(O, Z, mode=orc.QUAD)
        tg = float(t[Z]) / 2.0 ** 52
        k = bin(Z).count("1")
        tol = (2 * k + 2) ** 2 * bounds.U64 * cond
        rel = abs(tg - tq) / abs(tq)
        worst = max(worst, rel / tol)
        assert rel <= tol, (Z, tg, tq)
        assert (tg > 0) == (tq > 0)
    say(f"  {len(Zs)} terms; cond(I - O) = {cond:.1f}; worst relative error / bound = {worst:.3g}")


def test_terms_of_the_headline_workload(ctx):
    """Sampled terms of the n = 30 precision workload (r ~ U[.3, 1.2],
    eta = .9, seed 0; the benchmark's matrix, R about 1.5e14), each against
    the __float128 oracle's term for its subset.  A term t[Z] is the
    alternating sum of the exact subset sums g[S] over the 2^|Z| patterns S
    inside Z, so subsets of up to 14 modes are read back from the device."""
    import itertools
    import torch
    from paper_2109_04528_amd import TOR_OUTPUT_DEVICE, Context
    M = 30
    O = gen.random_O(M, 0, 0.3, 1.2, 0.9)
    say("case terms of the n=30 precision workload")
    rng = np.random.default_rng(30)
    Zs = [0, 1 << 29, 1 << 17, (1 << 29) | 1]
    for size in (2, 3, 5, 8, 11, 14):
        for _ in range(3):
            Zs.append(int(sum(1 << int(i) for i in rng.choice(M, size, replace=False))))
    ev = np.linalg.eigvalsh(np.eye(2 * M) - O)
    cond = ev.max() / ev.min()
    worst = 0.0
    with Context(device=0, flags=TOR_OUTPUT_DEVICE) as c:
        _, (hd, ld), r = c.click_all(O, tor=True, probs=False)
        torch.cuda.synchronize(0)
        assert r.status == 0
        for Z in Zs:
            bits = [i for i in range(M) if (Z >> i) & 1]
            subs = [sum(1 << b for b, on in zip(bits, sel) if on) for sel in itertools.product((0, 1), repeat=len(bits))]
            idx = torch.tensor(subs, dtype=torch.int64, device=hd.device)
            gh, gl = hd[idx].cpu().numpy(), ld[idx].cpu().numpy()
            tot = 0
            for S, h, l in zip(subs, gh, gl):
                # g[S] = (-1)^(M-|S|) Tor(O_S); t[Z] = sum over S of (-1)^(|Z|-|S|) g[S]
                sign = -1 if (M - len(bits)) & 1 else 1
                tot += sign * (int(h * 2.0 ** 52) + int(l * 2.0 ** 52))
            tg = tot / 2.0 ** 52
            d, tq = orc.det(O, Z, mode=orc.QUAD)
            tol = (2 * len(bits) + 2) ** 2 * bounds.U64 * cond
            rel = abs(tg - tq) / abs(tq)
            worst = max(worst, rel / tol)
            assert rel <= tol, (Z, tg, tq)
    say(f"  {len(Zs)} terms; cond(I - O) = {cond:.1f}; worst relative error / bound = {worst:.3g}")
