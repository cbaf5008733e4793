"""Device staging (tor_stage.hip): device-resident inputs read in place,
validation, the structure test, and positive definiteness reported by the
kernels' own pivot test.

A device input and the same matrix given from host memory are staged by the
same kernel into the same form, so every result must agree bit for bit.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2109_04528_amd import inputs as gen

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(O):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(O, dtype=np.complex128)).to("cuda:0")
    torch.cuda.synchronize()
    return t


def same(a, b):
    return (a.tor, a.tor_lo, a.sum_abs, a.path, a.status) == (b.tor, b.tor_lo, b.sum_abs, b.path, b.status)


def same_value(a, b):
    # the double-double sum of the terms is exact, but the FP64 sum of |t|
    # depends on the order, which serving (its own split) and the comparison
    # kernels (roots handed to waves as they come) do not fix
    return (a.tor, a.tor_lo, a.path, a.status) == (b.tor, b.tor_lo, b.path, b.status)


def kappa(O):
    C = np.eye(O.shape[0]) - O
    C = np.tril(C) + np.tril(C, -1).conj().T
    w = np.linalg.eigvalsh(C)
    return float(w[-1] / w[0])


@pytest.fixture(scope="module")
def ctxs():
    from paper_2109_04528_amd import Context, TOR_INPUT_DEVICE
    h = Context(device=0)
    d = Context(device=0, flags=TOR_INPUT_DEVICE)
    yield h, d
    h.close()
    d.close()


def test_device_input_eval_and_batch(ctxs):
    h, d = ctxs
    mats = [gen.random_O(14, 31, 0.3, 1.2, 0.9), gen.random_hpd_O(10, 32), gen.vacuum_O(0),
            gen.random_O(3, 33, 0.5, 1.0, 0.7)]
    say("case device input eval/batch")
    for O in mats:
        a, b = h.eval(O), d.eval(dev(O))
        say(f"  n={O.shape[0] // 2} path={a.path} host={a.value!r} device={b.value!r}")
        assert same(a, b)
    ra = h.eval_batch(mats)
    rb = d.eval_batch([dev(O) for O in mats])
    assert all(same(x, y) for x, y in zip(ra, rb))


def test_device_input_written_just_before_the_call():
    """A tensor torch is still writing when the call is made (a long matrix
    product queued ahead of the copy into it): the binding orders the
    library's reads after torch's queued work, on the library's own stream
    (the host waits) and on a torch stream of the caller's (the stream waits
    on the device).  A read that ran ahead would see zeros, the vacuum."""
    import torch
    from paper_2109_04528_amd import Context, TOR_INPUT_DEVICE
    O = gen.random_O(12, 51, 0.3, 1.2, 0.9)
    with Context(device=0) as h:
        want = h.eval(O)
    src = torch.from_numpy(O).pin_memory()
    for kind in ("library stream", "torch stream"):
        say(f"case device input written just before the call ({kind})")
        s = torch.cuda.Stream(device="cuda:0") if kind == "torch stream" else None
        with Context(device=0, flags=TOR_INPUT_DEVICE, stream=s) as d:
            t = torch.zeros(O.shape, dtype=torch.complex128, device="cuda:0")
            a = torch.full((4096, 4096), 1e-3, dtype=torch.float32, device="cuda:0")
            torch.cuda.synchronize()
            for _ in range(16):  # several milliseconds of queued work
                a = a @ a
            t.copy_(src, non_blocking=True)
            r = d.eval(t)
            torch.cuda.synchronize()
        assert same(r, want), (kind, r.value, want.value)


def test_convenience_function_takes_host_and_device_matrices():
    from paper_2109_04528_amd import tor
    O = gen.random_O(9, 43, 0.3, 1.2, 0.9)
    assert tor(O) == tor(dev(O))


def test_device_input_strided(ctxs):
    _, d = ctxs
    import torch
    O = gen.random_O(9, 34, 0.3, 1.2, 0.9)
    big = torch.zeros((30, 30), dtype=torch.complex128, device="cuda:0")
    big[:18, :18] = torch.from_numpy(O).to("cuda:0")
    big[:18, 18:] = float("nan")  # outside the matrix: never read
    torch.cuda.synchronize()
    view = big[:18, :18]
    assert view.stride(0) == 30
    say("case strided device input n=9, ld=30")
    a, b = d.eval(view), d.eval(dev(O))
    assert same(a, b)


def test_device_input_other_entry_points(ctxs):
    h, d = ctxs
    O = gen.random_O(10, 35, 0.5, 1.0, 0.7)
    say("case device input partials/plain/removal/click/submit")
    ka, pa, ra = h.eval_partials(O, 6)
    kb, pb, rb = d.eval_partials(dev(O), 6)
    assert ka == kb and np.array_equal(pa, pb) and same(ra, rb)
    assert same_value(h.eval_plain(O, 3, 900), d.eval_plain(dev(O), 3, 900))
    assert same_value(h.eval_removal(O), d.eval_removal(dev(O)))
    S = gen.random_O(12, 36, 0.5, 1.0, 0.7)
    pats = [0, 0b101, 0b111100001111, (1 << 12) - 1]
    p1, r1 = h.click_probs(S, pats)
    p2, r2 = d.click_probs(dev(S), pats)
    assert np.array_equal(p1, p2) and all(same(x, y) for x, y in zip(r1, r2))
    t = d.submit(dev(O))
    d.drain(60000)
    r = d.poll(t)
    assert same_value(r, h.eval(O))


def test_only_the_lower_triangle_is_read(ctxs):
    from paper_2109_04528_amd import Context, TOR_CHECK_HERMITIAN, TOR_E_INVAL, TorError
    h, _ = ctxs
    O = gen.random_O(8, 37, 0.3, 1.2, 0.9)
    junk = O.copy()
    iu = np.triu_indices(16, 1)
    junk[iu] = 7.0 + 3.0j
    junk[0, 5] = np.nan
    say("case lower triangle only / TOR_CHECK_HERMITIAN")
    assert same(h.eval(O), h.eval(junk))
    with Context(device=0, flags=TOR_CHECK_HERMITIAN) as c:
        assert same(c.eval(O), h.eval(O))
        with pytest.raises(TorError) as ei:
            c.eval(junk)
        assert ei.value.code == TOR_E_INVAL
        off = O.copy()
        off[1, 9] += 1e-9  # breaks Hermiticity beyond 1e-12
        with pytest.raises(TorError) as ei:
            c.eval(off)
        assert ei.value.code == TOR_E_INVAL


def test_structure_tolerance(ctxs):
    h, _ = ctxs
    O = gen.random_O(12, 38, 0.3, 1.2, 0.9)
    n = 12
    say("case structure test tolerance")
    # a change far below 64 ulp of max|C| keeps the real path; one far above
    # it (the lower-right block no longer conj of the upper-left) does not
    tiny, big = O.copy(), O.copy()
    tiny[n + 3, n + 1] += 1e-18
    tiny[n + 1, n + 3] += 1e-18
    big[n + 3, n + 1] += 1e-9
    big[n + 1, n + 3] += 1e-9
    rt, rb = h.eval(tiny), h.eval(big)
    assert rt.path == 1 and rb.path == 2
    # the GPU evaluates the perturbed matrix, the oracle the original: the
    # worst-case term bound also covers the first-order effect of 1e-18
    q = orc.tor(O, mode=orc.QUAD)
    assert abs(rt.value - q.value) <= 8.0 * n * kappa(O) * U * q.sum_abs


def test_not_positive_definite_from_the_kernels(ctxs):
    from paper_2109_04528_amd import TOR_E_NOT_PD, TOR_OK, TorError
    h, _ = ctxs
    good = gen.random_O(9, 39, 0.3, 1.2, 0.9)
    bad_real = gen.random_O(9, 40, 0.3, 1.2, 0.9) + 2.0 * np.eye(18)  # structured, C = -I - O'
    bad_cplx = np.eye(14, dtype=np.complex128) * 1.5
    bad_cplx[3, 2] = 0.2 + 0.1j  # no Gaussian-state structure
    say("case NOT_PD: batch with one bad matrix, and each path")
    rs = h.eval_batch([good, bad_real, bad_cplx, good], check=False)
    assert [r.status for r in rs] == [TOR_OK, TOR_E_NOT_PD, TOR_E_NOT_PD, TOR_OK]
    assert same_value(rs[0], h.eval(good)) and same(rs[3], rs[0])
    with pytest.raises(TorError) as ei:
        h.eval_batch([good, bad_real])
    assert ei.value.code == TOR_E_NOT_PD
    # barely positive definite stays valid: I - O = c I on the real path,
    # Tor = (1/c - 1)^n (each mode contributes 1/sqrt(c^2) - 1)
    O = np.eye(18, dtype=np.complex128) * (1.0 - 1e-6)
    c = 1.0 - (1.0 - 1e-6)
    r = h.eval(O)
    n = 9
    assert r.status == TOR_OK and r.path == 1
    want = (1.0 / c - 1.0) ** n
    assert abs(r.value - want) <= 1e-13 * want


def test_serving_reports_staging_errors():
    from paper_2109_04528_amd import Context, TOR_E_INVAL, TOR_E_NOT_PD
    O = gen.random_O(8, 41, 0.3, 1.2, 0.9)
    nanO = O.copy()
    nanO[5, 2] = np.nan
    badO = O + 2.0 * np.eye(16)
    say("case serving: a NaN input and a non-PD input among good ones")
    with Context(device=0) as c:
        ts = [c.submit(x) for x in (O, nanO, badO, O)]
        c.drain(60000)
        rs = [c.poll(t) for t in ts]
        ref = c.eval(O)
    assert rs[1].status == TOR_E_INVAL and rs[2].status == TOR_E_NOT_PD
    assert same_value(rs[0], ref) and same_value(rs[3], ref)


def coupled_O(n, i, j, c):
    """O = I - C for a Gaussian-state C = I/2 except the 2x2 mode coupling c
    between modes i and j (P = I/2 + c (E_ij + E_ji), Q = 0): positive
    definite iff |c| < 1/2.  Eliminating mode i first, mode j's pivot is
    1/2 - 2 c^2, the first to fail when |c| >= 1/2."""
    P = 0.5 * np.eye(n)
    P[i, j] = P[j, i] = c
    C = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    C[:n, :n] = P
    C[n:, n:] = P
    return np.eye(2 * n) - C


@pytest.mark.parametrize("n,i,j", [(30, 0, 29), (30, 0, 27), (30, 3, 21), (12, 0, 11), (8, 2, 7)])
def test_not_positive_definite_at_every_depth(ctxs, n, i, j):
    """The failing pivot is the last one of the factorisation order (inside
    the register tail), in the last few modes, in the tier-B range, and for
    matrices smaller than the kernel's minimum (padded)."""
    from paper_2109_04528_amd import Context, TOR_E_NOT_PD, TOR_FACTOR_DD, TOR_FORCE_COMPLEX, TOR_OK
    h, _ = ctxs
    say(f"case NOT_PD coupling modes {i},{j} of n={n}")
    good, bad = coupled_O(n, i, j, 0.49), coupled_O(n, i, j, 0.51)
    assert h.eval(good).status == TOR_OK
    assert h.eval(bad, check=False).status == TOR_E_NOT_PD
    if n <= 12:
        for fl in (TOR_FORCE_COMPLEX, TOR_FACTOR_DD):
            with Context(device=0, flags=fl) as c:
                assert c.eval(good).status == TOR_OK
                assert c.eval(bad, check=False).status == TOR_E_NOT_PD


def test_same_host_pointer_with_different_sizes(ctxs):
    """Through the C ABI: one host array passed twice in a batch, once whole
    and once as its leading 2m x 2m block (same pointer, larger leading
    dimension); the upload keeps one copy per (pointer, ld, size)."""
    import ctypes
    from paper_2109_04528_amd import _lib
    h, _ = ctxs
    O = np.ascontiguousarray(gen.random_O(10, 42, 0.3, 1.2, 0.9))
    sub = np.ascontiguousarray(O[:12, :12])
    say("case one host pointer, two sizes, one batch")
    ns = (ctypes.c_int * 3)(10, 6, 10)
    ptrs = (ctypes.c_void_p * 3)(O.ctypes.data, O.ctypes.data, O.ctypes.data)
    lds = (ctypes.c_long * 3)(20, 20, 20)
    res = (_lib.tor_result * 3)()
    rc = h._lib.tor_eval_batch(h._h, 3, ns, ptrs, lds, res)
    assert rc == 0
    got = [_lib.TorResult.from_c(res[i]) for i in range(3)]
    a, b = h.eval(O), h.eval(sub)
    assert same_value(got[0], a) and same_value(got[2], a)
    assert same_value(got[1], b)


def test_mixed_batch_statuses_and_values(ctxs):
    """One batch of both arithmetic paths (two launches), an input rejected
    by the staging checks, the empty matrix and a matrix that fails the
    pivot test: each matrix gets its own status, and every valid one the
    value it has alone, bit for bit."""
    from paper_2109_04528_amd import TOR_E_INVAL, TOR_E_NOT_PD, TOR_OK
    h, _ = ctxs
    real14 = gen.random_O(14, 61, 0.5, 1.0, 0.7)
    herm12 = gen.random_hpd_O(12, 62, 0.05, 0.9)
    nan8 = gen.random_O(8, 63, 0.5, 1.0, 0.7)
    nan8[5, 2] = np.nan  # lower triangle: read and rejected
    real20 = gen.random_O(20, 64, 0.3, 1.2, 0.9)
    bad10 = gen.random_O(10, 65, 0.3, 1.2, 0.9) + 2.0 * np.eye(20)
    empty = gen.vacuum_O(0)
    Os = [real14, nan8, herm12, empty, bad10, real20]
    say("case mixed batch: both paths, NaN input, empty, not positive definite")
    rs = h.eval_batch(Os, check=False)
    assert [r.status for r in rs] == [TOR_OK, TOR_E_INVAL, TOR_OK, TOR_OK, TOR_E_NOT_PD, TOR_OK]
    assert [rs[i].path for i in (0, 2, 5)] == [1, 2, 1]
    for i in (0, 2, 3, 5):
        assert same_value(rs[i], h.eval(Os[i])), i
    assert rs[3].tor == 1.0
