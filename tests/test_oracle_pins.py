"""Pins for the CPU oracle: it is checked against things other than itself.

* closed forms: vacuum (Tor = 0 for n >= 1, the binomial identity), n = 0
  (Tor = 1), n = 1 (1/sqrt(det(I - O)) - 1), product states (the Torontonian
  of a direct sum is the product of the single-mode values
  sqrt(1 + eta (2 - eta) sinh^2 r) - 1);
* the click-probability normalisation: p(S) = Tor(O_S) sqrt(det(I - O)) >= 0
  and sum_S Tor(O_S) = 1/sqrt(det(I - O)) (Moebius inversion of Eq. 2),
  with the right-hand side from numpy's determinant;
* Jacobi's complementary-minor identity, an independent numeric path:
  Tor(O) = sqrt(det sigma_Q) sum_W (-1)^|W| / sqrt(det (sigma_Q)_W),
  sigma_Q = (I - O)^{-1}, with numpy determinants;
* brute force of Eq. 2 in 40-digit mpmath (LU determinants, not Cholesky);
* invariances: mode permutation (the reordering remark in Sec. 2), complex
  conjugation, per-mode phase rotation;
* subtree restriction: the 2^k restricted sums add up to the full sum;
* the reported sums of |t| and t^2 of a product state against their closed
  forms prod (1 + a_i) and prod (1 + a_i^2), a_i = 1/sqrt(det(I - O_i));
* the x87 extended mode against mpmath, the closed forms and __float128.

The mutation tests at the end plant plausible mistakes in a copy of the
oracle's C source (a flipped sign, a dropped conjugate, a dropped term, a
wrong index) and check that at least one pin fails for each.
"""
import ctypes
import os
import shutil
import subprocess
import sys
import tempfile

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2109_04528_amd import inputs as gen

U64 = np.finfo(np.float64).eps / 2


def _closed_product(r, eta):
    r = np.asarray(r, dtype=np.float64)
    return float(np.prod(np.sqrt(1.0 + eta * (2.0 - eta) * np.sinh(r) ** 2) - 1.0))


# ---------------------------------------------------------------------------
# pins written against a generic "tor" callable so that mutants can reuse them
# ---------------------------------------------------------------------------

def pin_vacuum(tor):
    for n in range(1, 7):
        v = tor(gen.vacuum_O(n), orc.F64)
        assert v == 0.0, f"vacuum n={n}: {v}"
    assert tor(gen.vacuum_O(0), orc.F64) == 1.0


def pin_n1(tor):
    for seed in range(3):
        O = gen.random_O(1, seed, 0.3, 1.2, 0.8)
        want = 1.0 / np.sqrt(np.linalg.det(np.eye(2) - O).real) - 1.0
        got = tor(O, orc.QUAD)
        assert abs(got - want) <= 1e-13 * abs(want), (got, want)


def pin_product(tor):
    rng = np.random.default_rng(7)
    for n in (3, 4, 5):
        r = rng.uniform(0.3, 1.2, n)
        eta = float(rng.uniform(0.3, 1.0))
        ph = rng.uniform(0, 2 * np.pi, n)
        O = gen.product_state_O(r, eta, ph)
        want = _closed_product(r, eta)
        got = tor(O, orc.QUAD)
        # the closed form is evaluated in FP64 from the same r; O itself was
        # built in FP64, so agreement is at the FP64 input-rounding level
        assert abs(got - want) <= 1e-11 * abs(want), (n, got, want)


def pin_mobius(tor):
    for seed in range(2):
        n = 4
        O = gen.random_O(n, seed, 0.5, 1.0, 0.6)
        total = 0.0
        pmin = 1.0
        sq = np.sqrt(np.linalg.det(np.eye(2 * n) - O).real)
        for S in range(1 << n):
            modes = [i for i in range(n) if (S >> i) & 1]
            t = tor(gen.click_submatrix(O, modes), orc.QUAD) if modes else 1.0
            total += t
            pmin = min(pmin, t * sq)
        assert pmin >= -1e-15
        assert abs(total * sq - 1.0) <= 1e-12, total * sq


def _mp_tor(O, dps=40):
    import mpmath as mp
    mp.mp.dps = dps
    n = O.shape[0] // 2
    acc = mp.mpf(0)
    for Z in range(1 << n):
        modes = [i for i in range(n) if (Z >> i) & 1]
        d = len(modes)
        sign = -1 if (n - d) & 1 else 1
        if d == 0:
            acc += sign
            continue
        idx = modes + [m + n for m in modes]
        M = mp.matrix(2 * d, 2 * d)
        for a in range(2 * d):
            for b in range(2 * d):
                # Hermitian completion from the lower triangle of I - O
                ia, ib = idx[a], idx[b]
                if ia >= ib:
                    o = complex(O[ia, ib])
                    v = mp.mpc(o.real, o.imag)
                else:
                    o = complex(O[ib, ia])
                    v = mp.mpc(o.real, -o.imag)
                M[a, b] = (1 if ia == ib else 0) - v
        det = mp.re(mp.det(M))
        acc += sign / mp.sqrt(det)
    return acc


def pin_mpmath(tor):
    for seed, n in ((0, 3), (1, 4), (2, 5)):
        O = gen.random_O(n, seed, 0.3, 1.2, 0.9)
        want = _mp_tor(O)
        got = tor(O, orc.QUAD)
        rel = abs((got - float(want)) / float(want))
        assert rel <= 1e-20, (n, got, float(want), rel)


def pin_jacobi(tor):
    n = 5
    O = gen.random_O(n, 3, 0.5, 1.0, 0.7)
    sq = np.linalg.inv(np.eye(2 * n) - O)
    acc = 0.0
    absacc = 0.0
    for W in range(1 << n):
        modes = [i for i in range(n) if (W >> i) & 1]
        if modes:
            idx = modes + [m + n for m in modes]
            d = np.linalg.det(sq[np.ix_(idx, idx)]).real
        else:
            d = 1.0
        t = (-1.0) ** len(modes) / np.sqrt(d)
        acc += t
        absacc += abs(t)
    want = np.sqrt(np.linalg.det(sq).real) * acc
    got = tor(O, orc.QUAD)
    assert abs(got - want) <= 1e-13 * absacc * np.sqrt(np.linalg.det(sq).real), (got, want)


ALL_PINS = [pin_vacuum, pin_n1, pin_product, pin_mobius, pin_mpmath, pin_jacobi]


def _oracle_tor(O, mode):
    return orc.tor(O, mode=mode).value


@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin):
    pin(_oracle_tor)


# ---------------------------------------------------------------------------
# further properties of the oracle
# ---------------------------------------------------------------------------

def test_product_state_fp64_larger_n():
    r = np.linspace(0.5, 1.0, 12)
    O = gen.product_state_O(r, 0.5, np.linspace(0, 3, 12))
    res = orc.tor(O, mode=orc.F64)
    want = _closed_product(r, 0.5)
    # FP64 terms: the error is bounded by a few ulps of each term times R
    bound = 64 * U64 * res.sum_abs
    assert abs(res.value - want) <= bound, (res.value, want, bound)


def test_product_state_sums_of_abs_and_squares():
    # t_Z = (-1)^(n-|Z|) prod_{i in Z} a_i for a product state, so
    # sum |t| = prod (1 + a_i) and sum t^2 = prod (1 + a_i^2)
    rng = np.random.default_rng(21)
    r = rng.uniform(0.3, 1.2, 9)
    eta = 0.8
    O = gen.product_state_O(r, eta, rng.uniform(0, 2 * np.pi, 9))
    a = np.sqrt(1.0 + eta * (2.0 - eta) * np.sinh(r) ** 2)
    for mode in (orc.F64, orc.LD, orc.QUAD):
        res = orc.tor(O, mode=mode)
        assert abs(res.sum_abs / np.prod(1 + a) - 1) <= 1e-12, mode
        assert abs(res.sum_sq / np.prod(1 + a * a) - 1) <= 1e-12, mode
        assert res.count == 1 << 9


def test_extended_mode_pins():
    # x87 extended precision (64-bit significand): exact zero for the vacuum,
    # the product closed form, 40-digit mpmath, and __float128 at n = 14
    # within a few units of 2^-64 times sqrt(sum t^2) (independent per-term
    # roundings add in quadrature)
    for n in (1, 4, 7):
        assert orc.tor(gen.vacuum_O(n), mode=orc.LD).value == 0.0
    r = np.linspace(0.4, 1.1, 6)
    O = gen.product_state_O(r, 0.7, np.linspace(0, 2, 6))
    want = _closed_product(r, 0.7)
    assert abs(orc.tor(O, mode=orc.LD).value - want) <= 1e-11 * abs(want)
    for seed, n in ((0, 3), (1, 4)):
        O = gen.random_O(n, seed, 0.3, 1.2, 0.9)
        want = float(_mp_tor(O))
        got = orc.tor(O, mode=orc.LD).value
        assert abs(got - want) <= 1e-15 * abs(want), (n, got, want)
    O = gen.random_O(14, 2, 0.3, 1.2, 0.9)
    q = orc.tor(O, mode=orc.QUAD)
    e = orc.tor(O, mode=orc.LD)
    f = orc.tor(O, mode=orc.F64)
    spread = np.sqrt(q.sum_sq)
    assert abs(e.value - q.value) <= 32 * 2.0 ** -64 * spread, (e.value, q.value)
    assert abs(e.value - q.value) < abs(f.value - q.value)


def test_permutation_conjugation_phase_invariance():
    n = 6
    O = gen.random_O(n, 11, 0.3, 1.2, 0.9)
    # exact Hermitian completion of the lower triangle, so that a permutation
    # (which moves entries between triangles) changes no value that is read
    O = np.tril(O) + np.tril(O, -1).conj().T
    O[np.diag_indices(2 * n)] = O.diagonal().real
    base = orc.tor(O, mode=orc.QUAD).value
    perm = np.random.default_rng(0).permutation(n)
    idx = np.concatenate([perm, perm + n])
    Op = O[np.ix_(idx, idx)]
    phi = np.random.default_rng(1).uniform(0, 2 * np.pi, n)
    D = np.diag(np.concatenate([np.exp(1j * phi), np.exp(-1j * phi)]))
    Oph = D @ O @ D.conj().T
    sum_abs = orc.tor(O, mode=orc.QUAD).sum_abs
    # permutation and conjugation are exact on the input bytes; the phase
    # rotation is done in FP64 and perturbs O at the unit-roundoff level
    for other, tol in ((Op, 1e-24), (np.conj(O), 1e-24), (Oph, 1e-13)):
        v = orc.tor(other, mode=orc.QUAD).value
        assert abs(v - base) <= tol * sum_abs, (v, base)


def test_subtree_restriction_sums_to_total():
    n, k = 9, 3
    O = gen.random_O(n, 5)
    full = orc.tor(O, mode=orc.F64)
    parts = [orc.tor(O, mode=orc.F64, fix_mask=(1 << k) - 1, fix_val=v) for v in range(1 << k)]
    assert sum(p.count for p in parts) == 1 << n
    # FP64 terms are all >= 1 in magnitude, so their sums are exact in quad
    assert sum(p.hi for p in parts) == full.hi


def test_det_matches_numpy():
    n = 7
    O = gen.random_O(n, 2)
    C = np.eye(2 * n) - O
    C = np.tril(C) + np.tril(C, -1).conj().T  # Hermitian completion of the lower triangle
    rng = np.random.default_rng(3)
    for Z in rng.integers(1, 1 << n, size=20):
        modes = [i for i in range(n) if (int(Z) >> i) & 1]
        idx = modes + [m + n for m in modes]
        want = np.linalg.det(C[np.ix_(idx, idx)]).real
        got, t = orc.det(O, int(Z))
        assert abs(got - want) <= 1e-12 * want
        assert abs(abs(t) - 1 / np.sqrt(want)) <= 1e-12 / np.sqrt(want)


def test_not_positive_definite_raises():
    n = 3
    O = gen.random_O(n, 0)
    O = O + 2.0 * np.eye(2 * n)  # I - O has negative eigenvalues
    with pytest.raises(orc.OracleError):
        orc.tor(O)


def test_threads_do_not_change_fp64_result():
    O = gen.random_O(10, 0)
    a = orc.tor(O, threads=1)
    b = orc.tor(O, threads=7)
    assert a.hi == b.hi and a.sum_abs == b.sum_abs


def test_fp64_mode_within_error_model():
    O = gen.random_O(10, 0)  # first workload's generator: n = 10, r ~ U[.5, 1], eta = .5
    f = orc.tor(O, mode=orc.F64)
    q = orc.tor(O, mode=orc.QUAD)
    rel = abs(f.value - q.value) / abs(q.value)
    assert rel <= 1e-10, rel


# ---------------------------------------------------------------------------
# mutation tests: a planted mistake in the oracle must fail some pin
# ---------------------------------------------------------------------------

MUTANTS = {
    "sign_ignores_n": ("const int neg = (n - m / 2) & 1;", "const int neg = (m / 2) & 1;"),
    "no_conjugate": ("W[2 * ((long)i * m + j) + 1] -= li * br - lr * bi;",
                     "W[2 * ((long)i * m + j) + 1] -= li * br + lr * bi;"),
    "drop_empty_subset": ("uint64_t Z = deposit(c, jb->free_mask) | jb->fix_val;",
                          "uint64_t Z = deposit(c, jb->free_mask) | jb->fix_val;\n        if (!Z) continue;"),
    "short_update": ("for (int j = k + 1; j <= i; j++) {", "for (int j = k + 1; j < i; j++) {"),
    "det_not_squared": ("d *= p;", "d *= sqrt((double)p);"),
    "wrong_partner_row": ("idx[m++] = idx[t] + n;", "idx[m++] = (idx[t] + 1) % n + n;"),
}


def _build_mutant(name, tmp):
    src = open(os.path.join(os.path.dirname(orc.__file__), "tor_oracle.c")).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    src = src.replace(old, new)
    cpath = os.path.join(tmp, f"{name}.c")
    lpath = os.path.join(tmp, f"lib{name}.so")
    with open(cpath, "w") as f:
        f.write(src)
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-pthread", "-ffp-contract=off", cpath,
                    "-o", lpath, "-lquadmath", "-lm"], check=True)
    lib = ctypes.CDLL(lpath)
    lib.oracle_tor.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_long, ctypes.c_int,
                               ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                               ctypes.POINTER(ctypes.c_double)]

    def tor(O, mode):
        O = np.ascontiguousarray(O, dtype=np.complex128)
        n = O.shape[0] // 2
        out = (ctypes.c_double * 5)()
        rc = lib.oracle_tor(n, O.ctypes.data if n else None, max(2 * n, 1), mode, 2, 0, 0, out)
        if rc != 0:
            raise orc.OracleError(str(rc))
        return out[0] + out[1]

    return tor


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    with tempfile.TemporaryDirectory() as tmp:
        tor = _build_mutant(name, tmp)
        failed = []
        for pin in ALL_PINS:
            try:
                pin(tor)
            except (AssertionError, orc.OracleError, ZeroDivisionError, FloatingPointError):
                failed.append(pin.__name__)
        assert failed, f"mutant {name} passed every pin"
