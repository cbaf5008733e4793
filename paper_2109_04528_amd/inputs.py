"""Seeded synthetic inputs: Gaussian-state sampling matrices O (2n x 2n complex128).

This module only builds inputs.  It holds none of the Torontonian arithmetic and
is shared by the tests, the benchmark and the CPU oracle's callers, so that the
GPU path and the oracle see identical bytes.

The paper evaluates the Torontonian on the sampling matrix A = I - Sigma^{-1}
built from the Husimi covariance of a Gaussian state (Sec. 1, Eq. 1) and only
says "random sampling matrix" with a squeezing parameter; the concrete recipe
here is this project's reading:

* squeezing r_i ~ U[r_lo, r_hi], drawn first from ``numpy.random.default_rng(seed)``;
* a Haar unitary U: QR of an n x n complex Gaussian (real parts drawn before
  imaginary parts, each N(0,1)/sqrt(2)), phases fixed by Q diag(R_ii/|R_ii|)
  (Mezzadri's construction);
* S = [[U, 0], [0, conj U]] [[cosh r, sinh r], [sinh r, cosh r]],
  sigma = (eta S S^H + (1 - eta) I) / 2, sigma_Q = sigma + I/2,
  O = I - sigma_Q^{-1}  (block order a_1..a_n, a_1^dag..a_n^dag).

Mode i owns rows/columns {i, i + n}.  A click pattern S selects the principal
submatrix on {s, s + M : s in S} of an M-mode state.
"""
from __future__ import annotations

import hashlib

import numpy as np

__all__ = [
    "haar_unitary",
    "gaussian_state_O",
    "random_O",
    "product_state_O",
    "click_submatrix",
    "vacuum_O",
    "sigma_Q_from_O",
    "sha256",
    "batch_mix",
    "random_hpd_O",
]


def haar_unitary(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed n x n unitary (QR of a complex Gaussian, phase-fixed)."""
    re = rng.standard_normal((n, n))
    im = rng.standard_normal((n, n))
    z = (re + 1j * im) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    ph = d / np.abs(d)
    return q * ph[None, :]


def gaussian_state_O(U: np.ndarray, r: np.ndarray, eta: float) -> np.ndarray:
    """O = I - sigma_Q^{-1} for squeezed vacua r through U with uniform loss eta."""
    n = U.shape[0]
    r = np.asarray(r, dtype=np.float64)
    ch = np.diag(np.cosh(r))
    sh = np.diag(np.sinh(r))
    z = np.zeros((n, n), dtype=np.complex128)
    big_u = np.block([[U, z], [z, np.conj(U)]])
    sq = np.block([[ch, sh], [sh, ch]]).astype(np.complex128)
    S = big_u @ sq
    eye = np.eye(2 * n, dtype=np.complex128)
    sigma = (eta * (S @ S.conj().T) + (1.0 - eta) * eye) / 2.0
    sigma_q = sigma + eye / 2.0
    O = eye - np.linalg.inv(sigma_q)
    return np.ascontiguousarray(O, dtype=np.complex128)


def random_O(n: int, seed: int, r_lo: float = 0.5, r_hi: float = 1.0,
             eta: float = 0.5) -> np.ndarray:
    """The seeded generator: r first, then the Haar unitary, then O."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(r_lo, r_hi, n)
    U = haar_unitary(n, rng)
    return gaussian_state_O(U, r, eta)


def product_state_O(r, eta: float, phases=None) -> np.ndarray:
    """Independent single-mode squeezed states (U diagonal with given phases)."""
    r = np.asarray(r, dtype=np.float64)
    n = r.size
    if phases is None:
        phases = np.zeros(n)
    U = np.diag(np.exp(1j * np.asarray(phases, dtype=np.float64)))
    return gaussian_state_O(U, r, eta)


def vacuum_O(n: int) -> np.ndarray:
    return np.zeros((2 * n, 2 * n), dtype=np.complex128)


def sigma_Q_from_O(O: np.ndarray) -> np.ndarray:
    eye = np.eye(O.shape[0], dtype=np.complex128)
    return np.linalg.inv(eye - O)


def click_submatrix(O: np.ndarray, modes) -> np.ndarray:
    """Principal submatrix of an M-mode O on rows/cols {s, s+M : s in modes}."""
    M = O.shape[0] // 2
    modes = np.asarray(sorted(modes), dtype=np.int64)
    idx = np.concatenate([modes, modes + M])
    return np.ascontiguousarray(O[np.ix_(idx, idx)])


def random_hpd_O(n: int, seed: int, lam_lo: float = 0.05, lam_hi: float = 0.95) -> np.ndarray:
    """A generic Hermitian O with eigenvalues in [lam_lo, lam_hi] and no
    Gaussian-state structure (tests the general complex path)."""
    rng = np.random.default_rng(seed)
    V = haar_unitary(2 * n, rng)
    lam = rng.uniform(lam_lo, lam_hi, 2 * n)
    O = (V * lam[None, :]) @ V.conj().T
    O = (O + O.conj().T) / 2.0
    return np.ascontiguousarray(O, dtype=np.complex128)


def batch_mix(count: int = 512, n_lo: int = 12, n_hi: int = 26, seed: int = 4,
              base_seed: int = 1000):
    """Batched workload: n ~ U{n_lo..n_hi} from rng(seed); matrix i uses seed
    base_seed + i with r ~ U[.5, 1] and eta ~ U[.3, 1]."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    mats = []
    for i, n in enumerate(ns):
        r2 = np.random.default_rng(base_seed + i)
        eta = r2.uniform(0.3, 1.0)
        r = r2.uniform(0.5, 1.0, int(n))
        U = haar_unitary(int(n), r2)
        mats.append(gaussian_state_O(U, r, eta))
    return [int(v) for v in ns], mats


def structured_O(O: np.ndarray) -> np.ndarray:
    """O with the exact Gaussian-state block form: I - O = [[P, Q], [conj Q,
    conj P]] with Q symmetric, taking P and Q as the averages of the two
    copies each block has in a numerically computed state (they agree to
    rounding).  Inputs built this way describe the same matrix on every
    evaluation path."""
    n = O.shape[0] // 2
    C = np.eye(2 * n) - O
    C = np.tril(C) + np.tril(C, -1).conj().T
    P, Q, P2, Q2 = C[:n, :n], C[:n, n:], C[n:, n:], C[n:, :n]
    Pa = 0.5 * (P + P2.conj())
    Qa = 0.25 * (Q + Q.T + (Q2 + Q2.T).conj())
    Pa[np.diag_indices(n)] = Pa.diagonal().real
    Ca = np.block([[Pa, Qa], [Qa.conj(), Pa.conj()]])
    return np.eye(2 * n) - Ca


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
