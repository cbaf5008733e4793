"""The input helpers that serve both the oracle and the GPU path."""
import numpy as np

from oracle import oracle as orc
from paper_2109_04528_amd import inputs as gen


def test_structured_O_has_the_exact_block_form():
    for n, seed in [(5, 1), (12, 0)]:
        O = gen.structured_O(gen.random_O(n, seed, 0.3, 1.2, 0.9))
        C = np.eye(2 * n) - O
        assert np.array_equal(C, C.conj().T)
        assert np.array_equal(C[n:, n:], C[:n, :n].conj())
        assert np.array_equal(C[:n, n:], C[:n, n:].T)
        assert np.array_equal(C[n:, :n], C[:n, n:].conj())
        assert np.array_equal(gen.structured_O(O), O)  # a projection


def test_structured_O_moves_tor_by_rounding_only():
    # structured_O changes O by rounding only (its diagonal goes through
    # 1 - (1 - x) in FP64); Tor moves by a few 1e-16 relative, not by R
    # times that
    for n, seed in [(10, 0), (12, 3)]:
        O = gen.random_O(n, seed, 0.3, 1.2, 0.9)
        Oa = gen.structured_O(O)
        assert np.abs(O - Oa).max() < 1e-15
        q, qa = orc.tor(O, mode=orc.QUAD), orc.tor(Oa, mode=orc.QUAD)
        d = (q.hi - qa.hi) + (q.lo - qa.lo)
        assert q.cancellation > 1e4
        assert abs(d) <= 1e-14 * abs(q.value)


def test_gaussian_state_subset_determinants_lie_between_det_and_one():
    """For the O of a Gaussian state, sqrt(det(I - O)) / sqrt(det (I - O)_Z) is
    the probability that no mode outside Z clicks, so det(I - O) <= det (I -
    O)_Z <= 1 for every mode subset Z although I - O has eigenvalues above 1:
    every term of Eq. 2 is at least 1 in magnitude, which makes the
    double-double sums of the library exact."""
    import itertools
    for n, seed, lo, hi, eta in [(9, 0, 0.3, 1.2, 0.9), (8, 1, 0.5, 1.0, 0.7), (7, 2, 1.5, 2.0, 1.0)]:
        O = gen.random_O(n, seed, lo, hi, eta)
        C = np.eye(2 * n) - O
        assert np.linalg.eigvalsh(C).max() > 1.2  # not a contraction
        full = np.linalg.det(C).real
        for k in range(n + 1):
            for Z in itertools.combinations(range(n), k):
                idx = list(Z) + [z + n for z in Z]
                d = np.linalg.det(C[np.ix_(idx, idx)]).real if Z else 1.0
                assert full * (1 - 1e-12) <= d <= 1 + 1e-12
