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
