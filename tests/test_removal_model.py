"""The removal-order kernel's bookkeeping (tests/removal_model.py: per-level
trailing rows, rows looked up at the deepest level below their mode)
reproduces the oracle on small inputs."""
import pytest

from oracle import oracle as orc
from paper_2109_04528_amd import inputs as gen
from removal_model import model_removal_tor


@pytest.mark.parametrize("n,k", [(0, 0), (1, 0), (2, 1), (5, 0), (6, 2), (8, 3), (9, 9)])
def test_removal_model_matches_oracle(n, k):
    O = gen.random_O(n, 40 + n, 0.5, 1.0, 0.7) if n else gen.vacuum_O(0)
    v, cnt = model_removal_tor(O, k)
    q = orc.tor(O, mode=orc.QUAD)
    assert cnt == 1 << n
    assert abs(v - q.value) <= 64 * 1.1e-16 * max(n, 1) * q.sum_abs, (v, q.value)


def test_removal_model_general_hermitian():
    O = gen.random_hpd_O(7, 3)
    v, _ = model_removal_tor(O, 2)
    q = orc.tor(O, mode=orc.QUAD)
    assert abs(v - q.value) <= 64 * 1.1e-16 * 7 * q.sum_abs


@pytest.mark.parametrize("n", [1, 3, 6])
def test_removal_flop_model_matches_instrumented_count(n):
    from paper_2109_04528_amd.flops import removal_flops
    O = gen.random_O(n, 1, 0.5, 1.0, 0.7)
    cnt = [0]
    model_removal_tor(O, 0, cnt)
    assert cnt[0] == removal_flops(n)
