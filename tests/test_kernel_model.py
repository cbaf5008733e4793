"""The kernel's work split and sign bookkeeping, modelled in numpy
(tests/kernel_model.py), reproduces the oracle on small inputs."""
import math

import numpy as np
import pytest

import kernel_model as km
from kernel_model import model_tor
from oracle import oracle as orc
from paper_2109_04528_amd import inputs as gen


# the complex path: T = 3 register modes, B = 6 (64 lanes), L = 2 lane levels
# (12, 0) walks three tier-A levels (stack slots, stored determinants)
@pytest.mark.parametrize("n,k", [(0, 0), (1, 0), (5, 0), (9, 0), (10, 1), (11, 2), (12, 3), (12, 0)])
def test_model_matches_oracle(n, k):
    O = gen.random_O(n, 3 + n, 0.5, 1.0, 0.7) if n else gen.vacuum_O(0)
    v, cnt, sabs = model_tor(O, 3, 6, k, L=2)
    q = orc.tor(O, mode=orc.QUAD)
    assert cnt == 1 << max(n, 9)
    tol = 64 * 1.1e-16 * max(n, 9) * q.sum_abs
    assert abs(v - q.value) <= tol, (v, q.value, tol)
    # each padding mode (block I/2) turns a term t into -t and +2t
    pad = max(n, 9) - n
    assert abs(sabs - 3.0 ** pad * q.sum_abs) <= 1e-12 * sabs


def test_model_product_state_closed_form():
    r = np.array([0.6, 0.8, 1.0, 0.7, 0.9, 0.55, 0.65, 0.75, 0.85, 0.95, 0.5])
    O = gen.product_state_O(r, 0.6, np.arange(11.0))
    v, _, _ = model_tor(O, 3, 6, 1, L=1)
    single = np.sqrt(1 + 0.6 * 1.4 * np.sinh(r) ** 2)
    want = float(np.prod(single - 1))
    sum_abs = float(np.prod(single + 1))  # sum of |terms| of a product state
    assert abs(v - want) <= 64 * 1.1e-16 * 11 * sum_abs


# the real path: T = 5, B = 6, L = 2
@pytest.mark.parametrize("n,k", [(4, 0), (11, 0), (12, 1), (13, 2), (14, 0)])
def test_real_form_model_matches_oracle(n, k):
    O = gen.random_O(n, 50 + n, 0.3, 1.2, 0.9)
    v, cnt, sabs = model_tor(O, 5, 6, k, real=True, L=2)
    q = orc.tor(O, mode=orc.QUAD)
    assert cnt == 1 << max(n, 11)
    assert abs(v - q.value) <= 64 * 1.1e-16 * max(n, 11) * q.sum_abs, (v, q.value)
    pad = max(n, 11) - n
    assert abs(sabs - 3.0 ** pad * q.sum_abs) <= 1e-12 * sabs


# the double-double factor: real form, T = 3, B = 6, L = 2
@pytest.mark.parametrize("n,k", [(6, 0), (9, 0), (11, 1), (12, 2), (12, 0)])
def test_quad_config_model_matches_oracle(n, k):
    O = gen.random_O(n, 70 + n, 0.3, 1.2, 0.9)
    v, cnt, _ = model_tor(O, 3, 6, k, real=True, L=2)
    q = orc.tor(O, mode=orc.QUAD)
    assert cnt == 1 << max(n, 9)
    assert abs(v - q.value) <= 64 * 1.1e-16 * max(n, 9) * q.sum_abs, (v, q.value)


@pytest.mark.parametrize("n,k", [(12, 0), (13, 2), (14, 1)])
def test_stored_term_indices(n, k):
    """Every subset's term lands once at the index the storing kernel uses
    (bit N-1-l = mode l included), with the sign and value of Eq. 2: the
    model's store against a direct numpy determinant per subset."""
    import itertools
    O = gen.random_O(n, 7, 0.5, 1.0, 0.7)
    store = {}
    km.model_tor(O, T=5, B=6, k=k, real=True, L=2, store=store)
    N = max(n, 11)
    assert sorted(store) == list(range(1 << N))
    C = np.eye(2 * n) - O
    rng = np.random.default_rng(0)
    for idx in rng.choice(1 << N, 300, replace=False).tolist() + [0, (1 << N) - 1]:
        modes = [l for l in range(N) if (idx >> (N - 1 - l)) & 1]
        real_modes = [m for m in modes if m < n]
        sel = real_modes + [m + n for m in real_modes]
        d = np.linalg.det(C[np.ix_(sel, sel)]).real if real_modes else 1.0
        d *= 0.25 ** (len(modes) - len(real_modes))  # padding blocks I/2
        want = (-1) ** (N - len(modes)) / math.sqrt(d)
        assert abs(store[idx] - want) <= 1e-9 * abs(want)
