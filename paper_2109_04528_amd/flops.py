"""Algorithmic operation count of the recursive Torontonian (for rooflines).

The include/exclude tree over N modes has 2^l nodes at level l; each node's
include child is one elimination of the (N - l)-mode view, each leaf one term.
Counted as real FLOPs, an FMA counting 2 and a reciprocal or (reciprocal)
square root counting 1; the compensation steps of the double-double sum are
not counted.  For an elimination of s modes (p = 2s - 2 rows kept):

* complex path: pivot 10, pivot-row vectors 12 p, rank-2 update 8 p^2
  (an off-diagonal complex entry is 8 FMA = 16 FLOP, a real diagonal entry
  4 FMA = 8 FLOP): cost(s) = 8 p^2 + 12 p + 10;
* real path: pivot 8, vectors 4 p, update 2 p^2 + 2 p (2 FMA per entry):
  cost(s) = 2 p^2 + 6 p + 8;

the last mode (s = 1) only needs the 2x2 determinant (4 FLOP complex, 3 real),
and every include multiplies the running determinant (1 FLOP).  Each leaf
takes a reciprocal square root and one addition (2 FLOP).
"""


def elim_cost(s: int, real: bool = False) -> int:
    if s <= 1:
        return 3 if real else 4
    p = 2 * s - 2
    if real:
        return 2 * p * p + 6 * p + 8
    return 8 * p * p + 12 * p + 10


def tor_flops(n: int, real: bool = False) -> int:
    """Algorithmic FLOPs of one Torontonian of n modes (no padding counted)."""
    total = 2 * (1 << n)
    for level in range(n):
        total += (1 << level) * (elim_cost(n - level, real) + 1)
    return total


def flops_per_subset(n: int, real: bool = False) -> float:
    return tor_flops(n, real) / float(1 << n)


def plain_flops_per_subset(n: int, real: bool = False) -> float:
    """A fresh factorisation per subset: sum over subsets of the eliminations
    of sizes d, d-1, ..., 1 for |Z| = d, averaged (real: the quadrature form)."""
    from math import comb
    tot = 0
    for d in range(n + 1):
        c = sum(elim_cost(s, real) + 1 for s in range(1, d + 1)) + 2
        tot += comb(n, d) * c
    return tot / float(1 << n)


def chol_flops(s2: int) -> int:
    """Scalar complex Cholesky of an s2 x s2 Hermitian matrix (Algorithm 1):
    per column a square root and a reciprocal (2), the column scaled by a
    real (2 per entry), and the trailing lower triangle updated by one
    complex multiply-subtract per entry (8)."""
    tot = 0
    for j in range(s2):
        w = s2 - 1 - j
        tot += 2 + 2 * w + 8 * (w * (w + 1) // 2)
    return tot


def removal_flops(n: int) -> int:
    """Algorithmic FLOPs of the removal order (Sec. 2, Algorithm 2) for one
    Torontonian of n modes: one factorisation of the full matrix, then for
    every further subset -- remove mode i with c kept modes below it, of
    which there are C(i, c) -- the trailing block C22 - L21 L21^H (its lower
    triangle, 2m(2m+1)/2 entries of 2c complex multiply-subtracts, m = n-1-i)
    and its factorisation; every subset's term costs 2 more."""
    from math import comb
    tot = chol_flops(2 * n) + 2 * (1 << n)
    for i in range(n):
        m = n - 1 - i
        for c in range(i + 1):
            tot += comb(i, c) * (8 * 2 * c * (2 * m * (2 * m + 1) // 2) + chol_flops(2 * m))
    return tot
