"""A slow numpy model of the removal-order kernel's bookkeeping, for CPU
tests only (neither the oracle nor the library imports it).

The removal order of Sec. 2 (Algorithm 2): the Cholesky factor L of the
matrix of kept modes (interleaved order, a_q and a_q^dag of each kept mode q
in increasing q) is reused when a further mode i, larger than every mode
removed so far, is removed: the rows and columns of the kept modes below i
(L11) and the rows of the modes above i restricted to those columns (L21)
stay, and the trailing block is factorised afresh,
L22' = chol(C22 - L21 L21^H), with C22 the block of I - O on the modes above
i.

The kernel stores, per depth of its depth-first walk, only the rows of the
modes above that depth's removed mode.  A row of mode q never changes while
the walk stays below a removal smaller than q, and its columns (kept modes
below q) are the same in every such node, so the row of mode q in the
current node is the one stored at the deepest level whose removed mode is
below q.  The model follows exactly that layout.
"""
from __future__ import annotations

import math

import numpy as np


def interleaved_C(O: np.ndarray) -> np.ndarray:
    """Hermitian completion of the lower triangle of I - O, rows in the
    interleaved order a_0, a_0^dag, a_1, a_1^dag, ..."""
    n = O.shape[0] // 2
    C = np.eye(2 * n, dtype=np.complex128) - O
    C = np.tril(C) + np.tril(C, -1).conj().T
    perm = np.empty(2 * n, dtype=np.int64)
    perm[0::2] = np.arange(n)
    perm[1::2] = np.arange(n) + n
    Ci = C[np.ix_(perm, perm)]
    Ci[np.diag_indices(2 * n)] = Ci.diagonal().real
    return Ci


def chol_count(s2):
    """Operations of a scalar complex Cholesky of size s2, counted the way
    the kernel does them (sqrt and reciprocal, column scale, trailing
    multiply-subtracts)."""
    tot = 0
    for j in range(s2):
        for x in range(j + 1, s2):
            tot += 2  # scale by the real reciprocal
            for y in range(j + 1, x + 1):
                tot += 8  # complex multiply-subtract
        tot += 2
    return tot


def model_removal_tor(O: np.ndarray, k: int = 0, count: list | None = None):
    """Tor by the removal order with 2^k roots (the removal decisions on
    modes 0..k-1); returns (value, number of terms).  With count (a one-item
    list) the operations are tallied into count[0]."""
    n = O.shape[0] // 2
    C = interleaved_C(O)
    k = min(k, n)
    terms = []
    for root in range(1 << k):
        removed0 = [q for q in range(k) if (root >> q) & 1]
        kept0 = [q for q in range(n) if q not in removed0]
        # root node: a fresh factorisation
        idx = [2 * q + c for q in kept0 for c in (0, 1)]
        L0 = np.linalg.cholesky(C[np.ix_(idx, idx)]) if idx else np.zeros((0, 0))
        if count is not None:
            count[0] += chol_count(len(idx))
        # levels: (removed mode, {mode q: row pair of L for q}); level 0 has
        # every kept mode's rows, as if a mode -1 had been removed
        rows0 = {q: L0[2 * j:2 * j + 2, :2 * j + 2] for j, q in enumerate(kept0)}
        levels = [(-1, rows0)]

        def row_of(q):
            for rm, rows in reversed(levels):
                if rm < q:
                    return rows[q]
            raise AssertionError

        def kept_rank(q, removed):
            return q - sum(1 for r in removed if r < q)

        def term(removed):
            d = 1.0
            for q in range(n):
                if q in removed:
                    continue
                r = row_of(q)
                j = 2 * kept_rank(q, removed)
                d *= abs(r[0, j]) ** 2 * abs(r[1, j + 1]) ** 2
            terms.append((-1.0) ** len(removed) / math.sqrt(d))
            if count is not None:
                count[0] += 2

        removed = list(removed0)
        term(removed)

        def walk(last):
            for i in range(max(last + 1, k), n):
                c = kept_rank(i, removed)  # kept modes below i
                trail = list(range(i + 1, n))
                m = len(trail)
                # L21 from the rows of the trailing modes, first 2c columns
                L21 = np.zeros((2 * m, 2 * c), dtype=np.complex128)
                for t, q in enumerate(trail):
                    L21[2 * t:2 * t + 2] = row_of(q)[:, :2 * c]
                tix = [2 * q + cc for q in trail for cc in (0, 1)]
                S = C[np.ix_(tix, tix)] - L21 @ L21.conj().T
                if count is not None:
                    count[0] += 8 * (2 * c) * (2 * m * (2 * m + 1) // 2) + chol_count(2 * m)
                L22 = np.linalg.cholesky(S) if m else np.zeros((0, 0))
                rows = {}
                for t, q in enumerate(trail):
                    rows[q] = np.hstack([L21[2 * t:2 * t + 2], L22[2 * t:2 * t + 2, :2 * t + 2]])
                removed.append(i)
                levels.append((i, rows))
                term(removed)
                walk(i)
                levels.pop()
                removed.pop()

        walk(k - 1)
    return math.fsum(terms), len(terms)
