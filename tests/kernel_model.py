"""A slow numpy model of the GPU kernel's work split, for CPU tests only.

It follows the kernel's bookkeeping step by step -- the packed reversed
layout, the root split over modes 0..k-1, the tier-A binary counter with its
stack of include levels, the tier-B node ids and views, and the tier-C lane
decisions and signs -- so that an indexing or sign mistake in that design
shows up against the oracle without a GPU.  Neither the oracle nor the
library imports it.
"""
from __future__ import annotations

import math

import numpy as np


def E(s):
    return s * (2 * s + 1)


def pidx(x, y):
    return x * (x + 1) // 2 + y


def pack(O: np.ndarray, min_modes: int):
    """Device layout: Hermitian completion of the lower triangle of I - O,
    mode-interleaved rows, reversed, lower-packed; padded with modes whose
    block of I - O is I/2."""
    n = O.shape[0] // 2
    C = np.eye(2 * n, dtype=np.complex128) - O
    C = np.tril(C) + np.tril(C, -1).conj().T
    N = max(n, min_modes)
    out = np.zeros(E(N), dtype=np.complex128)

    def elem(qi, qj):
        mi, ci, mj, cj = qi // 2, qi % 2, qj // 2, qj % 2
        if mi >= n or mj >= n:
            return 0.5 if qi == qj else 0.0
        return C[mi + ci * n, mj + cj * n]

    for x in range(2 * N):
        for y in range(x + 1):
            v = elem(2 * N - 1 - x, 2 * N - 1 - y)
            out[pidx(x, y)] = v.real if x == y else v
    return out, N


def pack_real(O: np.ndarray, min_modes: int):
    """Real form of a Gaussian-state matrix: each mode block of I - O,
    [[p, q], [conj q, conj p]], conjugated by w = [[1, 1], [-i, i]]/sqrt(2),
    becomes [[Re p + Re q, Im q - Im p], [Im p + Im q, Re p - Re q]]."""
    n = O.shape[0] // 2
    C = np.eye(2 * n, dtype=np.complex128) - O
    C = np.tril(C) + np.tril(C, -1).conj().T
    w = np.array([[1, 1], [-1j, 1j]]) / np.sqrt(2)
    N = max(n, min_modes)
    M = np.zeros((2 * N, 2 * N))
    for i in range(N):
        for j in range(N):
            if i < n and j < n:
                blk = np.array([[C[i, j], C[i, j + n]], [C[i + n, j], C[i + n, j + n]]])
                r = w @ blk @ w.conj().T
                assert abs(r.imag).max() < 1e-12
                M[2 * i:2 * i + 2, 2 * j:2 * j + 2] = r.real
            elif i == j:
                M[2 * i:2 * i + 2, 2 * j:2 * j + 2] = 0.5 * np.eye(2)
    out = np.zeros(E(N))
    for x in range(2 * N):
        for y in range(x + 1):
            out[pidx(x, y)] = M[2 * N - 1 - x, 2 * N - 1 - y]
    return out, N


def eliminate(src: np.ndarray, s: int):
    """Include the next mode of an s-mode view: returns (s-1)-mode node, pivot det."""
    p = 2 * s - 2
    a = src[pidx(p, p)].real
    b = src[pidx(p + 1, p)]
    g = src[pidx(p + 1, p + 1)].real
    inv_a = 1.0 / a
    ba = b * inv_a
    g1 = g - abs(b) ** 2 * inv_a
    inv_g = 1.0 / g1
    r1 = np.array([src[pidx(p, y)] for y in range(p)])
    r2 = np.array([src[pidx(p + 1, y)] for y in range(p)]) - r1 * ba
    u1, u2 = r1 * inv_a, r2 * inv_g
    dst = np.zeros(E(s - 1), dtype=src.dtype)
    for x in range(p):
        for y in range(x + 1):
            v = src[pidx(x, y)] - np.conj(u1[x]) * r1[y] - np.conj(u2[x]) * r2[y]
            dst[pidx(x, y)] = v.real if x == y else v
    return dst, a * g1


def tail(h, M, det, sgn, terms, store=None, idx=0):
    """The last M modes of a lane; with store, each term is also recorded
    under its subset index (bit M-1 of the tail's part = the decision when M
    modes are left)."""
    if M == 0:
        terms.append(sgn / math.sqrt(det))
        if store is not None:
            assert idx not in store
            store[idx] = terms[-1]
        return
    tail(h, M - 1, det, -sgn, terms, store, idx)
    hn, pd = eliminate(h, M)
    tail(hn, M - 1, det * pd, sgn, terms, store, idx | (1 << (M - 1)))


def model_tor(O: np.ndarray, T: int = 3, B: int = 6, k: int = 0, real: bool = False, L: int = 1, store=None):
    """Tor, term count and sum |t| by the kernel's schedule.  With a dict
    store, every term is also recorded under the subset index the storing
    kernel writes it to: bit N-1-l for the decision at level l, formed as the
    root's k bits reversed, then the tier-A leaf x, then the lane, then the
    tail's bits."""
    R = T + B
    C, N = pack_real(O, R) if real else pack(O, R)
    LA = N - R
    k = min(k, LA)
    D = LA - k
    terms = []
    for root in range(1 << k):
        slots = {}
        rsrc, rdet, rinc = C, 1.0, 0
        for l in range(k):
            if (root >> l) & 1:
                rsrc, pd = eliminate(rsrc, N - l)
                rdet *= pd
                rinc += 1
        sdet, sinc = {}, {}
        for x in range(1 << D):
            if x == 0:
                lsrc, ldet, linc = rsrc, rdet, rinc
            else:
                t = (x & -x).bit_length() - 1
                lvl = LA - 1 - t
                xr = x >> (t + 1)
                if xr == 0:
                    s, sd, si = rsrc, rdet, rinc
                else:
                    sl = LA - (((xr & -xr).bit_length() - 1) + t + 1)
                    s, sd, si = slots[sl], sdet[sl], sinc[sl]
                    # the kernel does not store the count: it is the root's
                    # includes plus the set bits of x above level sl
                    assert si == rinc + bin(x >> (LA - sl)).count("1")
                dst, pd = eliminate(s, N - lvl)
                slots[lvl + 1] = dst
                sdet[lvl + 1] = sd * pd
                sinc[lvl + 1] = si + 1
                lsrc, ldet, linc = dst, sd * pd, si + 1
            # tier B: levels 1..B-1, node ids, views
            leaf = lsrc[: E(R)].copy()
            nodes = {}  # (level, include index) -> (array, det)

            def node_src(jl, i):
                if i == 0:
                    return leaf, ldet
                t2 = (i & -i).bit_length() - 1
                lev = jl - t2
                return nodes[(lev, (i >> t2) >> 1)]

            for J in range(1, B - L + 1):
                sp = R - (J - 1)
                for i in range(1 << (J - 1)):
                    par, pdp = node_src(J - 1, i)
                    child, pd = eliminate(par, sp)
                    nodes[(J, i)] = (child, pdp * pd)
            # tier C: lane l takes the last L levels, then the last T modes
            for lane in range(1 << B):
                ip = lane >> L
                src, det = node_src(B - L, ip)
                h = src[: E(T + L)].copy()
                includes = linc + bin(ip).count("1")
                for j in range(L):
                    inc = (lane >> (L - 1 - j)) & 1
                    M = T + L - j
                    if inc:
                        h, pd = eliminate(h, M)
                        det *= pd
                    else:
                        h = h[: E(M - 1)].copy()
                    includes += inc
                excluded = (N - T) - includes
                rrev = int(format(root, f"0{k}b")[::-1], 2) if k else 0
                base = (rrev << (N - k)) | (x << R) | (lane << T)
                tail(h, T, det, -1.0 if excluded & 1 else 1.0, terms, store, base)
    return math.fsum(terms), len(terms), math.fsum(abs(t) for t in terms)
