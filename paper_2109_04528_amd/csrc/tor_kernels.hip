// tor_kernels.hip -- gfx950 kernels of the recursive Torontonian.
//
// Tor(O) = sum_Z (-1)^(n-|Z|) / sqrt(det (I-O)_Z)   (Eq. 2)
//
// The include/exclude tree over the modes (in order 0..N-1) enumerates every
// subset Z once; a node at level l has decided modes 0..l-1 and carries the
// Schur complement of its included modes over the undecided ones (packed
// layout described in tor_device.hpp).  Excluding the next mode is free (a
// prefix), including it is one rank-2 update whose pivot determinant
// multiplies the running determinant (the product of the new squared diagonal
// entries of the Cholesky factor).  A leaf is one subset: its term is
// (-1)^(#excluded) / sqrt(det).  This is the reuse of Sec. 2 / Algorithm 2 --
// a child only appends the two rows of its new mode to the parent's factor --
// in right-looking form, so each child costs O(remaining modes^2) instead of
// a fresh factorisation.
//
// Work split (one persistent launch, one wavefront per workgroup):
//  * queue items are subtree roots: the include/exclude decisions on modes
//    0..k-1 (the paper's MPI layer hands over only the list of modes and lets
//    the receiver recompute the factor, Sec. 4; here a wave pops a root id
//    from an atomic counter and recomputes the root's Schur complement);
//  * tier A: the wave walks the levels k..N-R-1 depth first; each step that
//    changes the path is one wave-parallel rank-2 update, stacked per level
//    in a private global scratch area (L2-resident);
//  * tier B: from each tier-A leaf (R = T + B modes left) the wave expands
//    B-1 levels breadth first in LDS, every include node of a level updated
//    together (all lanes busy);
//  * tier C: lane l takes node l of level B (its parent is an LDS node of
//    level B-1; odd lanes include, even lanes exclude that mode) and finishes
//    the last T modes alone in registers: 2^T subsets per lane.
// Terms are summed per lane in double-double, reduced over the wave, and
// written to the root's partial slot; a second kernel sums the slots of each
// matrix in index order.
#include <type_traits>

#include "tor_device.hpp"
#include "tor_internal.hpp"

namespace tor {

// ---------------------------------------------------------------------------
// LDS layout of tier B: node 0 (the tier-A leaf, R modes), then for each level
// j = 1..B-1 the 2^(j-1) include nodes of R-j modes.
template <int R>
__host__ __device__ constexpr int offB(int j)
{
    int o = E(R);
    for (int jj = 1; jj < j; ++jj)
        o += (1 << (jj - 1)) * E(R - jj);
    return o;
}

template <int R, int B>
__host__ __device__ constexpr int vec_entries()
{
    int m = 4 * 2 * (MAX_N - 1);  // tier-A elimination of the largest node
    for (int j = 1; j < B; ++j) {
        int v = (1 << (j - 1)) * 4 * (2 * (R - j));
        if (v > m)
            m = v;
    }
    return m;
}

// The node of level jl with id i (bit jl-1-m of i = decision on mode m, 1 =
// include) is a prefix view of the deepest include node on its path.
template <class S, int R>
__device__ __forceinline__ void node_src(int jl, int i, S *bufB, const double *ndet, double leafDet,
                                         const S *&src, double &det)
{
    if (i == 0) {
        src = bufB;
        det = leafDet;
        return;
    }
    int t = __builtin_ctz(i);
    int lev = jl - t;
    int idx = (i >> t) >> 1;
    int off = E(R);
    // offB(lev) at run time (lev <= B-1, small loop)
    for (int jj = 1; jj < lev; ++jj)
        off += (1 << (jj - 1)) * E(R - jj);
    src = bufB + off + idx * E(R - lev);
    det = ndet[(1 << (lev - 1)) - 1 + idx];
}

template <class S>
__device__ __forceinline__ S fix_diag(S v, bool d);
template <>
__device__ __forceinline__ double fix_diag<double>(double v, bool) { return v; }
template <>
__device__ __forceinline__ c64 fix_diag<c64>(c64 v, bool d) { return c64{v.x, d ? 0.0 : v.y}; }

// ---------------------------------------------------------------------------
// one include step on global memory (tier A and root set-up): src is a view
// of s modes (2s rows), dst receives the Schur complement of s-1 modes.
template <class S>
__device__ void elim_global(const S *__restrict__ src, S *__restrict__ dst, int s, S *vec, int lane,
                            double &pdet, int &bad)
{
    const int p = 2 * s - 2;
    const double a = re(src[pidx(p, p)]);
    const S b = src[pidx(p + 1, p)];
    const double g = re(src[pidx(p + 1, p + 1)]);
    Piv<S> pv = pivot(a, b, g);
    pdet = pv.pdet;
    if (!(a > 0.0) || !(pv.pdet > 0.0))
        bad = 1;
    for (int y = lane; y < p; y += 64) {
        S r1 = src[pidx(p, y)];
        S r2 = sub_mul(src[pidx(p + 1, y)], r1, pv.ba);
        vec[y] = scale(r1, pv.inv_a);
        vec[p + y] = r1;
        vec[2 * p + y] = scale(r2, pv.inv_g);
        vec[3 * p + y] = r2;
    }
    __syncthreads();
    const int eo = p * (p + 1) / 2;
    int x = 0, y = lane;
    while (y > x) {
        y -= x + 1;
        ++x;
    }
    for (int e = lane; e < eo; e += 64) {
        S h = src[e];
        S v = upd(h, vec[x], vec[p + y], vec[2 * p + x], vec[3 * p + y]);
        dst[e] = fix_diag(v, x == y);
        y += 64;
        while (y > x) {
            y -= x + 1;
            ++x;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// tier B, level J: every include node of level J from its parent of level J-1
template <class S, int R, int J>
__device__ __forceinline__ void tierB_level(S *bufB, S *vec, double *ndet, const uint16_t *tab,
                                            double leafDet, int lane, int &bad)
{
    constexpr int sp = R - (J - 1);  // modes of the parent view
    constexpr int pv = 2 * sp - 2;   // first pivot row; rows of the child
    constexpr int NN = 1 << (J - 1); // include nodes at level J
    constexpr int EO = E(sp - 1);
    constexpr int OUT = offB<R>(J);
#pragma unroll
    for (int it0 = 0; it0 < NN * pv; it0 += 64) {
        int it = it0 + lane;
        if (it < NN * pv) {
            int i = it / pv, y = it - i * pv;
            const S *par;
            double pdp;
            node_src<S, R>(J - 1, i, bufB, ndet, leafDet, par, pdp);
            double a = re(par[pidx(pv, pv)]);
            S b = par[pidx(pv + 1, pv)];
            double g = re(par[pidx(pv + 1, pv + 1)]);
            Piv<S> pq = pivot(a, b, g);
            S r1 = par[pidx(pv, y)];
            S r2 = sub_mul(par[pidx(pv + 1, y)], r1, pq.ba);
            S *v = vec + i * 4 * pv;
            v[y] = scale(r1, pq.inv_a);
            v[pv + y] = r1;
            v[2 * pv + y] = scale(r2, pq.inv_g);
            v[3 * pv + y] = r2;
            if (y == 0) {
                ndet[NN - 1 + i] = pdp * pq.pdet;
                if (!(a > 0.0) || !(pq.pdet > 0.0))
                    bad = 1;
            }
        }
    }
    __syncthreads();
#pragma unroll 4
    for (int it0 = 0; it0 < NN * EO; it0 += 64) {
        int it = it0 + lane;
        if (it < NN * EO) {
            int i = it / EO, e = it - i * EO;
            int xy = tab[e];
            int x = xy & 0xff, y = xy >> 8;
            const S *par;
            double pdp;
            node_src<S, R>(J - 1, i, bufB, ndet, leafDet, par, pdp);
            const S *v = vec + i * 4 * pv;
            S o = upd(par[e], v[x], v[pv + y], v[2 * pv + x], v[3 * pv + y]);
            bufB[OUT + i * EO + e] = fix_diag(o, x == y);
        }
    }
    __syncthreads();
}

template <class S, int R, int J, int B>
__device__ __forceinline__ void tierB(S *bufB, S *vec, double *ndet, const uint16_t *tab, double leafDet,
                                      int lane, int &bad)
{
    if constexpr (J < B) {
        tierB_level<S, R, J>(bufB, vec, ndet, tab, leafDet, lane, bad);
        tierB<S, R, J + 1, B>(bufB, vec, ndet, tab, leafDet, lane, bad);
    }
}

// ---------------------------------------------------------------------------
// register-resident include step: h has M modes, hn receives M-1 modes
template <class S, int M>
__device__ __forceinline__ void elim_regs(const S *h, const Piv<S> &pq, S *hn)
{
    constexpr int p = 2 * M - 2;
    S u1[p], r1[p], u2[p], r2[p];
#pragma unroll
    for (int y = 0; y < p; ++y) {
        r1[y] = h[pidx(p, y)];
        r2[y] = sub_mul(h[pidx(p + 1, y)], r1[y], pq.ba);
        u1[y] = scale(r1[y], pq.inv_a);
        u2[y] = scale(r2[y], pq.inv_g);
    }
#pragma unroll
    for (int x = 0; x < p; ++x)
#pragma unroll
        for (int y = 0; y <= x; ++y) {
            if (x == y)
                hn[pidx(x, y)] = upd_diag(h[pidx(x, y)], u1[x], r1[y], u2[x], r2[y]);
            else
                hn[pidx(x, y)] = upd(h[pidx(x, y)], u1[x], r1[y], u2[x], r2[y]);
        }
}

// all 2^M subsets below a register-resident node of M modes.
// sgn = (-1)^(#excluded so far); det = running determinant.
template <class S, int M, class Acc>
__device__ __forceinline__ void tail(const S *h, double det, double sgn, Acc &acc, int &bad)
{
    if constexpr (M == 0) {
        acc.add(sgn * rsqrt_nr(det));
    } else {
        tail<S, M - 1, Acc>(h, det, -sgn, acc, bad);  // exclude the next mode
        constexpr int p = 2 * M - 2;
        const double a = re(h[pidx(p, p)]);
        const S b = h[pidx(p + 1, p)];
        const double g = re(h[pidx(p + 1, p + 1)]);
        if constexpr (M == 1) {
            double pd = fma(a, g, -abs2(b));  // det of the last 2x2 block
            if (!(a > 0.0) || !(pd > 0.0))
                bad = 1;
            acc.add(sgn * rsqrt_nr(det * pd));
        } else {
            Piv<S> pq = pivot(a, b, g);
            if (!(a > 0.0) || !(pq.pdet > 0.0))
                bad = 1;
            S hn[E(M - 1)];
            elim_regs<S, M>(h, pq, hn);
            tail<S, M - 1, Acc>(hn, det * pq.pdet, sgn, acc, bad);
        }
    }
}

// tier C: lane l finishes node l of level B
template <class S, int T, int B, class Acc>
__device__ __forceinline__ void tierC(S *bufB, const double *ndet, double leafDet, int leafInc, int N,
                                      int lane, Acc &acc, int &bad)
{
    constexpr int R = T + B;
    const int ip = lane >> 1;  // parent: node of level B-1
    const S *src;
    double sdet;
    node_src<S, R>(B - 1, ip, bufB, ndet, leafDet, src, sdet);
    S h[E(T + 1)];
#pragma unroll
    for (int e = 0; e < E(T + 1); ++e)
        h[e] = src[e];
    constexpr int p = 2 * T;
    const double a = re(h[pidx(p, p)]);
    const S b = h[pidx(p + 1, p)];
    const double g = re(h[pidx(p + 1, p + 1)]);
    Piv<S> pq = pivot(a, b, g);
    const bool inc = lane & 1;
    if (inc && (!(a > 0.0) || !(pq.pdet > 0.0)))
        bad = 1;
    if (!inc) {  // exclude: the update below becomes an exact copy
        pq.inv_a = 0.0;
        pq.inv_g = 0.0;
        pq.ba = zero_of(b);
        pq.pdet = 1.0;
    }
    S hT[E(T)];
    elim_regs<S, T + 1>(h, pq, hT);
    const int includes = leafInc + __popc(ip) + (inc ? 1 : 0);
    const int excluded = (N - T) - includes;
    const double sgn = (excluded & 1) ? -1.0 : 1.0;
    tail<S, T, Acc>(hT, sdet * pq.pdet, sgn, acc, bad);
}

// ---------------------------------------------------------------------------
template <class S, int T, int B, class Acc>
__global__ void __launch_bounds__(64) tor_main(MainParams prm)
{
    constexpr int R = T + B;
    __shared__ S bufB[offB<R>(B)];
    __shared__ S vec[vec_entries<R, B>()];
    __shared__ double ndet[1 << (B - 1)];
    __shared__ uint16_t tab[E(R - 1)];
    __shared__ double sdet[MAX_N + 1];
    __shared__ int sinc[MAX_N + 1];

    const int lane = threadIdx.x;
    for (int e = lane; e < E(R - 1); e += 64) {
        int x = 0, y = e;
        while (y > x) {
            y -= x + 1;
            ++x;
        }
        tab[e] = (uint16_t)(x | (y << 8));
    }
    __syncthreads();
    S *wscr = reinterpret_cast<S *>(prm.scratch + (long long)blockIdx.x * prm.scratch_stride);

    for (;;) {
        // every lane issues the same atomic (only lane 0 adds 1), so the
        // ticket needs no lane-dependent control flow; lane 0's old value is
        // the ticket, taken into scalar registers
        const unsigned long long item = bcast_first(atomicAdd(prm.counter, lane == 0 ? 1ull : 0ull));
        if ((long long)item >= prm.total_items)
            break;
        int lo = 0, hi = prm.nprob - 1;  // last problem with item_begin <= item
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (prm.probs[mid].item_begin <= (long long)item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const ProblemDesc P = prm.probs[lo];
        const long long root = (long long)item - P.item_begin;
        const int N = P.N, k = P.k, LA = N - R, D = LA - k;
        const S *C = reinterpret_cast<const S *>(P.C);
        int bad = 0;

        // root: decisions on modes 0..k-1 given by the bits of root
        const S *rsrc = C;
        double rdet = 1.0;
        int rinc = 0;
        for (int l = 0; l < k; ++l) {
            if ((root >> l) & 1) {
                S *dst = wscr + slot_off(N, l + 1);
                double pd;
                elim_global<S>(rsrc, dst, N - l, vec, lane, pd, bad);
                rdet *= pd;
                ++rinc;
                rsrc = dst;
            }
        }

        Acc acc;
        const long long nleaf = 1ll << D;
        for (long long x = 0; x < nleaf; ++x) {
            const S *lsrc;
            double ldet;
            int linc;
            if (x == 0) {
                lsrc = rsrc;
                ldet = rdet;
                linc = rinc;
            } else {
                // leaf x differs from leaf x-1 from level lvl on: lvl becomes an
                // include, every deeper tier-A level an exclude
                const int t = __builtin_ctzll(x);
                const int lvl = LA - 1 - t;
                const long long xr = x >> (t + 1);
                const S *s;
                double sd;
                int si;
                if (xr == 0) {
                    s = rsrc;
                    sd = rdet;
                    si = rinc;
                } else {
                    const int sl = LA - (__builtin_ctzll(xr) + t + 1);
                    s = wscr + slot_off(N, sl);
                    sd = sdet[sl];
                    si = sinc[sl];
                }
                S *dst = wscr + slot_off(N, lvl + 1);
                double pd;
                elim_global<S>(s, dst, N - lvl, vec, lane, pd, bad);
                lsrc = dst;
                ldet = sd * pd;
                linc = si + 1;
                if (lane == 0) {
                    sdet[lvl + 1] = ldet;
                    sinc[lvl + 1] = linc;
                }
            }
            for (int e = lane; e < E(R); e += 64)
                bufB[e] = lsrc[e];
            __syncthreads();
            tierB<S, R, 1, B>(bufB, vec, ndet, tab, ldet, lane, bad);
            tierC<S, T, B, Acc>(bufB, ndet, ldet, linc, N, lane, acc, bad);
            __syncthreads();
        }

        double h = acc.hi, l = acc.lo, ab = acc.abs_sum;
        constexpr bool is_dd = sizeof(Acc) == sizeof(AccDD) && std::is_same<Acc, AccDD>::value;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            double oh = __shfl_xor(h, off), ol = __shfl_xor(l, off), oa = __shfl_xor(ab, off);
            if constexpr (is_dd)
                dd_add2(h, l, oh, ol);
            else
                h += oh;
            ab += oa;
        }
        const int anybad = __any(bad);
        if (lane == 0) {
            double *sl = prm.slots + 4 * item;
            sl[0] = h;
            sl[1] = l;
            sl[2] = ab;
            sl[3] = anybad ? 1.0 : 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// per-matrix sum of the root slots, in index order
template <bool DD>
__global__ void __launch_bounds__(64) tor_reduce(const ProblemDesc *probs, const double *slots,
                                                 double *results)
{
    const int q = blockIdx.x, lane = threadIdx.x;
    const ProblemDesc P = probs[q];
    const long long nroots = 1ll << P.k;
    double h = 0.0, l = 0.0, ab = 0.0, bad = 0.0;
    for (long long r = lane; r < nroots; r += 64) {
        const double *s = slots + 4 * (P.item_begin + r);
        if (DD)
            dd_add2(h, l, s[0], s[1]);
        else
            h += s[0];
        ab += s[2];
        bad = fmax(bad, s[3]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        double oh = __shfl_xor(h, off), ol = __shfl_xor(l, off);
        if (DD)
            dd_add2(h, l, oh, ol);
        else
            h += oh;
        ab += __shfl_xor(ab, off);
        bad = fmax(bad, __shfl_xor(bad, off));
    }
    if (lane == 0) {
        results[4 * q + 0] = h;
        results[4 * q + 1] = l;
        results[4 * q + 2] = ab;
        results[4 * q + 3] = bad;
    }
}

__global__ void tor_zero(unsigned long long *p, int count)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        p[i] = 0ull;
}

// ---------------------------------------------------------------------------
// Comparison baseline: a fresh factorisation per subset (Algorithm 1 applied
// to each (I-O)_Z independently, two rows at a time), one wave per subset.
constexpr int PLAIN_MAX_N = 34;

template <class S>
__global__ void __launch_bounds__(64) tor_plain(PlainParams prm)
{
    __shared__ S A[E(PLAIN_MAX_N)];
    __shared__ S vec[4 * 2 * PLAIN_MAX_N];
    __shared__ int rows[2 * PLAIN_MAX_N];
    const int lane = threadIdx.x;
    const int n = prm.n;
    const S *C = reinterpret_cast<const S *>(prm.C);
    AccDD acc;
    int bad = 0;
    for (;;) {
        const unsigned long long c = bcast_first(atomicAdd(prm.counter, lane == 0 ? 1ull : 0ull));
        const unsigned long long z0 = prm.mask_begin + c * (unsigned long long)prm.chunk;
        if (z0 >= prm.mask_end)
            break;
        unsigned long long z1 = z0 + prm.chunk;
        if (z1 > prm.mask_end)
            z1 = prm.mask_end;
        for (unsigned long long Z = z0; Z < z1; ++Z) {
            const int d = __popcll(Z);
            // reversed interleaved rows of (I-O)_Z in terms of the full matrix
            for (int q2 = lane; q2 < 2 * d; q2 += 64) {
                // q2 -> mode rank r (from the top), component
                int r = q2 >> 1, cmp = q2 & 1;
                // the r-th highest mode in Z
                unsigned long long zz = Z;
                int m = 63 - __clzll(zz);
                for (int q = 0; q < r; ++q) {
                    zz &= ~(1ull << m);
                    m = 63 - __clzll(zz);
                }
                rows[q2] = 2 * n - 1 - (2 * m + (1 - cmp));
            }
            __syncthreads();
            const int ed = E(d);
            {
                int x = 0, y = lane;
                while (y > x) {
                    y -= x + 1;
                    ++x;
                }
                for (int e = lane; e < ed; e += 64) {
                    A[e] = C[pidx(rows[x], rows[y])];
                    y += 64;
                    while (y > x) {
                        y -= x + 1;
                        ++x;
                    }
                }
            }
            __syncthreads();
            double det = 1.0;
            for (int s = d; s >= 1; --s) {
                const int p = 2 * s - 2;
                const double a = re(A[pidx(p, p)]);
                const S b = A[pidx(p + 1, p)];
                const double g = re(A[pidx(p + 1, p + 1)]);
                Piv<S> pv = pivot(a, b, g);
                if (!(a > 0.0) || !(pv.pdet > 0.0))
                    bad = 1;
                det *= pv.pdet;
                if (s == 1)
                    break;
                for (int y = lane; y < p; y += 64) {
                    S r1 = A[pidx(p, y)];
                    S r2 = sub_mul(A[pidx(p + 1, y)], r1, pv.ba);
                    vec[y] = scale(r1, pv.inv_a);
                    vec[p + y] = r1;
                    vec[2 * p + y] = scale(r2, pv.inv_g);
                    vec[3 * p + y] = r2;
                }
                __syncthreads();
                const int eo = p * (p + 1) / 2;
                int x = 0, y = lane;
                while (y > x) {
                    y -= x + 1;
                    ++x;
                }
                for (int e = lane; e < eo; e += 64) {
                    S v = upd(A[e], vec[x], vec[p + y], vec[2 * p + x], vec[3 * p + y]);
                    A[e] = fix_diag(v, x == y);
                    y += 64;
                    while (y > x) {
                        y -= x + 1;
                        ++x;
                    }
                }
                __syncthreads();
            }
            if (lane == 0) {
                const double t = rsqrt_nr(det);
                acc.add(((n - d) & 1) ? -t : t);
            }
            __syncthreads();
        }
    }
    const int anybad = __any(bad);
    if (lane == 0) {
        double *o = prm.partials + 4 * blockIdx.x;
        o[0] = acc.hi;
        o[1] = acc.lo;
        o[2] = acc.abs_sum;
        o[3] = anybad ? 1.0 : 0.0;
    }
}

__global__ void __launch_bounds__(64) tor_plain_reduce(const double *parts, int nwaves, double *out)
{
    const int lane = threadIdx.x;
    double h = 0.0, l = 0.0, ab = 0.0, bad = 0.0;
    for (int w = lane; w < nwaves; w += 64) {
        dd_add2(h, l, parts[4 * w], parts[4 * w + 1]);
        ab += parts[4 * w + 2];
        bad = fmax(bad, parts[4 * w + 3]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        double oh = __shfl_xor(h, off), ol = __shfl_xor(l, off);
        dd_add2(h, l, oh, ol);
        ab += __shfl_xor(ab, off);
        bad = fmax(bad, __shfl_xor(bad, off));
    }
    if (lane == 0) {
        out[0] = h;
        out[1] = l;
        out[2] = ab;
        out[3] = bad;
    }
}

// accuracy probe of the device reciprocal / reciprocal square root
__global__ void tor_math_probe(const double *x, double *out, int count)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        out[2 * i] = rsqrt_nr(x[i]);
        out[2 * i + 1] = rcp_nr(x[i]);
    }
}

// ---------------------------------------------------------------------------
hipError_t launch_main(bool real_path, bool dd, const MainParams &p, int grid, hipStream_t s)
{
    if (real_path) {
        if (dd)
            hipLaunchKernelGGL((tor_main<double, REAL_T, REAL_B, AccDD>), dim3(grid), dim3(64), 0, s, p);
        else
            hipLaunchKernelGGL((tor_main<double, REAL_T, REAL_B, AccF64>), dim3(grid), dim3(64), 0, s, p);
        return hipGetLastError();
    }
    if (dd)
        hipLaunchKernelGGL((tor_main<c64, CPLX_T, CPLX_B, AccDD>), dim3(grid), dim3(64), 0, s, p);
    else
        hipLaunchKernelGGL((tor_main<c64, CPLX_T, CPLX_B, AccF64>), dim3(grid), dim3(64), 0, s, p);
    return hipGetLastError();
}

template <class S, int T, int B>
constexpr int lds_bytes()
{
    constexpr int R = T + B;
    return (int)(sizeof(S) * (offB<R>(B) + vec_entries<R, B>()) + sizeof(double) * (1 << (B - 1)) + 2 * E(R - 1) +
                 (sizeof(double) + sizeof(int)) * (MAX_N + 1));
}

int main_lds_bytes(bool real_path)
{
    return real_path ? lds_bytes<double, REAL_T, REAL_B>() : lds_bytes<c64, CPLX_T, CPLX_B>();
}

hipError_t launch_reduce(const ProblemDesc *probs, int nprob, const double *slots, double *results, bool dd,
                         hipStream_t s)
{
    if (dd)
        hipLaunchKernelGGL((tor_reduce<true>), dim3(nprob), dim3(64), 0, s, probs, slots, results);
    else
        hipLaunchKernelGGL((tor_reduce<false>), dim3(nprob), dim3(64), 0, s, probs, slots, results);
    return hipGetLastError();
}

hipError_t launch_zero(unsigned long long *p, int count, hipStream_t s)
{
    hipLaunchKernelGGL(tor_zero, dim3((count + 63) / 64), dim3(64), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_plain(const PlainParams &p, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((tor_plain<c64>), dim3(grid), dim3(64), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_plain_reduce(const double *partials, int nwaves, double *result, hipStream_t s)
{
    hipLaunchKernelGGL(tor_plain_reduce, dim3(1), dim3(64), 0, s, partials, nwaves, result);
    return hipGetLastError();
}

hipError_t launch_math_probe(const double *x, double *out, int count, hipStream_t s)
{
    hipLaunchKernelGGL(tor_math_probe, dim3((count + 63) / 64), dim3(64), 0, s, x, out, count);
    return hipGetLastError();
}

}  // namespace tor
