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
//    in a private global scratch area (L2-resident).  On the real path the
//    node one level above the tier-A leaf (R+1 modes) is kept whole in LDS,
//    so the last tier-A level is included in place in LDS and has no stack
//    slot;
//  * tier B: from each tier-A leaf (R = T + B modes left) the wave expands
//    B-L levels breadth first in LDS, every include node of a level updated
//    together (all lanes busy);
//  * tier C: lane l takes node l of level B.  Its ancestor of level B-L is
//    an LDS node; the lane makes the last L decisions itself (an exclude is
//    a zero update, so all lanes run the same code), fused into one pass over
//    that node, and finishes the last T modes alone in registers: 2^T
//    subsets per lane.
// Terms are summed per lane in double-double, reduced over the wave, and
// written to the root's partial slot; a second kernel sums the slots of each
// matrix in index order.
// The double-double factor's instantiation of the main kernel is built in
// tor_kernels_quad.hip, which includes this file with
// TOR_KERNELS_TEMPLATES_ONLY defined (templates only, no launchers).
#include <type_traits>

#include "tor_device.hpp"
#include "tor_internal.hpp"

namespace tor {

// ---------------------------------------------------------------------------
// LDS placement of the nodes tier B stores: node 0 is the tier-A leaf (R
// modes), node 2^(j-1) + i the include node i of level j (R - j modes), for
// j = 1..BL.  Nodes follow one another in that order, each on a 16-byte
// boundary.  Tier C reads the same entry of all 2^BL nodes in one
// instruction, 2^L lanes per node (lane l reads the node that level-BL view
// l >> L stands for).  LDS serves such an access in groups of lanes that move
// 128 bytes per cycle (256 with 64 banks), and two lanes of one group that
// touch different words of one bank wait for each other.  Each node is
// therefore moved forward (by at most 15 granules) to the first place where
// the start of each of its granule arrays, as a 16-byte slot modulo 8 (and
// modulo 16), differs from that of the other nodes read by the same group of
// lanes; failing that, to the place with the fewest such clashes.
template <int R, int BL, int ESZ, int L, int X0 = 0>
struct NodePlacement {
    static constexpr int NN = 1 << BL;
    int off[NN + 1];
    // the level-BL view whose stored node is t: the include node i of
    // level j is followed by excludes only
    static constexpr int reader(int t)
    {
        if (t == 0)
            return 0;
        int lev = 0;
        while ((1 << lev) <= t)
            ++lev;
        const int idx = t - (1 << (lev - 1));
        return ((idx << 1) | 1) << (BL - lev);
    }
    static constexpr int level(int t)
    {
        int lev = 0;
        while ((1 << lev) <= t)
            ++lev;
        return lev;
    }
    constexpr NodePlacement() : off{}
    {
        constexpr int gpb = 4 / EPG(ESZ);          // granule arrays per node
        constexpr int acc = ESZ == 8 ? 8 : 16;     // bytes per lane per access
        // nodes per lane group and slot modulus: 32 banks, then 64 banks
        constexpr int grp[2] = {(128 / acc) >> L, (256 / acc) >> L};
        constexpr int mods[2] = {8, 16};
        int slot[NN] = {};
        int pos = 0;
        for (int t = 0; t < NN; ++t) {
            const int nb = t == 0 ? NB(R + X0) : NB(R - level(t));
            const int b0 = (pos + 15) & ~15;
            int best = b0, bestc = 1 << 30;
            for (int k = 0; k < 16 && bestc > 0; ++k) {
                const int st = (b0 >> 4) + k;
                int c = 0;
                for (int u = 0; u < t; ++u) {
                    const int unb = u == 0 ? NB(R + X0) : NB(R - level(u));
                    for (int mdl = 0; mdl < 2; ++mdl) {
                        const int G = grp[mdl] > 1 ? grp[mdl] : 1;
                        if (reader(u) / G != reader(t) / G)
                            continue;
                        for (int g = 0; g < gpb; ++g)
                            if ((st + g * nb) % mods[mdl] == (slot[u] + g * unb) % mods[mdl])
                                ++c;
                    }
                }
                if (c < bestc) {
                    bestc = c;
                    best = b0 + 16 * k;
                }
            }
            off[t] = best;
            slot[t] = best >> 4;
            pos = best + ESZ * (t == 0 ? NSZ(R + X0) : NSZ(R - level(t)));
        }
        off[NN] = pos;
    }
};

// 2x2 pivot of the highest mode m of a node, and the update of one output
// block (a, b), a >= b, m > a:
//   H'[x][y] = H[x][y] - conj(r1[x]) r1[y] / alpha - conj(r2'[x]) r2'[y] / gamma1
// with r1 = row 2m, r2' = row 2m+1 - r1 beta/alpha (the LDL form of the 2x2
// pivot); rows 2a, 2a+1 read r1, r2 from block (m, a), columns from (m, b).
//
// A whole block moves as 16-byte granules (node bases and granule arrays
// are 16-byte aligned), one 128-bit access each: lanes on neighbouring
// blocks then touch neighbouring 16-byte words, which LDS serves without
// bank conflicts (two 64-bit halves of a 16-byte stride would conflict)
template <class S>
struct __align__(16) Gran {
    S e[EPG((int)sizeof(S))];
};
template <class S>
__device__ __forceinline__ void get_block(const S *node, int nb, int bi, S *v)
{
    constexpr int G = EPG((int)sizeof(S));
#pragma unroll
    for (int g = 0; g < 4 / G; ++g) {
        const Gran<S> q = *reinterpret_cast<const Gran<S> *>(node + gpos((int)sizeof(S), nb, bi, g * G));
#pragma unroll
        for (int j = 0; j < G; ++j)
            v[g * G + j] = q.e[j];
    }
}
template <class S>
__device__ __forceinline__ void put_block(S *node, int nb, int bi, const S *o)
{
    constexpr int G = EPG((int)sizeof(S));
#pragma unroll
    for (int g = 0; g < 4 / G; ++g) {
        Gran<S> q;
#pragma unroll
        for (int j = 0; j < G; ++j)
            q.e[j] = o[g * G + j];
        *reinterpret_cast<Gran<S> *>(node + gpos((int)sizeof(S), nb, bi, g * G)) = q;
    }
}

// the same accesses through global-address-space pointers (tier A and the
// root path read and write the wave's stack and the matrix in global memory;
// a generic pointer would make them flat accesses)
typedef double dv2 __attribute__((ext_vector_type(2)));
template <class S>
__device__ __forceinline__ void get_block_g(const S *node, int nb, int bi, S *v)
{
    typedef const __attribute__((address_space(1))) dv2 GG;
    constexpr int G = EPG((int)sizeof(S));
#pragma unroll
    for (int g = 0; g < 4 / G; ++g) {
        const dv2 raw = *(GG *)(node + gpos((int)sizeof(S), nb, bi, g * G));
        Gran<S> q;
        __builtin_memcpy(&q, &raw, 16);
#pragma unroll
        for (int j = 0; j < G; ++j)
            v[g * G + j] = q.e[j];
    }
}
template <class S>
__device__ __forceinline__ void put_block_g(S *node, int nb, int bi, const S *o)
{
    typedef __attribute__((address_space(1))) dv2 GG;
    constexpr int G = EPG((int)sizeof(S));
#pragma unroll
    for (int g = 0; g < 4 / G; ++g) {
        Gran<S> q;
#pragma unroll
        for (int j = 0; j < G; ++j)
            q.e[j] = o[g * G + j];
        dv2 raw;
        __builtin_memcpy(&raw, &q, 16);
        *(GG *)(node + gpos((int)sizeof(S), nb, bi, g * G)) = raw;
    }
}
__device__ __forceinline__ double ld_g(const double *p) { return *(const __attribute__((address_space(1))) double *)p; }
template <class S>
__device__ __forceinline__ S ld_g(const S *p)
{
    const dv2 raw = *(const __attribute__((address_space(1))) dv2 *)p;
    S v;
    __builtin_memcpy(&v, &raw, 16);
    return v;
}
template <class S>
__device__ __forceinline__ Piv<S> node_pivot_g(const S *node, int nb, int m)
{
    const int bi = bidx(m, m);
    return pivot(re(ld_g(&blk(node, nb, bi, 0))), ld_g(&blk(node, nb, bi, 2)), re(ld_g(&blk(node, nb, bi, 3))));
}

template <class S>
__device__ __forceinline__ Piv<S> node_pivot(const S *node, int nb, int m)
{
    const int bi = bidx(m, m);
    return pivot(re(blk(node, nb, bi, 0)), blk(node, nb, bi, 2), re(blk(node, nb, bi, 3)));
}

// the update of block (a, b) from its row blocks A = (m, a), Bk = (m, b)
template <class S>
__device__ __forceinline__ void elim_math(const S *A, const S *Bk, const S *H, bool diag, const Piv<S> &pv, S *o)
{
    const S ra0 = A[0], ra1 = A[1];
    const S qa0 = sub_mul(A[2], ra0, pv.ba), qa1 = sub_mul(A[3], ra1, pv.ba);
    const S rb0 = Bk[0], rb1 = Bk[1];
    const S qb0 = sub_mul(Bk[2], rb0, pv.ba), qb1 = sub_mul(Bk[3], rb1, pv.ba);
    const S ua0 = scale(ra0, pv.inv_a), ua1 = scale(ra1, pv.inv_a);
    const S va0 = scale(qa0, pv.inv_g), va1 = scale(qa1, pv.inv_g);
    o[0] = upd(H[0], ua0, rb0, va0, qb0);
    o[1] = upd(H[1], ua0, rb1, va0, qb1);
    o[2] = upd(H[2], ua1, rb0, va1, qb0);
    o[3] = upd(H[3], ua1, rb1, va1, qb1);
    // diagonal block: real diagonal, conjugate upper entry.  Nothing reads
    // the upper entry of a diagonal block (pivots read entries 0, 2, 3, the
    // lanes read the lower triangle), so real scalars leave it as computed.
    if constexpr (std::is_same<S, c64>::value) {
        if (diag) {
            o[0] = fix_diag(o[0]);
            o[3] = fix_diag(o[3]);
            o[1] = conj_of(o[2]);
        }
    }
}

template <class S, bool GLOBAL = false>
__device__ __forceinline__ void elim_block(const S *node, int nb, int m, int a, int b, int ih, const Piv<S> &pv,
                                           S *o)
{
    S A[4], Bk[4], H[4];
    if constexpr (GLOBAL) {
        get_block_g(node, nb, bidx(m, a), A);
        get_block_g(node, nb, bidx(m, b), Bk);
        get_block_g(node, nb, ih, H);
    } else {
        get_block(node, nb, bidx(m, a), A);
        get_block(node, nb, bidx(m, b), Bk);
        get_block(node, nb, ih, H);
    }
    elim_math(A, Bk, H, a == b, pv, o);
}


// ---------------------------------------------------------------------------
// one include step on global memory (tier A and the root path): src is a view
// of s modes of a node with snb blocks per granule array, dst receives the
// Schur complement of s-1 modes as a node with dnb blocks per granule array.
// Every lane forms the pivot itself; lane l updates blocks l, l+64, ...  dst
// (global, may be null) receives the whole child; lds (may be null) receives
// its first nlds blocks (the tier-A leaf) as a node of nlds blocks.
//
// dst may be src itself (the root path eliminates in place, with dnb = snb):
// block (a, b) of the child is read and rewritten by the same lane, and the
// pivot rows (blocks of mode s-1) are never written, so no lane reads a
// block another lane has already replaced.  Block indices do not depend on
// the node's size, so the same lane owns the same block at every step.
template <class S>
__device__ __forceinline__ void elim_global_body(const S *src, int snb, S *dst, int dnb, S *lds, int nlds, int s,
                                                 int lane, RT<S> &pdet, int &bad)
{
    const int m = s - 1;
    const Piv<S> pv = node_pivot_g(src, snb, m);
    pdet = pv.pdet;
    if (!is_pos(pv.pdet) || !is_pos(pv.inv_a))
        bad = 1;
    const int nbo = dst ? NB(m) : nlds;
    for (int bi = lane; bi < nbo; bi += 64) {
        int a, b;
        block_ab(bi, a, b);
        S o[4];
        elim_block<S, true>(src, snb, m, a, b, bidx(a, b), pv, o);
        if (dst)
            put_block_g(dst, dnb, bi, o);
        if (lds && bi < nlds)
            put_block(lds, nlds, bi, o);
    }
    __syncthreads();
}

// the same with src and dst distinct (tier A).  A step of at most 128
// blocks (every step that makes a tier-A leaf, and the deeper stack levels)
// issues the loads of the pivot and of both of each lane's blocks before any
// arithmetic, so it waits for L2 once instead of once for the pivot and once
// per pass; larger steps take the loop above.
template <class S>
__device__ void elim_global(const S *__restrict__ src, int snb, S *__restrict__ dst, int dnb, S *lds, int nlds, int s,
                            int lane, RT<S> &pdet, int &bad)
{
    const int m = s - 1;
    const int nbo = dst ? NB(m) : nlds;
    if (nbo > 128) {
        elim_global_body(src, snb, dst, dnb, lds, nlds, s, lane, pdet, bad);
        return;
    }
    const int bi0 = lane, bi1 = lane + 64;
    const bool h0 = bi0 < nbo, h1 = bi1 < nbo;
    int a0 = 0, b0 = 0, a1 = 0, b1 = 0;
    block_ab(bi0, a0, b0);
    block_ab(bi1, a1, b1);
    S A0[4], B0[4], H0[4], A1[4], B1[4], H1[4];
    const int dbi = bidx(m, m);
    const RT<S> al = re(ld_g(&blk(src, snb, dbi, 0)));
    const S be = ld_g(&blk(src, snb, dbi, 2));
    const RT<S> ga = re(ld_g(&blk(src, snb, dbi, 3)));
    if (h0) {
        get_block_g(src, snb, bidx(m, a0), A0);
        get_block_g(src, snb, bidx(m, b0), B0);
        get_block_g(src, snb, bidx(a0, b0), H0);
    }
    if (h1) {
        get_block_g(src, snb, bidx(m, a1), A1);
        get_block_g(src, snb, bidx(m, b1), B1);
        get_block_g(src, snb, bidx(a1, b1), H1);
    }
    const Piv<S> pv = pivot(al, be, ga);
    pdet = pv.pdet;
    if (!is_pos(pv.pdet) || !is_pos(pv.inv_a))
        bad = 1;
    if (h0) {
        S o[4];
        elim_math(A0, B0, H0, a0 == b0, pv, o);
        if (dst)
            put_block_g(dst, dnb, bi0, o);
        if (lds && bi0 < nlds)
            put_block(lds, nlds, bi0, o);
    }
    if (h1) {
        S o[4];
        elim_math(A1, B1, H1, a1 == b1, pv, o);
        if (dst)
            put_block_g(dst, dnb, bi1, o);
        if (lds && bi1 < nlds)
            put_block(lds, nlds, bi1, o);
    }
    __syncthreads();
}

// in place (dst == src, or src the read-only matrix): the root path
template <class S>
__device__ void elim_inplace(const S *src, int snb, S *dst, int dnb, int s, int lane, RT<S> &pdet, int &bad)
{
    elim_global_body(src, snb, dst, dnb, (S *)nullptr, 0, s, lane, pdet, bad);
}

// the root path in LDS: one include step in place on a node of s modes with
// nb blocks per granule array (each lane rewrites only blocks it reads, and
// never a pivot row, as in elim_inplace)
template <class S>
__device__ __forceinline__ void elim_lds(S *node, int nb, int s, int lane, RT<S> &pdet, int &bad)
{
    const int m = s - 1;
    const Piv<S> pv = node_pivot(node, nb, m);
    pdet = pv.pdet;
    if (!is_pos(pv.pdet) || !is_pos(pv.inv_a))
        bad = 1;
    for (int bi = lane; bi < NB(m); bi += 64) {
        int a, b;
        block_ab(bi, a, b);
        S o[4];
        elim_block<S, false>(node, nb, m, a, b, bidx(a, b), pv, o);
        put_block(node, nb, bi, o);
    }
    __syncthreads();
}

__device__ __forceinline__ void st_g(double *p, double v) { *(__attribute__((address_space(1))) double *)p = v; }
template <class S>
__device__ __forceinline__ void st_g(S *p, S v)
{
    dv2 raw;
    __builtin_memcpy(&raw, &v, 16);
    *(__attribute__((address_space(1))) dv2 *)p = raw;
}

// the first s modes of a node with snb blocks per granule array, copied into
// a node with dnb (global source or destination as flagged)
template <class S, bool SRC_G, bool DST_G>
__device__ __forceinline__ void copy_node(const S *src, int snb, S *dst, int dnb, int s, int lane)
{
    constexpr int G = EPG((int)sizeof(S));
    const int ga = G * NB(s);  // scalars of one granule array
    for (int e = lane; e < NSZ(s); e += 64) {
        const int g = e / ga, r = e - g * ga;
        const S v = SRC_G ? ld_g(&src[g * G * snb + r]) : src[g * G * snb + r];
        if constexpr (DST_G)
            st_g(&dst[g * G * dnb + r], v);
        else
            dst[g * G * dnb + r] = v;
    }
}

// ---------------------------------------------------------------------------
// View t of the tier-B tables: for the node of level jl with id i (bit
// jl-1-m of i = decision on the m-th mode below the tier-A leaf, 1 =
// include; t = (2^jl - 1) + i) the LDS offset of the stored node it is a
// view of, that node's blocks per granule array, and the slot of its
// determinant (0xff: the tier-A leaf).  The include node (lev, idx) keeps
// its determinant at (2^(lev-1) - 1) + idx.
template <int R, int B, int ESZ, int L, int X0>
__device__ __forceinline__ void view_entry(int t, int &off, int &nb, int &det)
{
    static constexpr NodePlacement<R, B - 1, ESZ, L, X0> place{};
    const int jl = 31 - __clz(t + 1);
    const int i = t + 1 - (1 << jl);
    if (i == 0) {
        off = 0;
        nb = NB(R + X0);
        det = 0xff;
    } else {
        const int tz = __builtin_ctz(i);
        const int lev = jl - tz;
        const int idx = (i >> tz) >> 1;
        off = place.off[(1 << (lev - 1)) + idx] / ESZ;
        nb = NB(R - lev);
        det = (1 << (lev - 1)) - 1 + idx;
    }
}

// tier B tables, built once per wave: the view entries above; per include
// node i of level J (record (2^(J-1) - 1) + i) its parent's stored offset
// and blocks per array and its own stored offset, packed in 64 bits; per
// block bi of a child (a, b) and its block index bidx(a, b) packed.
template <class S, int R, int B, int L>
__device__ __forceinline__ void build_tables(uint16_t *srcOff, uint8_t *srcNB, uint8_t *srcDet,
                                             unsigned long long *nodeRec, uint32_t *blkRec, int lane)
{
    constexpr int esz = (int)sizeof(S);
    constexpr int X0 = std::is_same<S, double>::value ? 1 : 0;
    for (int t = lane; t < (1 << B) - 1; t += 64) {
        int off, nb, det;
        view_entry<R, B, esz, L, X0>(t, off, nb, det);
        srcOff[t] = (uint16_t)off;
        srcNB[t] = (uint8_t)nb;
        srcDet[t] = (uint8_t)det;
    }
    // include nodes of levels 1..B-1 (their children are views of level B-1
    // at most)
    for (int t = lane; t < (1 << (B - 1)) - 1; t += 64) {
        const int J = 32 - __clz(t + 1);  // t = (2^(J-1) - 1) + i
        const int i = t + 1 - (1 << (J - 1));
        int poff, pnb, pdet, coff, cnb, cdet;
        view_entry<R, B, esz, L, X0>(t, poff, pnb, pdet);
        view_entry<R, B, esz, L, X0>((1 << J) + 2 * i, coff, cnb, cdet);
        nodeRec[t] = (unsigned long long)(poff * esz) | ((unsigned long long)(16 * pnb) << 16) |
                     ((unsigned long long)(coff * esz) << 32);
    }
    for (int bi = lane; bi < NB(R - 1); bi += 64) {
        int a, b;
        block_ab(bi, a, b);
        blkRec[bi] = (uint32_t)(16 * bidx(a, b) | (16 * a) << 16 | (16 * b) << 24);
    }
}

// LDS tables of tier B (see build_tables) and its per-node pivot scalars
template <class S>
struct TierB {
    S *buf;                 // stored nodes (NodePlacement)
    const uint16_t *srcOff; // per view: offset of its stored node
    const uint8_t *srcNB;   // per view: blocks per granule array of that node
    const uint8_t *srcDet;  // per view: determinant slot (0xff: tier-A leaf)
    const unsigned long long *nodeRec;  // per include node, bytes: parent | its granule array stride << 16 | own << 32
    const uint32_t *blkRec;             // block index, bytes: 16 bidx(a, b) | 16 a << 16 | 16 b << 24
    RT<S> *nInv;            // per include node of a level: 1/alpha, 1/gamma1
    S *nBa;                 // per include node of a level: beta/alpha
    RT<S> *ndet;            // per include node: running determinant
};

// tier B, level J: every include node of level J from its parent of level J-1
template <class S, int R, int J>
__device__ __forceinline__ void tierB_level(const TierB<S> &tb, RT<S> leafDet, int lane, int &bad)
{
    constexpr int m = R - J;          // pivot mode of the parent (it has m+1 modes)
    constexpr int NN = 1 << (J - 1);  // include nodes at level J
    constexpr int NBO = NB(m);        // blocks of a child
    if (lane < NN) {
        const S *par = tb.buf + tb.srcOff[NN - 1 + lane];
        const int di = tb.srcDet[NN - 1 + lane];
        const RT<S> pdp = di == 0xff ? leafDet : tb.ndet[di];
        const Piv<S> pq = node_pivot(par, (int)tb.srcNB[NN - 1 + lane], m);
        tb.nInv[2 * lane] = pq.inv_a;
        tb.nInv[2 * lane + 1] = pq.inv_g;
        tb.nBa[lane] = pq.ba;
        tb.ndet[NN - 1 + lane] = rmul(pdp, pq.pdet);
        if (!is_pos(pq.pdet) || !is_pos(pq.inv_a))
            bad = 1;
    }
    __syncthreads();
    // granule g of the block at byte offset o of a node at byte offset p
    // with arrays st bytes apart: buf + p + g st + o
    char *const lb = reinterpret_cast<char *>(tb.buf);
    constexpr int GPB = 4 / EPG((int)sizeof(S));  // granules per block
    // 16-byte scalars: each node's blocks start on a 16-lane boundary (NS
    // lanes per node), so the 16 lanes one LDS cycle serves of a 128-bit
    // access never span two nodes, whose neighbouring 16-byte words would
    // meet in the same banks.  This costs no pass at the levels of the
    // complex and double-double kernels and halves their LDS bank-conflict
    // cycles; the 8-byte path keeps packed nodes (its passes hold two
    // granules per block, and the extra index registers cost it waves).
    constexpr bool AL = !std::is_same<S, double>::value;
    constexpr int NS = AL ? (NBO + 15) / 16 * 16 : NBO;  // lanes per node in a pass
    auto pass = [&](int it) {
        const int i = (int)((unsigned)it / NS), bi = it - i * NS;
        if (AL && bi >= NBO)
            return;
        const unsigned long long rec = tb.nodeRec[NN - 1 + i];
        const uint32_t br = tb.blkRec[bi];
        const int par = (int)(rec & 0xffffu), st = (int)((rec >> 16) & 0xffffu), cof = (int)(rec >> 32);
        const int a16 = (int)((br >> 16) & 0xffu), b16 = (int)(br >> 24), h16 = (int)(br & 0xffffu);
        Piv<S> pq;
        pq.inv_a = tb.nInv[2 * i];
        pq.inv_g = tb.nInv[2 * i + 1];
        pq.ba = tb.nBa[i];
        S A[4], Bk[4], H[4], o[4];
        const char *pa = lb + par + a16 + 16 * NB(m), *pb = lb + par + b16 + 16 * NB(m), *ph = lb + par + h16;
#pragma unroll
        for (int g = 0; g < GPB; ++g) {
            const Gran<S> qa = *reinterpret_cast<const Gran<S> *>(pa + g * st);
            const Gran<S> qb = *reinterpret_cast<const Gran<S> *>(pb + g * st);
            const Gran<S> qh = *reinterpret_cast<const Gran<S> *>(ph + g * st);
#pragma unroll
            for (int j = 0; j < EPG((int)sizeof(S)); ++j) {
                A[g * EPG((int)sizeof(S)) + j] = qa.e[j];
                Bk[g * EPG((int)sizeof(S)) + j] = qb.e[j];
                H[g * EPG((int)sizeof(S)) + j] = qh.e[j];
            }
        }
        elim_math(A, Bk, H, a16 == b16, pq, o);
        // the include child i of level J is view 2i+1 of that level
        char *pc = lb + cof + 16 * bi;
#pragma unroll
        for (int g = 0; g < GPB; ++g) {
            Gran<S> q;
#pragma unroll
            for (int j = 0; j < EPG((int)sizeof(S)); ++j)
                q.e[j] = o[g * EPG((int)sizeof(S)) + j];
            *reinterpret_cast<Gran<S> *>(pc + g * 16 * NBO) = q;
        }
    };
    constexpr int TOT = NN * NS, FULL = TOT / 64;
    // real path: an empty asm hides that the lane index is the same in every
    // leaf, so the passes' node and block indices are recomputed per leaf
    // instead of being held in registers across the whole leaf loop (10
    // registers less, which the one-wait tier-A step uses; the complex path
    // has them to spare)
    int ln = lane;
    if constexpr (std::is_same<S, double>::value)
        __asm__ volatile("" : "+v"(ln));
#pragma unroll 2
    for (int it0 = 0; it0 < 64 * FULL; it0 += 64)
        pass(it0 + ln);
    if constexpr (TOT % 64 != 0) {
        if (64 * FULL + ln < TOT)
            pass(64 * FULL + ln);
    }
    __syncthreads();
}

template <class S, int R, int J, int B>
__device__ __forceinline__ void tierB(const TierB<S> &tb, RT<S> leafDet, int lane, int &bad)
{
    if constexpr (J < B) {
        tierB_level<S, R, J>(tb, leafDet, lane, bad);
        tierB<S, R, J + 1, B>(tb, leafDet, lane, bad);
    }
}

// ---------------------------------------------------------------------------
// register-resident include step (packed lower triangle): h has M modes, hn
// receives M-1 modes
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

// all 2^M subsets below a register-resident node of M modes.  SG is the sign
// (-1)^(#excluded) of its subsets relative to the lane's frame (see the
// accumulators); det is the running determinant.
template <class S, int M, int SG, class Acc, int TB = 0>
__device__ __forceinline__ void tail(const S *h, RT<S> det, Acc &acc, int &bad)
{
    if constexpr (M == 0) {
        acc.template add<SG, TB>(rsqrt_nr(det));
    } else if constexpr (M == 1) {
        // exclude (sign -SG) and include (sign SG) of the last mode
        const RT<S> a = re(h[0]);
        const S b = h[1];
        const RT<S> g = re(h[2]);
        const RT<S> pd = det_last(a, b, g);  // det of the last 2x2 block
        acc.template add_pair<SG, TB>(rsqrt_nr(det), rsqrt_nr(rmul(det, pd)));
    } else {
        tail<S, M - 1, -SG, Acc, TB>(h, det, acc, bad);  // exclude the next mode
        constexpr int p = 2 * M - 2;
        const RT<S> a = re(h[pidx(p, p)]);
        const S b = h[pidx(p + 1, p)];
        const RT<S> g = re(h[pidx(p + 1, p + 1)]);
        const Piv<S> pq = pivot(a, b, g);
        S hn[E(M - 1)];
        elim_regs<S, M>(h, pq, hn);
        tail<S, M - 1, SG, Acc, TB | (1 << (M - 1))>(hn, rmul(det, pq.pdet), acc, bad);
    }
}

// The include chain of a register-resident node of M modes: its 2x2 pivots
// in turn, each tested (alpha > 0, alpha gamma1 > 0), down to the last mode.
// Run on the lane that holds the all-include subset, this completes the test
// of every pivot of the factorisation of I - O itself: positive definiteness
// of I - O is equivalent to all of them passing (the block form of
// Sylvester's criterion), and it implies it for every other subset.
template <class S, int M>
__device__ __forceinline__ void include_chain_test(const S *h, int &bad)
{
    if constexpr (M == 1) {
        const RT<S> a = re(h[0]);
        if (!is_pos(a) || !is_pos(det_last(a, h[1], re(h[2]))))
            bad = 1;
    } else if constexpr (M > 1) {
        constexpr int p = 2 * M - 2;
        const RT<S> a = re(h[pidx(p, p)]);
        const Piv<S> pq = pivot(a, h[pidx(p + 1, p)], re(h[pidx(p + 1, p + 1)]));
        if (!is_pos(a) || !is_pos(pq.pdet))
            bad = 1;
        S hn[E(M - 1)];
        elim_regs<S, M>(h, pq, hn);
        include_chain_test<S, M - 1>(hn, bad);
    }
}

// element (x, y), y <= x, of a node with nb blocks per granule array
template <class S>
__device__ __forceinline__ S node_el(const S *node, int nb, int x, int y)
{
    return blk(node, nb, bidx(x >> 1, y >> 1), ((x & 1) << 1) + (y & 1));
}

// pivot of one lane-level decision: an include lane takes the 2x2 pivot, an
// exclude lane a zero update (inverses and beta/alpha zero, determinant 1),
// which leaves the prefix exactly as it is, so that both kinds of lanes run
// the same instructions.
template <class S>
__device__ __forceinline__ Piv<S> lane_pivot(RT<S> a, S b, RT<S> g, bool inc, int &bad)
{
    Piv<S> pq = pivot(a, b, g);
    if (inc && (!is_pos(a) || !is_pos(pq.pdet)))
        bad = 1;
    if (!inc) {
        pq.inv_a = rconst<RT<S>>(0.0);
        pq.inv_g = rconst<RT<S>>(0.0);
        pq.ba = zero_of(b);
        pq.pdet = rconst<RT<S>>(1.0);
    }
    return pq;
}

// tier C: lane l finishes node l of level B.  Its ancestor of level B-L is an
// LDS node of T+L modes; the lane takes the last L decisions itself (bit
// L-1-j of l is the decision at level B-L+1+j) and then the last T modes.
// The L lane levels are fused into one pass over the LDS node: the pivot
// rows of every level are formed first, then each remaining entry is read
// once and receives the L rank-2 updates in turn, so only the pivot rows and
// the T-mode result are held in registers.
template <class S, int T, int B, int L, class Acc>
__device__ __forceinline__ void tierC(const TierB<S> &tb, RT<S> leafDet, int leafInc, int N, int lane, Acc &acc,
                                      int &bad, bool full_leaf)
{
    static_assert(L == 1 || L == 2, "one or two lane levels");
    constexpr int NP = (1 << (B - L)) - 1;  // table base of level B-L
    constexpr int pT = 2 * T;               // rows of the T-mode result
    constexpr int p1 = 2 * (T + L) - 2;     // pivot rows of the first lane level
    const int ip = lane >> L;
    const S *src = tb.buf + tb.srcOff[NP + ip];
    const int snb = tb.srcNB[NP + ip];
    const int di = tb.srcDet[NP + ip];
    RT<S> det = di == 0xff ? leafDet : tb.ndet[di];
    const bool inc1 = (lane >> (L - 1)) & 1;  // first lane level
    const bool inc0 = lane & 1;               // second (L == 2)

    // first level: pivot of mode T+L-1 and its rows, r2 in LDL form
    const Piv<S> q1 = lane_pivot(re(node_el(src, snb, p1, p1)), node_el(src, snb, p1 + 1, p1),
                                 re(node_el(src, snb, p1 + 1, p1 + 1)),
                                 inc1, bad);
    S r1[p1], r2[p1];
#pragma unroll
    for (int y = 0; y < p1; ++y) {
        r1[y] = node_el(src, snb, p1, y);
        r2[y] = sub_mul(node_el(src, snb, p1 + 1, y), r1[y], q1.ba);
    }
    det = rmul(det, q1.pdet);
    int includes = leafInc + __popc(ip) + inc1;

    // second level (L == 2): its pivot rows are rows pT, pT+1 of the first
    // child, formed here from the node and the first level's rows
    Piv<S> q2;
    S s1[pT], s2[pT];
    if constexpr (L == 2) {
        S c[2][pT + 2];
#pragma unroll
        for (int x = pT; x < pT + 2; ++x) {
            const S u1 = scale(r1[x], q1.inv_a), u2 = scale(r2[x], q1.inv_g);
#pragma unroll
            for (int y = 0; y <= x; ++y) {
                const S v = node_el(src, snb, x, y);
                c[x - pT][y] = (x == y) ? upd_diag(v, u1, r1[y], u2, r2[y]) : upd(v, u1, r1[y], u2, r2[y]);
            }
        }
        q2 = lane_pivot(re(c[0][pT]), c[1][pT], re(c[1][pT + 1]), inc0, bad);
#pragma unroll
        for (int y = 0; y < pT; ++y) {
            s1[y] = c[0][y];
            s2[y] = sub_mul(c[1][y], s1[y], q2.ba);
        }
        det = rmul(det, q2.pdet);
        includes += inc0;
    }

    // the T-mode result: every entry read once, updated level by level
    S hT[E(T)];
#pragma unroll
    for (int x = 0; x < pT; ++x) {
        const S u1 = scale(r1[x], q1.inv_a), u2 = scale(r2[x], q1.inv_g);
        S w1, w2;
        if constexpr (L == 2) {
            w1 = scale(s1[x], q2.inv_a);
            w2 = scale(s2[x], q2.inv_g);
        }
#pragma unroll
        for (int y = 0; y <= x; ++y) {
            const S v = node_el(src, snb, x, y);
            S o = (x == y) ? upd_diag(v, u1, r1[y], u2, r2[y]) : upd(v, u1, r1[y], u2, r2[y]);
            if constexpr (L == 2)
                o = (x == y) ? upd_diag(o, w1, s1[y], w2, s2[y]) : upd(o, w1, s1[y], w2, s2[y]);
            hT[pidx(x, y)] = o;
        }
    }
    const int excluded = (N - T) - includes;
    acc.set_frame((excluded & 1) ? -1.0 : 1.0);
    if (full_leaf)  // wave-uniform: the leaf that holds the all-include subset
        include_chain_test<S, T>(hT, bad);
    tail<S, T, 1, Acc>(hT, det, acc, bad);
}

// ---------------------------------------------------------------------------
template <class S, int T, int B, int L, class Acc>
__global__ void __launch_bounds__(64) tor_main(MainParams prm)
{
    constexpr int R = T + B;
    constexpr int BL = B - L;                // levels expanded in LDS
    constexpr int NN_MAX = 1 << (BL - 1);    // include nodes of the last LDS level
    // real path: node 0 holds the level-(LA-1) node (R+1 modes), whose
    // exclude view is the tier-A leaf and whose include child the next one
    constexpr int X0 = std::is_same<S, double>::value ? 1 : 0;
    constexpr int kBufScalars = NodePlacement<R, BL, (int)sizeof(S), L, X0>{}.off[1 << BL] / (int)sizeof(S);
    __shared__ S bufB[kBufScalars];
    __shared__ S nBa[NN_MAX];
    __shared__ RT<S> nInv[2 * NN_MAX];
    __shared__ RT<S> ndet[1 << BL];
    __shared__ uint16_t srcOff[(1 << (BL + 1)) - 1];
    __shared__ uint8_t srcNB[(1 << (BL + 1)) - 1];
    __shared__ uint8_t srcDet[(1 << (BL + 1)) - 1];
    __shared__ uint32_t blkRec[NB(R - 1)];
    __shared__ unsigned long long nodeRec[(1 << BL) - 1];

    const int lane = threadIdx.x;
    build_tables<S, R, BL + 1, L>(srcOff, srcNB, srcDet, nodeRec, blkRec, lane);
    __syncthreads();
    const TierB<S> tb{bufB, srcOff, srcNB, srcDet, nodeRec, blkRec, nInv, nBa, ndet};
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
        const long long root = P.root_begin + ((long long)item - P.item_begin);
        const int N = P.N, k = P.k, LA = N - R, D = LA - k;
        const S *C = reinterpret_cast<const S *>(P.C);
        // the wave's stack (tslot_off): the root node, tier-A slots k+1 ..
        // LA-1, and the running determinants of the tier-A levels on the
        // current path (used only when the root has more than one leaf)
        RT<S> *sdet = reinterpret_cast<RT<S> *>(wscr + tslot_off(N, k, LA));
        int bad = 0;

        // root: decisions on modes 0..k-1 given by the bits of root.  When
        // the node at the first included level fits the LDS buffer (free
        // until the first leaf), it is copied there, every include
        // eliminates in place in LDS, and only the final root node (N-k
        // modes, stride NB(N-k)) is written to the wave's stack.  Otherwise
        // the first include reads the matrix and the later ones rewrite the
        // root node in place in the stack with the matrix's stride NB(N).
        const S *rsrc = C;
        int rnb = NB(N);
        RT<S> rdet = rconst<RT<S>>(1.0);
        int rinc = 0;
        const unsigned long long rbits = (unsigned long long)root & ((1ull << k) - 1);
        const int l0 = rbits ? __builtin_ctzll(rbits) : k;  // first included level
        if (rbits && NSZ(N - l0) <= kBufScalars) {
            const int nb0 = NB(N - l0);
            copy_node<S, true, false>(C, NB(N), bufB, nb0, N - l0, lane);
            __syncthreads();
            for (int l = l0; l < k; ++l) {
                if ((rbits >> l) & 1) {
                    RT<S> pd;
                    elim_lds<S>(bufB, nb0, N - l, lane, pd, bad);
                    rdet = rmul(rdet, pd);
                    ++rinc;
                }
            }
            copy_node<S, false, true>(bufB, nb0, wscr, NB(N - k), N - k, lane);
            __syncthreads();
            rsrc = wscr;
            rnb = NB(N - k);
        } else {
            for (int l = 0; l < k; ++l) {
                if ((rbits >> l) & 1) {
                    RT<S> pd;
                    elim_inplace<S>(rsrc, rnb, wscr, rnb, N - l, lane, pd, bad);
                    rdet = rmul(rdet, pd);
                    ++rinc;
                    rsrc = wscr;
                }
            }
        }

        Acc acc;
        const long long nleaf = 1ll << D;
        for (long long x = 0; x < nleaf; ++x) {
            // double-double factor: an empty asm hides that the lane index
            // is the same in every leaf, so what the tiers derive from it
            // (block and node indices, table entries) is recomputed in each
            // leaf instead of being held in registers across the whole loop.
            // That brings the kernel to 256 registers, two waves per SIMD
            // (the real FP64 kernel does the same for tier B only).
            int lane = threadIdx.x;
            if constexpr (std::is_same<S, ddr>::value)
                __asm__ volatile("" : "+v"(lane));
            RT<S> ldet;
            int linc;
            if (x == 0) {
                if constexpr (X0) {
                    // the first R+1 modes of the root node (R when the root
                    // is the leaf), restrided to NB(R + 1)
                    copy_node<S, true, false>(rsrc, rnb, bufB, NB(R + 1), min(R + 1, N - k), lane);
                } else {
                    // the first R modes of the root node, restrided to NB(R)
                    constexpr int GA = EPG((int)sizeof(S)) * NB(R);  // scalars per granule array
                    for (int e = lane; e < NSZ(R); e += 64) {
                        const int g = e / GA;
                        bufB[e] = ld_g(&rsrc[g * EPG((int)sizeof(S)) * rnb + (e - g * GA)]);
                    }
                }
                ldet = rdet;
                linc = rinc;
            } else {
                // leaf x differs from leaf x-1 from level lvl on: lvl becomes an
                // include, every deeper tier-A level an exclude
                const int t = __builtin_ctzll(x);
                const int lvl = LA - 1 - t;
                const long long xr = x >> (t + 1);
                const S *s;
                int snb;
                RT<S> sd;
                int si;
                if (xr == 0) {
                    s = rsrc;
                    snb = rnb;
                    sd = rdet;
                    si = rinc;
                } else {
                    const int sl = LA - (__builtin_ctzll(xr) + t + 1);
                    s = wscr + tslot_off(N, k, sl);
                    snb = NB(N - sl);
                    sd = sdet[sl];
                    // includes on the path down to level sl: the root's and
                    // the tier-A decisions above sl, bits LA-1-l of x
                    si = rinc + __popcll((unsigned long long)x >> (LA - sl));
                }
                RT<S> pd;
                if (X0 && t == 0) {
                    // the include at level LA-1: its source, the level-(LA-1)
                    // node of this path, is LDS node 0, updated in place
                    elim_lds<S>(bufB, NB(R + 1), R + 1, lane, pd, bad);
                } else {
                    // the deepest slot a later step reads (level LA, or LA-1
                    // when node 0 holds that level) gets the child in LDS
                    // only; shallower ones also go to their stack slot
                    S *dst = (lvl + 1 < LA - X0) ? wscr + tslot_off(N, k, lvl + 1) : nullptr;
                    elim_global<S>(s, snb, dst, NB(N - lvl - 1), bufB, NB(R + X0), N - lvl, lane, pd, bad);
                }
                ldet = rmul(sd, pd);
                linc = si + 1;
                if (lane == 0)
                    sdet[lvl + 1] = ldet;
            }
            __syncthreads();
            if constexpr (std::is_same<Acc, AccStore>::value) {
                // subset index of the lane's first term: bit N-1-l is the
                // decision at level l, so the root's k bits reversed on top,
                // then the leaf index x (tier A, level LA-1 lowest), then the
                // lane (tier B's view bits and tier C's two lane levels), then
                // the T bits of the tail
                const unsigned long long rrev = k ? __builtin_bitreverse64((unsigned long long)root) >> (64 - k) : 0ull;
                acc.begin_leaf(prm.terms + ((rrev << (N - k)) | ((unsigned long long)x << R) | ((unsigned long long)lane << T)));
            }
            tierB<S, R, 1, BL + 1>(tb, ldet, lane, bad);
            tierC<S, T, B, L, Acc>(tb, ldet, linc, N, lane, acc, bad, root == (1ll << k) - 1 && x == nleaf - 1);
            __syncthreads();
        }

        double h = acc.hi * acc.frame, l = acc.lo * acc.frame, ab = acc.abs_sum;
        constexpr bool is_dd = Acc::kDD;
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
            // slots are overwritten, never accumulated, so running a root
            // again (the host's recovery from a numeric failure) is idempotent
            const bool forced = (long long)item + 1 == prm.fail_item1;
            double *sl = P.slots + 4 * root;
            sl[0] = forced ? __builtin_nan("") : h;
            sl[1] = l;
            sl[2] = ab;
            sl[3] = anybad ? SLOT_NOT_PD : (forced || !__builtin_isfinite(h)) ? SLOT_NUMERIC : 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// per-matrix sum of the root slots: thread t takes roots t, t + RED_THREADS,
// ... in index order, then the threads are combined by a fixed tree (within
// each wave, then across the waves), so the result does not depend on timing.
constexpr int RED_THREADS = 1024;

template <bool DD>
__device__ inline void red_step(double &h, double &l, double &ab, double &bad, int off)
{
    const double oh = __shfl_xor(h, off), ol = __shfl_xor(l, off);
    if (DD)
        dd_add2(h, l, oh, ol);
    else
        h += oh;
    ab += __shfl_xor(ab, off);
    bad = fmax(bad, __shfl_xor(bad, off));
}

template <bool DD>
__global__ void __launch_bounds__(RED_THREADS) tor_reduce(const ProblemDesc *probs, double *results)
{
    constexpr int NW = RED_THREADS / 64;
    __shared__ double part[4][NW];
    const int q = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
    const ProblemDesc P = probs[q];
    const long long nroots = 1ll << P.k;
    double h = 0.0, l = 0.0, ab = 0.0, bad = 0.0;
    for (long long r = t; r < nroots; r += RED_THREADS) {
        const double *s = P.slots + 4 * r;
        if (DD)
            dd_add2(h, l, s[0], s[1]);
        else
            h += s[0];
        ab += s[2];
        bad = fmax(bad, s[3]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        red_step<DD>(h, l, ab, bad, off);
    if (lane == 0) {
        part[0][w] = h;
        part[1][w] = l;
        part[2][w] = ab;
        part[3][w] = bad;
    }
    __syncthreads();
    if (w == 0) {
        const bool in = lane < NW;
        h = in ? part[0][lane] : 0.0;
        l = in ? part[1][lane] : 0.0;
        ab = in ? part[2][lane] : 0.0;
        bad = in ? part[3][lane] : 0.0;
#pragma unroll
        for (int off = NW / 2; off >= 1; off >>= 1)
            red_step<DD>(h, l, ab, bad, off);
        if (lane == 0) {
            results[4 * q + 0] = h;
            results[4 * q + 1] = l;
            results[4 * q + 2] = ab;
            results[4 * q + 3] = bad;
        }
    }
}

#ifndef TOR_KERNELS_TEMPLATES_ONLY
// Everything below is built once, in this translation unit; the
// double-double factor's kernel is instantiated and launched from
// tor_kernels_quad.hip, which includes the templates above on their own.
__global__ void tor_zero(unsigned long long *p, int count)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        p[i] = 0ull;
}

// ---------------------------------------------------------------------------
hipError_t launch_main_store(const MainParams &p, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((tor_main<double, REAL_T, REAL_B, REAL_L, AccStore>), dim3(grid), dim3(64), 0, s, p);
    return hipGetLastError();
}

int main_store_occupancy()
{
    int n = 0;
    const hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, tor_main<double, REAL_T, REAL_B, REAL_L, AccStore>, 64, 0);
    return e == hipSuccess ? n : 0;
}

hipError_t launch_main(int path, bool dd, const MainParams &p, int grid, hipStream_t s)
{
    if (path == PATH_QUAD) {
        return launch_main_quad(p, grid, s);
    } else if (path == PATH_REAL) {
        if (dd)
            hipLaunchKernelGGL((tor_main<double, REAL_T, REAL_B, REAL_L, AccDD>), dim3(grid), dim3(64), 0, s, p);
        else
            hipLaunchKernelGGL((tor_main<double, REAL_T, REAL_B, REAL_L, AccF64>), dim3(grid), dim3(64), 0, s, p);
    } else {
        if (dd)
            hipLaunchKernelGGL((tor_main<c64, CPLX_T, CPLX_B, CPLX_L, AccDD>), dim3(grid), dim3(64), 0, s, p);
        else
            hipLaunchKernelGGL((tor_main<c64, CPLX_T, CPLX_B, CPLX_L, AccF64>), dim3(grid), dim3(64), 0, s, p);
    }
    return hipGetLastError();
}

int main_occupancy(int path)
{
    int n = 0;
    hipError_t e;
    if (path == PATH_QUAD)
        return main_occupancy_quad();
    if (path == PATH_REAL)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, tor_main<double, REAL_T, REAL_B, REAL_L, AccDD>, 64, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, tor_main<c64, CPLX_T, CPLX_B, CPLX_L, AccDD>, 64, 0);
    return e == hipSuccess ? n : 0;
}

hipError_t launch_reduce(const ProblemDesc *probs, int nprob, double *results, bool dd, hipStream_t s)
{
    if (dd)
        hipLaunchKernelGGL((tor_reduce<true>), dim3(nprob), dim3(RED_THREADS), 0, s, probs, results);
    else
        hipLaunchKernelGGL((tor_reduce<false>), dim3(nprob), dim3(RED_THREADS), 0, s, probs, results);
    return hipGetLastError();
}

hipError_t launch_zero(unsigned long long *p, int count, hipStream_t s)
{
    hipLaunchKernelGGL(tor_zero, dim3((count + 63) / 64), dim3(64), 0, s, p, count);
    return hipGetLastError();
}
#endif  // TOR_KERNELS_TEMPLATES_ONLY

}  // namespace tor
