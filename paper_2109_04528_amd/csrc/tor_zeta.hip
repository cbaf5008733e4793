// tor_zeta.hip -- click probabilities of every pattern of one state at once.
//
// The probability that threshold detectors click exactly on the modes S of a
// Gaussian state is p(S) = Tor(O_S) sqrt(det(I - O)) (Sec. 1), and Tor(O_S)
// is Eq. 2 for the principal submatrix O_S: a signed sum of
// 1/sqrt(det (I - O)_Z) over the subsets Z of S.  Every pattern therefore
// draws its terms from the same 2^M subset determinants of I - O.  One launch
// of the recursive kernel over the whole state stores each signed term
//     t[Z] = (-1)^(N-|Z|) / sqrt(det (I - O)_Z)
// (N the modes of the staged form, index bit N-1-l = the decision at level l,
// which is mode l), so every prefix factor of the state is formed once for all
// patterns.  The subset sums
//     g[S] = sum over Z subset of S of t[Z]
// (the zeta transform over the subset lattice) then give every pattern at
// once: Tor(O_S) = (-1)^(N-|S|) g[S].  That is 2^M determinants and M passes
// of additions over 2^M entries, against 3^M determinants for the patterns
// one by one.
//
// The transform adds along one index bit at a time (g[S] += g[S without bit b]
// for every S with bit b set).  The low 10 to 12 bits run in one workgroup per
// block of 1024 to 4096 entries, its threads adding along a few bits in
// registers and exchanging the block through LDS between those rounds; the
// higher bits in global passes of up to ZG = 5 bits, each thread holding the
// 32 entries that differ only in those bits.  Every pass reads and writes
// all 2^M sums once, so the launch takes as few passes as 12 bits in the
// first stage allow, with the smallest block that reaches that count: a
// 4096-entry block (64 KB of LDS) leaves room for two workgroups per CU and
// keeps fewer loads in flight than a 1024-entry one (16 KB).  At M = 32 that
// is 12 bits first and four 5-bit passes, against 10 bits and six passes of
// 4 bits (226 ms to 172 ms for all 2^32 patterns); at M = 24 and 28, 10 bits
// first.
//
// Exactness: for a Gaussian state every subset determinant is at most 1
// (sqrt(det(I - O)) / sqrt(det (I - O)_Z) is the probability that no mode
// outside Z clicks, at least the probability sqrt(det(I - O)) that none
// does), so every term is a double of magnitude at least 1, a multiple of
// 2^-52, and the additions are double-double sums built from Knuth's TwoSum
// alone.  While a partial sum stays below 2^53 in magnitude,
// every intermediate quantity is a multiple of 2^-52 that fits its double, so
// every g[S] is the exact sum of its terms, whatever the order.
#include "tor_internal.hpp"

namespace tor {

namespace {

constexpr int ZB_MAX = 12;  // most index bits transformed in LDS (blocks of 4096 entries)
constexpr int ZG = 5;       // index bits per global pass
// whole 12- and 10-bit blocks: threads and register bits of tor_zeta_lds_r
// (threads 0: the bit-by-bit LDS kernel).  At M = 32, 256 threads of 16
// entries gave 159.8 ms per call, 512 of 8 161.0, 1024 of 4 164.8, the
// bit-by-bit kernel 167.5-168.8 (M = 24: 0.56 against 0.58 ms).
#ifndef ZR12_T
#define ZR12_T 256
#define ZR12_RB 4
#endif
#ifndef ZR10_T
#define ZR10_T 256
#define ZR10_RB 2
#endif

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// a + b in double-double from error-free sums only (see the file comment)
__device__ __forceinline__ void dd_acc(double &ah, double &al, double bh, double bl)
{
    double s, e, t, f;
    two_sum(ah, bh, s, e);
    two_sum(al, bl, t, f);
    e += t;
    two_sum(s, e, s, e);
    e += f;
    two_sum(s, e, ah, al);
}

// bits 0 .. nb-1 of a block of 2^nb entries (nb <= ZB), terms in,
// double-double out; ZT threads
template <int ZB, int ZT>
__global__ void __launch_bounds__(ZT) tor_zeta_lds(const double *t, ddr *g, int nb)
{
    __shared__ double hs[1 << ZB], ls[1 << ZB];
    const int size = 1 << nb;
    const long long base = (long long)blockIdx.x << nb;
    for (int i = threadIdx.x; i < size; i += ZT) {
        hs[i] = t[base + i];
        ls[i] = 0.0;
    }
    __syncthreads();
    for (int b = 0; b < nb; ++b) {
        const int low = (1 << b) - 1;
        for (int p = threadIdx.x; p < size / 2; p += ZT) {
            const int i1 = ((p & ~low) << 1) | (1 << b) | (p & low);  // the p-th index with bit b set
            const int i0 = i1 ^ (1 << b);
            double h = hs[i1], l = ls[i1];
            dd_acc(h, l, hs[i0], ls[i0]);
            hs[i1] = h;
            ls[i1] = l;
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < size; i += ZT)
        g[base + i] = ddr{hs[i], ls[i]};
}

// All ZB bits of a block of 2^ZB entries, with the additions in registers:
// each of the ZT threads holds E = 2^RB entries that differ only in RB index
// bits and adds along those bits; between rounds (bits from the highest down)
// the block moves through LDS so that each thread holds the entries of the
// next RB bits.  Per entry that is 4 doubles of LDS traffic per round and
// two barriers, against 3 doubles and one barrier per bit.  The LDS index is
// XOR-swizzled within each run of 16 entries, i ^ ((i >> RB) & 15), which
// leaves no two of the 16 lanes that one cycle of a 64-bit access serves on
// the same bank in any round or in the final copy.  The first round reads
// the terms straight from global memory (consecutive lanes, consecutive
// entries); the last one goes out through LDS so that the double-double
// sums are written in consecutive runs.  Terms in, double-double out.
template <int ZB, int ZT, int RB>
__global__ void __launch_bounds__(ZT) tor_zeta_lds_r(const double *t, ddr *g)
{
    static_assert((ZT << RB) == (1 << ZB) && ZB % RB == 0, "a block is ZT threads of 2^RB entries");
    constexpr int E = 1 << RB;
    __shared__ double hs[1 << ZB], ls[1 << ZB];
    const long long base = (long long)blockIdx.x << ZB;
    const int q = threadIdx.x;
    auto sw = [](int i) { return i ^ ((i >> RB) & 15); };
    // entry j of thread q in the round of bits s .. s+RB-1
    auto idx = [&](int s, int j) { return (q & ((1 << s) - 1)) | (j << s) | ((q >> s) << (s + RB)); };
    double h[E], l[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        h[j] = t[base + idx(ZB - RB, j)];
        l[j] = 0.0;
    }
#pragma unroll
    for (int s = ZB - RB; s >= 0; s -= RB) {
#pragma unroll
        for (int b = 0; b < RB; ++b)
#pragma unroll
            for (int j = 0; j < E; ++j)
                if ((j >> b) & 1)
                    dd_acc(h[j], l[j], h[j ^ (1 << b)], l[j ^ (1 << b)]);
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int i = sw(idx(s, j));
            hs[i] = h[j];
            ls[i] = l[j];
        }
        __syncthreads();
        if (s == 0)
            break;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int i = sw(idx(s - RB, j));
            h[j] = hs[i];
            l[j] = ls[i];
        }
        __syncthreads();  // every entry is read before the next round writes
    }
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const int i = q + k * ZT;
        g[base + i] = ddr{hs[sw(i)], ls[sw(i)]};
    }
}

// bits b0 .. b0+nb-1 (nb <= ZG) over all 2^nbits entries: thread q holds the
// 2^nb entries whose index has q's bits below b0 and above b0+nb-1
// NT: streaming (non-temporal) loads and stores, for sums too large to stay
// in the caches between passes
template <bool NT>
__global__ void __launch_bounds__(256) tor_zeta_bits(ddr *g, int nbits, int b0, int nb)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (1ll << (nbits - nb)))
        return;
    const long long lowm = (1ll << b0) - 1;
    const long long base = (q & lowm) | ((q & ~lowm) << nb);
    double h[1 << ZG], l[1 << ZG];
#pragma unroll
    for (int j = 0; j < (1 << ZG); ++j)
        if (j < (1 << nb)) {
            const double *pv = reinterpret_cast<const double *>(g + base + ((long long)j << b0));
            if constexpr (NT) {
                h[j] = __builtin_nontemporal_load(pv);
                l[j] = __builtin_nontemporal_load(pv + 1);
            } else {
                h[j] = pv[0];
                l[j] = pv[1];
            }
        }
#pragma unroll
    for (int b = 0; b < ZG; ++b)
        if (b < nb) {
#pragma unroll
            for (int j = 0; j < (1 << ZG); ++j)
                if (j < (1 << nb) && ((j >> b) & 1))
                    dd_acc(h[j], l[j], h[j ^ (1 << b)], l[j ^ (1 << b)]);
        }
#pragma unroll
    for (int j = 0; j < (1 << ZG); ++j)
        if (j < (1 << nb)) {
            if constexpr (NT) {
                double *pv = reinterpret_cast<double *>(g + base + ((long long)j << b0));
                __builtin_nontemporal_store(h[j], pv);
                __builtin_nontemporal_store(l[j], pv + 1);
            } else {
                g[base + ((long long)j << b0)] = ddr{h[j], l[j]};
            }
        }
}

// one pattern's outputs from its subset sum v
__device__ __forceinline__ void put_pattern(long long S, int N, ddr v, double sq, double *probs, double *tor_hi,
                                            double *tor_lo)
{
    const double sg = ((N - __popcll((unsigned long long)S)) & 1) ? -1.0 : 1.0;
    if (tor_hi)
        tor_hi[S] = sg * v.hi;
    if (tor_lo)
        tor_lo[S] = sg * v.lo;
    if (probs)
        probs[S] = sg * (v.hi + v.lo) * sq;
}

// Pattern S's sum sits at index bitreverse_N(S) (S's bit i is mode i, the
// decision at level i, index bit N-1-i).  Without padding modes (M = N) the
// permutation runs in tiles: a workgroup fixes the middle N-2A index bits,
// reads the 2^A x 2^A entries of its top and bottom A bits in runs of 2^A
// neighbours, and writes them out again in runs of 2^A neighbours of S
// through LDS (the top A bits of S are the bottom A bits of the index
// reversed, and the other way round).
constexpr int TA = 5;
__global__ void __launch_bounds__(256) tor_click_out_tiled(const ddr *g, int N, const double *sqrt_det, double *probs,
                                                            double *tor_hi, double *tor_lo)
{
    __shared__ double th[1 << TA][(1 << TA) + 1], tl[1 << TA][(1 << TA) + 1];
    const long long mid = blockIdx.x;
    const int nm = N - 2 * TA;
    for (int q = threadIdx.x; q < (1 << (2 * TA)); q += 256) {
        const int h = q >> TA, l = q & ((1 << TA) - 1);
        const ddr v = g[((long long)h << (N - TA)) | (mid << TA) | l];
        th[h][l] = v.hi;
        tl[h][l] = v.lo;
    }
    __syncthreads();
    const long long rmid = nm > 0 ? (long long)(__builtin_bitreverse64((unsigned long long)mid) >> (64 - nm)) : 0;
    const double sq = sqrt_det[0];
    for (int q = threadIdx.x; q < (1 << (2 * TA)); q += 256) {
        const int rl = q >> TA, rh = q & ((1 << TA) - 1);
        const int h = (int)(__builtin_bitreverse32((unsigned)rh) >> (32 - TA));
        const int l = (int)(__builtin_bitreverse32((unsigned)rl) >> (32 - TA));
        const long long S = ((long long)rl << (N - TA)) | (rmid << TA) | rh;
        put_pattern(S, N, ddr{th[h][l], tl[h][l]}, sq, probs, tor_hi, tor_lo);
    }
}

// one thread per pattern S < 2^M (any M <= N): a gather, for the padded forms
__global__ void __launch_bounds__(256) tor_click_out(const ddr *g, int N, int M, const double *sqrt_det,
                                                      double *probs, double *tor_hi, double *tor_lo)
{
    const long long S = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (S >= (1ll << M))
        return;
    const unsigned long long idx = __builtin_bitreverse64((unsigned long long)S) >> (64 - N);
    put_pattern(S, N, g[idx], sqrt_det[0], probs, tor_hi, tor_lo);
}

}  // namespace

hipError_t launch_zeta(const double *t, ddr *g, int nbits, hipStream_t s)
{
    // global passes after zb bits in LDS
    auto passes = [&](int zb) { return nbits > zb ? (nbits - zb + ZG - 1) / ZG : 0; };
    const int zb = passes(10) == passes(ZB_MAX) ? 10 : passes(11) == passes(ZB_MAX) ? 11 : ZB_MAX;
    const int nb = nbits < zb ? nbits : zb;
    const dim3 grid((unsigned)(1ll << (nbits - nb)));
    bool done = false;
#if ZR12_T > 0
    if (nb == 12) {
        hipLaunchKernelGGL((tor_zeta_lds_r<12, ZR12_T, ZR12_RB>), grid, dim3(ZR12_T), 0, s, t, g);
        done = true;
    }
#endif
#if ZR10_T > 0
    if (nb == 10) {
        hipLaunchKernelGGL((tor_zeta_lds_r<10, ZR10_T, ZR10_RB>), grid, dim3(ZR10_T), 0, s, t, g);
        done = true;
    }
#endif
    if (done)
        ;
    else if (zb == 10)
        hipLaunchKernelGGL((tor_zeta_lds<10, 256>), grid, dim3(256), 0, s, t, g, nb);
    else if (zb == 11)
        hipLaunchKernelGGL((tor_zeta_lds<11, 512>), grid, dim3(512), 0, s, t, g, nb);
    else
        hipLaunchKernelGGL((tor_zeta_lds<12, 1024>), grid, dim3(1024), 0, s, t, g, nb);
    hipError_t e = hipGetLastError();
    for (int b0 = nb; e == hipSuccess && b0 < nbits; b0 += ZG) {
        const int w = nbits - b0 < ZG ? nbits - b0 : ZG;
        const long long threads = 1ll << (nbits - w);
        // streaming accesses once the sums (16 B each) pass 1 GiB: at M = 28
        // and 32 they took the call from 10.6 to 10.3 ms and from 159.6 to
        // 156.0 ms, at M = 24 (268 MB, mostly held by the caches) from 0.56 to
        // 0.59 ms the other way
        if (nbits >= 26)
            hipLaunchKernelGGL((tor_zeta_bits<true>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, g,
                               nbits, b0, w);
        else
            hipLaunchKernelGGL((tor_zeta_bits<false>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, g,
                               nbits, b0, w);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_click_out(const ddr *g, int N, int M, const double *sqrt_det, double *probs, double *tor_hi,
                            double *tor_lo, hipStream_t s)
{
    if (M == N && N >= 2 * TA) {
        hipLaunchKernelGGL(tor_click_out_tiled, dim3((unsigned)(1ll << (N - 2 * TA))), dim3(256), 0, s, g, N, sqrt_det,
                           probs, tor_hi, tor_lo);
        return hipGetLastError();
    }
    const long long n = 1ll << M;
    hipLaunchKernelGGL(tor_click_out, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, N, M, sqrt_det, probs,
                       tor_hi, tor_lo);
    return hipGetLastError();
}

}  // namespace tor
