// tor_device.hpp -- device-side arithmetic for the recursive Torontonian.
//
// Packed layout used everywhere on the device
// -------------------------------------------
// A node of the include/exclude tree carries the Schur complement H of the
// modes it has included, restricted to the modes [a, N) it has not decided
// yet.  Rows are mode-interleaved (a_i, a_i^dag) and then REVERSED, so that the
// next mode to decide owns the two highest rows.  The lower triangle of the
// reversed matrix is stored row by row: entry (x, y), y <= x, sits at
// x(x+1)/2 + y.  Dropping the next mode (an "exclude" child) is then a prefix
// of the same array, so exclude children cost nothing; an "include" child is
// the rank-2 update that removes the two highest rows (a 2x2 pivot block).
//
// The include child is the two-row append of Sec. 2 in right-looking form:
// with the 2x2 pivot block P = [[alpha, conj(beta)], [beta, gamma]] and its
// Cholesky/LDL factor, the new rows of L for every later mode are
// H[x][P] P^{-1/2}, and the determinant grows by det P = alpha * gamma1,
// gamma1 = gamma - |beta|^2 / alpha, the product of the two new squared
// diagonal entries of L (det = prod |L_ii|^2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tor_internal.hpp"

namespace tor {

// ---- scalar helpers, overloaded for the real (double) and complex (c64) paths
__device__ __forceinline__ double re(double a) { return a; }
__device__ __forceinline__ double re(c64 a) { return a.x; }
__device__ __forceinline__ double abs2(double a) { return a * a; }
__device__ __forceinline__ double abs2(c64 a) { return fma(a.x, a.x, a.y * a.y); }
__device__ __forceinline__ double scale(double a, double s) { return a * s; }
__device__ __forceinline__ c64 scale(c64 a, double s) { return c64{a.x * s, a.y * s}; }
__device__ __forceinline__ double zero_of(double) { return 0.0; }
__device__ __forceinline__ c64 zero_of(c64) { return c64{0.0, 0.0}; }
// a - b*c  (plain product, no conjugate)
__device__ __forceinline__ double sub_mul(double a, double b, double c) { return fma(-b, c, a); }
__device__ __forceinline__ c64 sub_mul(c64 a, c64 b, c64 c)
{
    return c64{fma(b.y, c.y, fma(-b.x, c.x, a.x)), fma(-b.y, c.x, fma(-b.x, c.y, a.y))};
}
__device__ __forceinline__ double conj_of(double a) { return a; }
__device__ __forceinline__ c64 conj_of(c64 a) { return c64{a.x, -a.y}; }
__device__ __forceinline__ double fix_diag(double a) { return a; }
__device__ __forceinline__ c64 fix_diag(c64 a) { return c64{a.x, 0.0}; }
// h - conj(u1) r1 - conj(u2) r2   (one entry of the rank-2 update)
__device__ __forceinline__ double upd(double h, double u1, double r1, double u2, double r2)
{
    return fma(-u2, r2, fma(-u1, r1, h));
}
__device__ __forceinline__ c64 upd(c64 h, c64 u1, c64 r1, c64 u2, c64 r2)
{
    double xr = fma(-u1.x, r1.x, h.x);
    xr = fma(-u1.y, r1.y, xr);
    xr = fma(-u2.x, r2.x, xr);
    xr = fma(-u2.y, r2.y, xr);
    double xi = fma(-u1.x, r1.y, h.y);
    xi = fma(u1.y, r1.x, xi);
    xi = fma(-u2.x, r2.y, xi);
    xi = fma(u2.y, r2.x, xi);
    return c64{xr, xi};
}
// diagonal entries are real: the imaginary part is dropped exactly
__device__ __forceinline__ double upd_diag(double h, double u1, double r1, double u2, double r2)
{
    return fma(-u2, r2, fma(-u1, r1, h));
}
__device__ __forceinline__ c64 upd_diag(c64 h, c64 u1, c64 r1, c64 u2, c64 r2)
{
    double xr = fma(-u1.x, r1.x, h.x);
    xr = fma(-u1.y, r1.y, xr);
    xr = fma(-u2.x, r2.x, xr);
    xr = fma(-u2.y, r2.y, xr);
    return c64{xr, 0.0};
}

// ---- double-double arithmetic (the factor of the higher-precision mode) -----
// Error-free transformations: Knuth's TwoSum, Dekker's Fast2Sum, and the
// exact product by FMA; the double-double operations built from them follow
// Dekker (1971) and Hida, Li and Bailey's double-double library: results are
// renormalised so that |lo| <= ulp(hi) / 2, with relative errors of a few
// units of 2^-104 (the "sloppy" addition: absolute error a few 2^-104 times
// |a| + |b|, which is the error model the Cholesky backward-error analysis
// needs).  Contraction of a product and a sum into one FMA is switched off
// inside these routines: it would round the product away from the value its
// separately computed rounding error belongs to, and the transformation
// would no longer be exact.
__device__ __forceinline__ ddr fast2sum(double a, double b)
{
#pragma clang fp contract(off)
    const double s = a + b;
    return ddr{s, b - (s - a)};
}
__device__ __forceinline__ ddr dd_add(ddr a, ddr b)
{
#pragma clang fp contract(off)
    const double s = a.hi + b.hi;
    const double bb = s - a.hi;
    double e = (a.hi - (s - bb)) + (b.hi - bb);
    e += a.lo + b.lo;
    return fast2sum(s, e);
}
__device__ __forceinline__ ddr dd_neg(ddr a) { return ddr{-a.hi, -a.lo}; }
__device__ __forceinline__ ddr dd_mul(ddr a, ddr b)
{
#pragma clang fp contract(off)
    const double p = a.hi * b.hi;
    double e = fma(a.hi, b.hi, -p);
    e = fma(a.hi, b.lo, e);
    e = fma(a.lo, b.hi, e);
    return fast2sum(p, e);
}
// h - u1 r1 - u2 r2 with one renormalisation: the two leading products and
// their sum with h.hi are error-free, every lower-order part is summed in
// double
__device__ __forceinline__ ddr dd_upd(ddr h, ddr u1, ddr r1, ddr u2, ddr r2)
{
#pragma clang fp contract(off)
    const double p1 = u1.hi * r1.hi, p2 = u2.hi * r2.hi;
    const double e1 = fma(u1.hi, r1.hi, -p1), e2 = fma(u2.hi, r2.hi, -p2);
    double s = h.hi - p1;
    double bb = s - h.hi;
    double t = (h.hi - (s - bb)) + (-p1 - bb);
    const double s2 = s - p2;
    bb = s2 - s;
    t += (s - (s2 - bb)) + (-p2 - bb);
    double lo = h.lo - e1 - e2;
    lo = fma(-u1.hi, r1.lo, lo);
    lo = fma(-u1.lo, r1.hi, lo);
    lo = fma(-u2.hi, r2.lo, lo);
    lo = fma(-u2.lo, r2.hi, lo);
    return fast2sum(s2, t + lo);
}

__device__ __forceinline__ ddr re(ddr a) { return a; }
__device__ __forceinline__ ddr abs2(ddr a) { return dd_mul(a, a); }
__device__ __forceinline__ ddr scale(ddr a, ddr s) { return dd_mul(a, s); }
__device__ __forceinline__ ddr zero_of(ddr) { return ddr{0.0, 0.0}; }
__device__ __forceinline__ ddr sub_mul(ddr a, ddr b, ddr c) { return dd_add(a, dd_neg(dd_mul(b, c))); }
__device__ __forceinline__ ddr conj_of(ddr a) { return a; }
__device__ __forceinline__ ddr fix_diag(ddr a) { return a; }
__device__ __forceinline__ ddr upd(ddr h, ddr u1, ddr r1, ddr u2, ddr r2) { return dd_upd(h, u1, r1, u2, r2); }
__device__ __forceinline__ ddr upd_diag(ddr h, ddr u1, ddr r1, ddr u2, ddr r2) { return dd_upd(h, u1, r1, u2, r2); }

// real type of a scalar: double for double and c64, ddr for ddr
template <class S>
struct RealOf {
    using type = double;
};
template <>
struct RealOf<ddr> {
    using type = ddr;
};
template <class S>
using RT = typename RealOf<S>::type;

template <class R>
__device__ __forceinline__ R rconst(double x);
template <>
__device__ __forceinline__ double rconst<double>(double x) { return x; }
template <>
__device__ __forceinline__ ddr rconst<ddr>(double x) { return ddr{x, 0.0}; }
__device__ __forceinline__ double rmul(double a, double b) { return a * b; }
__device__ __forceinline__ ddr rmul(ddr a, ddr b) { return dd_mul(a, b); }
__device__ __forceinline__ bool is_pos(double a) { return a > 0.0; }
__device__ __forceinline__ bool is_pos(ddr a) { return a.hi > 0.0; }
// determinant of the last 2x2 block [[a, conj b], [b, g]]
__device__ __forceinline__ double det_last(double a, double b, double g) { return fma(a, g, -abs2(b)); }
__device__ __forceinline__ double det_last(double a, c64 b, double g) { return fma(a, g, -abs2(b)); }
__device__ __forceinline__ ddr det_last(ddr a, ddr b, ddr g) { return dd_add(dd_mul(a, g), dd_neg(dd_mul(b, b))); }

// ---- reciprocal and reciprocal square root ---------------------------------
// The hardware seeds (v_rcp_f64, v_rsq_f64) are good to about 2^-24; one
// correction of third order brings them to within one unit in the last place:
//   1/x:        e = 1 - x y,    y' = y + y (e + e^2)
//   1/sqrt(x):  d = 1 - x y^2,  y' = y + y d (1/2 + 3/8 d)
// (the Taylor series of (1 - e)^-1 and (1 - d)^-1/2 to second order; the
// neglected terms are O(e^3), O(d^3) ~ 2^-72).
__device__ __forceinline__ double rcp_nr(double x)
{
    const double y = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, y, 1.0);
    return fma(y, fma(e, e, e), y);
}

__device__ __forceinline__ double rsqrt_nr(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double h = x * y;
    const double d = fma(-h, y, 1.0);
    return fma(y * d, fma(d, 0.375, 0.5), y);
}

// double-double versions: the double result y0 (about one ulp) and one
// Newton correction with the residual formed to double-double accuracy,
//   1/x:        r = 1 - x y0,      y = y0 + y0 r
//   1/sqrt(x):  r = 1 - x y0^2,    y = y0 + y0 r / 2
// (r is about 2^-52, so the neglected r^2 terms are below 2^-104)
__device__ __forceinline__ ddr rcp_nr(ddr x)
{
#pragma clang fp contract(off)
    const double y0 = rcp_nr(x.hi);
    const double p = x.hi * y0;
    const double pe = fma(x.hi, y0, -p);
    const double r = fma(-x.lo, y0, (1.0 - p) - pe);
    return fast2sum(y0, y0 * r);
}

__device__ __forceinline__ ddr rsqrt_nr(ddr x)
{
#pragma clang fp contract(off)
    const double y0 = rsqrt_nr(x.hi);
    const double q = y0 * y0;
    const double qe = fma(y0, y0, -q);
    const double p = x.hi * q;
    const double pe = fma(x.hi, q, -p);
    double r = (1.0 - p) - pe;
    r = fma(-x.hi, qe, r);
    r = fma(-x.lo, q, r);
    return fast2sum(y0, 0.5 * y0 * r);
}

// ---- node entries
// entry e of block bi of a node whose granule arrays hold nb blocks
template <class S>
__device__ __forceinline__ S &blk(S *node, int nb, int bi, int e)
{
    return node[gpos((int)sizeof(S), nb, bi, e)];
}
template <class S>
__device__ __forceinline__ const S &blk(const S *node, int nb, int bi, int e)
{
    return node[gpos((int)sizeof(S), nb, bi, e)];
}

// triangular index -> (a, b), a >= b, with a(a+1)/2 + b = bi: the mode block
// of a block index (bidx), or the row and column of a packed entry (pidx)
__device__ __forceinline__ void block_ab(int bi, int &a, int &b)
{
    a = (int)((sqrtf(8.0f * (float)bi + 1.0f) - 1.0f) * 0.5f);
    if (a * (a + 1) / 2 > bi)
        --a;
    if ((a + 1) * (a + 2) / 2 <= bi)
        ++a;
    b = bi - a * (a + 1) / 2;
}

// ---- wave-uniform broadcast ------------------------------------------------
// The value of the first active lane, in scalar registers.  Loop bounds and
// exits built from it are provably uniform, so the compiler emits scalar
// branches and every lane runs the same iterations (a value broadcast with a
// lane shuffle is not known to be uniform, and a loop exiting on it may be
// structured so that lanes iterate without the lane that produced it).
__device__ __forceinline__ unsigned long long bcast_first(unsigned long long v)
{
    unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// ---- 2x2 pivot of one include step
template <class S>
struct Piv {
    RT<S> inv_a, inv_g, pdet;
    S ba;  // beta / alpha
};

template <class S>
__device__ __forceinline__ Piv<S> pivot(double a, S b, double g)
{
    Piv<S> p;
    p.inv_a = rcp_nr(a);
    p.ba = scale(b, p.inv_a);
    double g1 = g - p.inv_a * abs2(b);  // gamma - |beta|^2 / alpha
    p.inv_g = rcp_nr(g1);
    p.pdet = a * g1;  // |L_pp|^2 |L_p+1,p+1|^2
    return p;
}

__device__ __forceinline__ Piv<ddr> pivot(ddr a, ddr b, ddr g)
{
#pragma clang fp contract(off)
    Piv<ddr> p;
    p.inv_a = rcp_nr(a);
    p.ba = dd_mul(b, p.inv_a);
    const ddr g1 = sub_mul(g, b, p.ba);  // gamma - beta^2 / alpha
    p.inv_g = rcp_nr(g1);
    p.pdet = dd_mul(a, g1);
    return p;
}

// ---- accumulators ----------------------------------------------------------
// Terms are added with a sign known at compile time (SG = +1 or -1) relative
// to a lane's running sign `frame`; when the lane's sign changes between
// leaves the sums are negated (exact), and the final sum is hi * frame.
// r, r0, r1 are reciprocal square roots of determinants (positive).
//
// Double-double sum by Knuth's TwoSum (TAOCP vol. 2, 4.2.2): hi + lo carries
// the running sum, lo collects the exact rounding error of every addition.
// The pair of the last mode, SG (r1 - r0), is formed first by Dekker's
// Fast2Sum, r1 - r0 = s + err, which is exact when r1 >= r0 / 2 (then
// exponent(r1) >= exponent(r0), or the difference is exact by Sterbenz's
// lemma), i.e. whenever that mode's pivot determinant is at most 4.
struct AccDD {
    static constexpr bool kDD = true;  // reduce as double-double
    double hi = 0.0, lo = 0.0, abs_sum = 0.0, frame = 1.0;
    __device__ __forceinline__ void begin_leaf(double *) {}
    __device__ __forceinline__ void two_sum(double t)
    {
        double s = hi + t;
        double bb = s - hi;
        double e = (hi - (s - bb)) + (t - bb);
        hi = s;
        lo += e;
    }
    template <int SG, int TB = 0>
    __device__ __forceinline__ void add(double r)
    {
        two_sum(SG * r);
        abs_sum += r;
    }
    template <int SG, int TB = 0>
    __device__ __forceinline__ void add_pair(double r0, double r1)
    {
        const double s = r1 - r0;
        const double z = s - r1;
        const double err = -r0 - z;
        two_sum(SG * s);
        lo += SG * err;
        abs_sum += r0 + r1;
    }
    __device__ __forceinline__ void set_frame(double f)
    {
        const double m = f * frame;
        hi *= m;
        lo *= m;
        frame = f;
    }
};
// plain FP64 sum of the same terms, one by one, kept only for the dd-vs-FP64
// comparison
struct AccF64 {
    static constexpr bool kDD = false;
    double hi = 0.0, lo = 0.0, abs_sum = 0.0, frame = 1.0;
    __device__ __forceinline__ void begin_leaf(double *) {}
    template <int SG, int TB = 0>
    __device__ __forceinline__ void add(double r)
    {
        hi += SG * r;
        abs_sum += r;
    }
    template <int SG, int TB = 0>
    __device__ __forceinline__ void add_pair(double r0, double r1)
    {
        hi += -SG * r0;
        hi += SG * r1;
        abs_sum += r0 + r1;
    }
    __device__ __forceinline__ void set_frame(double f)
    {
        hi *= f * frame;
        frame = f;
    }
};

// every term stored instead of summed (all click patterns at once): the lane's
// 2^T terms of one tier-A leaf go to out[TB], TB the subset below the lane's
// node (bit M-1 of TB = the decision when M modes are left), each with its
// full sign (-1)^(#excluded); only the sum of |t| is kept
struct AccStore {
    static constexpr bool kDD = false;
    static constexpr double hi = 0.0, lo = 0.0;
    double abs_sum = 0.0, frame = 1.0;
    double *out = nullptr;
    __device__ __forceinline__ void begin_leaf(double *p) { out = p; }
    template <int SG, int TB = 0>
    __device__ __forceinline__ void add(double r)
    {
        *(__attribute__((address_space(1))) double *)(out + TB) = SG * frame * r;
        abs_sum += r;
    }
    template <int SG, int TB = 0>
    __device__ __forceinline__ void add_pair(double r0, double r1)
    {
        static_assert((TB & 1) == 0, "the last mode's pair is two neighbouring subsets");
        typedef double v2 __attribute__((ext_vector_type(2)));
        const v2 v = {-SG * frame * r0, SG * frame * r1};
        *(__attribute__((address_space(1))) v2 *)(out + TB) = v;
        abs_sum += r0 + r1;
    }
    __device__ __forceinline__ void set_frame(double f) { frame = f; }
};

// double-double sum of double-double terms (the higher-precision mode); the
// pair of the last mode is formed as a double-double difference first
struct AccQ {
    static constexpr bool kDD = true;
    double hi = 0.0, lo = 0.0, abs_sum = 0.0, frame = 1.0;
    __device__ __forceinline__ void begin_leaf(double *) {}
    __device__ __forceinline__ void acc(double th, double tl)
    {
        const ddr s = dd_add(ddr{hi, lo}, ddr{th, tl});
        hi = s.hi;
        lo = s.lo;
    }
    template <int SG, int TB = 0>
    __device__ __forceinline__ void add(ddr r)
    {
        acc(SG * r.hi, SG * r.lo);
        abs_sum += r.hi;
    }
    template <int SG, int TB = 0>
    __device__ __forceinline__ void add_pair(ddr r0, ddr r1)
    {
        const ddr d = dd_add(r1, dd_neg(r0));
        acc(SG * d.hi, SG * d.lo);
        abs_sum += r0.hi + r1.hi;
    }
    __device__ __forceinline__ void set_frame(double f)
    {
        const double m = f * frame;
        hi *= m;
        lo *= m;
        frame = f;
    }
};

// (a_hi, a_lo) + (b_hi, b_lo), renormalised
__device__ __forceinline__ void dd_add2(double &ahi, double &alo, double bhi, double blo)
{
    double s = ahi + bhi;
    double bb = s - ahi;
    double e = (ahi - (s - bb)) + (bhi - bb);
    e += alo + blo;
    double h = s + e;
    alo = e - (h - s);
    ahi = h;
}

}  // namespace tor
