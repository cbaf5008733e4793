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
    double inv_a, inv_g, pdet;
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
    double hi = 0.0, lo = 0.0, abs_sum = 0.0, frame = 1.0;
    __device__ __forceinline__ void two_sum(double t)
    {
        double s = hi + t;
        double bb = s - hi;
        double e = (hi - (s - bb)) + (t - bb);
        hi = s;
        lo += e;
    }
    template <int SG>
    __device__ __forceinline__ void add(double r)
    {
        two_sum(SG * r);
        abs_sum += r;
    }
    template <int SG>
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
    double hi = 0.0, lo = 0.0, abs_sum = 0.0, frame = 1.0;
    template <int SG>
    __device__ __forceinline__ void add(double r)
    {
        hi += SG * r;
        abs_sum += r;
    }
    template <int SG>
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
