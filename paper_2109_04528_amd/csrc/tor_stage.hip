// tor_stage.hip -- device staging of the input matrices, and sqrt(det(I - O)).
//
// One workgroup per matrix turns the caller's O (2n x 2n complex128,
// row-major, only its lower triangle read) into the layout a kernel reads:
//   * C = I - O as the Hermitian completion of its lower triangle;
//   * validation: every value read must be finite, and with
//     STAGE_CHECK_HERM the upper triangle must be the conjugate transpose of
//     the lower one (to 1e-12 relative);
//   * the Gaussian-state structure test.  The sampling matrix of a Gaussian
//     state in block order has the form [[P, Q], [conj Q, conj P]] with Q
//     symmetric (Sec. 1: A = I - Sigma^-1 from the Husimi covariance), and so
//     has C.  For such C the unitary w = [[1, 1], [-i, i]] / sqrt(2) applied
//     to every mode pair turns each 2x2 mode block [[p, q], [conj q, conj p]]
//     into the real block [[Re p + Re q, Im q - Im p], [Im p + Im q,
//     Re p - Re q]]; the result is real symmetric, and every principal
//     mode-submatrix keeps its determinant (w is unitary and acts inside
//     each mode), so the Torontonian is unchanged.  C is taken as structured
//     when both relations hold to 64 units of roundoff of max |C|; it is then
//     symmetrised exactly (P <- (P + conj P)/2 of the two diagonal blocks,
//     Q <- (Q + Q^T)/2) before the transform;
//   * packing: the node layout of tor_internal.hpp (real form in FP64, or in
//     double-double built from O itself for the double-double factor, or
//     the complex matrix), padded to the kernel's minimum size with
//     decoupled modes whose block of I - O is I/2 (such a mode multiplies the
//     Torontonian by 1/sqrt(1/4) - 1 = 1); or, for the removal-order kernel,
//     the complex matrix in the interleaved order a_0, a_0^dag, a_1, ... of
//     Sec. 2, lower triangle packed by rows.
// Positive definiteness is not tested here: every kernel tests the pivots
// of each subset it factorises, and the all-include subset is I - O itself.
//
// A pattern (sel) stages the principal submatrix of an M-mode O on the rows
// and columns {s, s + M : s in sel}, the matrix of a click pattern.
#include "tor_device.hpp"
#include "tor_internal.hpp"

namespace tor {

namespace {

constexpr double kStageU = 1.1102230246251565e-16;  // FP64 unit roundoff

// (a, b), a >= b, of the t-th entry of a lower triangle numbered by rows
__device__ inline void tri_ab(int t, int &a, int &b)
{
    a = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    if (a * (a + 1) / 2 > t)
        --a;
    if ((a + 1) * (a + 2) / 2 <= t)
        ++a;
    b = t - a * (a + 1) / 2;
}

// the input seen as a 2n x 2n matrix; with lds set, its lower triangle is
// read from there (packed by rows, pidx) instead of global memory
struct View {
    const double *O;
    long ld;
    int n;
    const int *sel;
    int M;
    const c64 *lds;
    __device__ int row(int a) const { return sel ? (a < n ? sel[a] : sel[a - n] + M) : a; }
    __device__ c64 og(int a, int b) const
    {
        const double *p = O + 2 * ((size_t)row(a) * (size_t)ld + (size_t)row(b));
        return c64{p[0], p[1]};
    }
    // entry (a, b), a >= b, of O
    __device__ c64 o(int a, int b) const { return lds ? lds[pidx(a, b)] : og(a, b); }
    // C = I - O, Hermitian completion of the lower triangle
    __device__ c64 c(int a, int b) const
    {
        if (a >= b) {
            const c64 v = o(a, b);
            return a == b ? c64{1.0 - v.x, 0.0} : c64{-v.x, -v.y};
        }
        const c64 v = o(b, a);
        return c64{-v.x, v.y};
    }
};

// host-order double-double helpers for the double-double form
struct hd {
    double hi, lo;
};
__device__ inline hd two_sum(double a, double b)
{
#pragma clang fp contract(off)
    const double s = a + b, bb = s - a;
    return hd{s, (a - (s - bb)) + (b - bb)};
}
__device__ inline hd hd_add(hd a, hd b)
{
#pragma clang fp contract(off)
    hd s = two_sum(a.hi, b.hi);
    const hd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return two_sum(s.hi, s.lo);
}
__device__ inline hd hd_neg(hd a) { return hd{-a.hi, -a.lo}; }
__device__ inline hd hd_half(hd a) { return hd{0.5 * a.hi, 0.5 * a.lo}; }

// entry (a, b) of I - O in double-double
__device__ inline void c_dd(const View &v, int a, int b, hd &re_, hd &im_)
{
    const bool up = a < b;
    const int i = up ? b : a, j = up ? a : b;
    const c64 x = v.o(i, j);
    re_ = two_sum(i == j ? 1.0 : 0.0, -x.x);
    im_ = hd{i == j ? 0.0 : (up ? x.y : -x.y), 0.0};
}

// real form entry: modes (mi, mj), components (ci, cj), of the symmetrised C
__device__ inline double real_entry(const View &v, int mi, int mj, int ci, int cj)
{
    const int n = v.n;
    const c64 p1 = v.c(mi, mj), p2 = v.c(mi + n, mj + n);
    const c64 q1 = v.c(mi, mj + n), q2 = v.c(mj, mi + n);
    const double pr = 0.5 * (p1.x + p2.x);
    const double pi = 0.5 * (p1.y - p2.y);
    const double qr = 0.5 * (q1.x + q2.x);
    const double qi = 0.5 * (q1.y + q2.y);
    if (ci == 0 && cj == 0)
        return pr + qr;
    if (ci == 0 && cj == 1)
        return qi - pi;
    if (ci == 1 && cj == 0)
        return pi + qi;
    return pr - qr;
}

__device__ inline hd quad_entry(const View &v, int mi, int mj, int ci, int cj)
{
    const int n = v.n;
    hd p1r, p1i, p2r, p2i, q1r, q1i, q2r, q2i;
    c_dd(v, mi, mj, p1r, p1i);
    c_dd(v, mi + n, mj + n, p2r, p2i);
    c_dd(v, mi, mj + n, q1r, q1i);
    c_dd(v, mj, mi + n, q2r, q2i);
    const hd pr = hd_half(hd_add(p1r, p2r)), pi = hd_half(hd_add(p1i, hd_neg(p2i)));
    const hd qr = hd_half(hd_add(q1r, q2r)), qi = hd_half(hd_add(q1i, q2i));
    if (ci == 0 && cj == 0)
        return hd_add(pr, qr);
    if (ci == 0 && cj == 1)
        return hd_add(qi, hd_neg(pi));
    if (ci == 1 && cj == 0)
        return hd_add(pi, qi);
    return hd_add(pr, hd_neg(qr));
}

__device__ inline double sq(double x, double y) { return x * x + y * y; }

// block-wide maxima of the K values v (every thread receives them); red
// holds K * NT / 64 doubles
template <int NT, int K>
__device__ inline void block_max(double (&v)[K], double *red)
{
    const int t = threadIdx.x;
    for (int k = 0; k < K; ++k)
        for (int off = 32; off >= 1; off >>= 1)
            v[k] = fmax(v[k], __shfl_xor(v[k], off));
    __syncthreads();
    if ((t & 63) == 0)
        for (int k = 0; k < K; ++k)
            red[k * (NT / 64) + (t >> 6)] = v[k];
    __syncthreads();
    for (int k = 0; k < K; ++k) {
        double r = red[k * (NT / 64)];
        for (int w = 1; w < NT / 64; ++w)
            r = fmax(r, red[k * (NT / 64) + w]);
        v[k] = r;
    }
}

}  // namespace

// lower-triangle entries staged in LDS: inputs up to n = 40 (51.8 KB);
// larger ones are read from global memory throughout
constexpr int STAGE_LDS_ENTRIES = NB(80);

template <int NT>
__global__ void __launch_bounds__(NT) tor_stage(const StageDesc *descs)
{
    __shared__ double red[5 * (NT / 64)];
    __shared__ c64 tri[STAGE_LDS_ENTRIES];
    const StageDesc D = descs[blockIdx.x];
    const int t = threadIdx.x;
    const int n = D.n, n2 = 2 * n;
    const bool in_lds = NB(n2) <= STAGE_LDS_ENTRIES;
    View v{D.O, D.ld, n, D.sel, D.M, nullptr};
    const unsigned fl = D.flags;

    // one pass over global memory: validation, max |C|, the Hermitian check,
    // and the lower triangle of O into LDS (a NaN fails every comparison
    // below, so it is caught by the finite test alone)
    double nonfin = 0.0, cmax2 = 0.0, dev2 = 0.0, hs2 = 0.0, hd2 = 0.0;
    const bool herm = (fl & STAGE_CHECK_HERM) != 0;
    auto lower = [&](int q, int a, int b) {
        const c64 x = v.og(a, b);
        if (!isfinite(x.x) || !isfinite(x.y))
            nonfin = 1.0;
        const c64 y = a == b ? c64{1.0 - x.x, 0.0} : c64{-x.x, -x.y};
        cmax2 = fmax(cmax2, sq(y.x, y.y));
        if (in_lds)
            tri[q] = x;
    };
    if (!herm) {
        // the lower triangle only, entry q = pidx(a, b)
        for (int q = t; q < NB(n2); q += NT) {
            int a, b;
            tri_ab(q, a, b);
            lower(q, a, b);
        }
    } else {
        for (int q = t; q < n2 * n2; q += NT) {
            const int a = q / n2, b = q - a * n2;
            if (a >= b)
                lower(pidx(a, b), a, b);
            const c64 x = v.og(a, b), y = v.og(b, a);
            if (!isfinite(x.x) || !isfinite(x.y))
                nonfin = 1.0;
            hs2 = fmax(hs2, sq(x.x, x.y));
            hd2 = fmax(hd2, sq(x.x - y.x, x.y + y.y));
        }
    }
    __syncthreads();
    if (in_lds)
        v.lds = tri;
    const bool interleaved = (fl & STAGE_INTERLEAVED) != 0;
    const bool dd = (fl & STAGE_DD) != 0;
    const bool want_real = !interleaved && (dd || (n > 0 && !(fl & STAGE_FORCE_CPLX)));
    if (want_real) {
        for (int q = t; q < n * n; q += NT) {
            const int i = q / n, j = q - i * n;
            // lower-right block = conj(upper-left); lower-left block symmetric
            const c64 d1a = v.c(i + n, j + n), d1b = v.c(i, j);
            const c64 d2a = v.c(i + n, j), d2b = v.c(j + n, i);
            dev2 = fmax(dev2, sq(d1a.x - d1b.x, d1a.y + d1b.y));
            dev2 = fmax(dev2, sq(d2a.x - d2b.x, d2a.y - d2b.y));
        }
    }
    double mx[5] = {nonfin, cmax2, dev2, hs2, hd2};
    block_max<NT, 5>(mx, red);
    nonfin = mx[0];
    cmax2 = mx[1];
    dev2 = mx[2];
    hs2 = mx[3];
    hd2 = mx[4];
    const double tol = 64.0 * kStageU * fmax(sqrt(cmax2), 1.0);
    const bool structured = want_real && dev2 <= tol * tol;
    int status = 0;
    if (nonfin != 0.0 || (herm && hd2 > 1e-24 * fmax(hs2, 1.0)) || (dd && !structured))
        status = STAGE_BAD_INPUT;
    const int path = structured ? (dd ? PATH_QUAD : PATH_REAL) : PATH_CPLX;
    const int N = interleaved ? n
                  : path == PATH_REAL ? max(n, REAL_R)
                  : path == PATH_QUAD ? max(n, QUAD_R)
                                      : max(n, D.min_cplx);
    if (t == 0) {
        D.info->status = status;
        D.info->path = path;
        D.info->N = N;
        D.info->cmax = sqrt(cmax2);
    }
    if (status != 0)
        return;

    if (interleaved) {
        // the removal-order layout: row x = 2 q + c is a_q (c = 0) or a_q^dag
        c64 *out = (c64 *)D.out;
        for (int q = t; q < NB(n2); q += NT) {
            int x, y;
            tri_ab(q, x, y);
            out[pidx(x, y)] = v.c((x >> 1) + (x & 1) * n, (y >> 1) + (y & 1) * n);
        }
        return;
    }
    // node layout: block bi = (a, b) of the reversed interleaved rows
    const int nb = NB(N);
    for (int q = t; q < 4 * nb; q += NT) {
        const int bi = q >> 2, e = q & 3;
        int a, b;
        tri_ab(bi, a, b);
        const int x = 2 * a + (e >> 1), y = 2 * b + (e & 1);
        const int qi = 2 * N - 1 - x, qj = 2 * N - 1 - y;
        const int mi = qi >> 1, ci = qi & 1, mj = qj >> 1, cj = qj & 1;
        const bool padm = mi >= n || mj >= n;
        if (path == PATH_REAL) {
            const double val = padm ? (qi == qj ? 0.5 : 0.0) : real_entry(v, mi, mj, ci, cj);
            ((double *)D.out)[gpos((int)sizeof(double), nb, bi, e)] = val;
        } else if (path == PATH_QUAD) {
            const hd val = padm ? hd{qi == qj ? 0.5 : 0.0, 0.0} : quad_entry(v, mi, mj, ci, cj);
            ((ddr *)D.out)[gpos((int)sizeof(ddr), nb, bi, e)] = ddr{val.hi, val.lo};
        } else {
            c64 val = padm ? c64{qi == qj ? 0.5 : 0.0, 0.0} : v.c(mi + ci * n, mj + cj * n);
            if (x == y)
                val.y = 0.0;
            ((c64 *)D.out)[gpos((int)sizeof(c64), nb, bi, e)] = val;
        }
    }
}

// sqrt(det(I - O)) of an M-mode O (device, leading dimension ld), by a
// Cholesky factorisation of the Hermitian completion of the lower triangle
// of C = I - O in the caller's scratch (2M x 2M c64): the product of the
// diagonal of L.  out[0] receives it, out[1] = 1 when a pivot was not
// positive (or not a number).  One workgroup, a barrier per column.
template <int NT>
__global__ void __launch_bounds__(NT) tor_sqrt_det(const double *O, long ld, int M, c64 *A, double *out)
{
    const int t = threadIdx.x, m2 = 2 * M;
    const View v{O, ld, M, nullptr, M, nullptr};
    for (int q = t; q < m2 * m2; q += NT) {
        const int a = q / m2, b = q - a * m2;
        if (a >= b)
            A[(size_t)a * m2 + b] = v.c(a, b);
    }
    __syncthreads();
    double prod = 1.0;
    bool bad = false;
    for (int j = 0; j < m2; ++j) {
        const double d = A[(size_t)j * m2 + j].x;
        if (!(d > 0.0))
            bad = true;
        const double ljj = sqrt(d);
        prod *= ljj;
        const double inv = 1.0 / ljj;
        // column j of L, then the trailing update of the lower triangle
        for (int i = j + 1 + t; i < m2; i += NT) {
            c64 &x = A[(size_t)i * m2 + j];
            x = c64{x.x * inv, x.y * inv};
        }
        __syncthreads();
        const int r = m2 - j - 1;
        for (int q = t; q < r * (r + 1) / 2; q += NT) {
            int a, b;
            tri_ab(q, a, b);
            a += j + 1;
            b += j + 1;
            const c64 la = A[(size_t)a * m2 + j], lb = A[(size_t)b * m2 + j];
            c64 &x = A[(size_t)a * m2 + b];
            // x -= la * conj(lb)
            x.x -= la.x * lb.x + la.y * lb.y;
            x.y -= la.y * lb.x - la.x * lb.y;
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = prod;
        out[1] = bad ? 1.0 : 0.0;
    }
}

constexpr int STAGE_THREADS = 1024;
constexpr int DET_THREADS = 1024;

hipError_t launch_stage(const StageDesc *descs, int count, hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((tor_stage<STAGE_THREADS>), dim3(count), dim3(STAGE_THREADS), 0, s, descs);
    return hipGetLastError();
}

hipError_t launch_sqrt_det(const double *O, long ld, int M, c64 *scratch, double *out, hipStream_t s)
{
    hipLaunchKernelGGL((tor_sqrt_det<DET_THREADS>), dim3(1), dim3(DET_THREADS), 0, s, O, ld, M, scratch, out);
    return hipGetLastError();
}

}  // namespace tor
