// tor_runtime.cpp -- host runtime and C ABI of libtor (see include/tor.h).
//
// Host side of one evaluation:
//   1. validate the arguments and every value of the lower triangle;
//   2. form I - O from its lower triangle (Hermitian completion) and run one
//      FP64 Cholesky of the full matrix: positive definiteness of I - O
//      implies it for every principal submatrix (Cauchy interlacing), so
//      this single check covers all 2^n subsets;
//   3. pack the matrix in the device layout (tor_internal.hpp), padded to the
//      kernel's minimum size with decoupled modes whose block of I - O is
//      I/2 -- such a mode multiplies the Torontonian by 1/sqrt(1/4) - 1 = 1;
//      Gaussian-state matrices are also packed in their real form;
//   4. one persistent launch over all (matrix, subtree root) items, then the
//      fixed-order per-matrix reduction of the root slots, one copy back.
//
// Serving (tor_submit / tor_poll) keeps each admitted request's matrix and
// root slots in a device pool and runs them in chunked launches: every launch
// takes a bounded number of subsets from the admitted requests, smallest
// remaining work first, so requests that arrive while others run join the
// next launch instead of waiting for the longest one to finish.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/tor.h"
#include "tor_internal.hpp"

using namespace tor;

namespace {

constexpr double kU = 1.1102230246251565e-16;  // FP64 unit roundoff
constexpr double kUdd = 4.930380657631324e-32; // 2^-104, double-double roundoff

struct Staged {
    int n = 0;                    // modes of the input
    int N = 0;                    // modes after padding (complex path)
    std::vector<c64> packed;      // complex device layout
    int path = PATH_CPLX;         // PATH_REAL when the Gaussian-state structure is found
    int Nr = 0;                   // modes after padding (real and double-double paths)
    std::vector<double> packed_r; // real symmetric form, same layout
    std::vector<ddr> packed_q;    // the same form in double-double
};

struct Request {
    unsigned long long ticket = 0;
    Staged st;
    tor_result res{};
    bool done = false;
    // device state once admitted
    int path = PATH_CPLX;
    int N = 0, k = 0;
    long long nroots = 0, next_root = 0;
    long long root_work = 0;  // subsets per root
    size_t pool_off = 0, pool_len = 0;
    char *dC = nullptr;
    double *dSlots = nullptr;
    float device_ms = 0.f;
};

struct TuneEntry {
    bool valid = false;
    int k = 0, waves = 0;
    float ms = 0.f;
};

}  // namespace

struct tor_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    tor_options opt{};
    int num_cu = 0;
    int fit[NPATH] = {1, 1, 1};  // resident one-wave workgroups per CU, per path
    int grid[NPATH] = {0, 0, 0}; // persistent grid per path
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::mutex mu;        // serialises device work on this context
    TuneEntry tune[NPATH][MAX_N + 1];
    std::string arch;

    // serving
    std::mutex smu;
    std::condition_variable scv;
    std::deque<Request *> pending;
    std::unordered_map<unsigned long long, Request *> live;
    unsigned long long next_ticket = 1;
    std::thread worker;
    bool stop = false;
    int admitted = 0;
    int max_queue = 1 << 16;
    long long chunk_subsets = 1ll << 29;  // work per serving launch
    double oldest_share = 0.5;            // of it, guaranteed to the oldest request
    char *pool = nullptr;
    size_t pool_bytes = 256ull << 20;
    std::map<size_t, size_t> pool_free;  // offset -> length
};

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? TOR_OK : (e == hipErrorOutOfMemory ? TOR_E_NOMEM : TOR_E_DEVICE); }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Cholesky of the Hermitian 2n x 2n matrix C (full storage), FP64, as
// C = U^H U with U upper triangular, row by row: row j is scaled by the
// reciprocal square root of its pivot, then subtracted from every later row
// (contiguous updates, no serial dot products).  True when every pivot is
// positive.
bool hpd_check(int n2, const std::vector<double> &C)
{
    std::vector<double> U(C);
    for (int j = 0; j < n2; j++) {
        double *uj = &U[2 * (size_t)j * n2];
        const double d = uj[2 * j];
        if (!(d > 0.0))
            return false;
        const double inv = 1.0 / std::sqrt(d);
        for (int k = 2 * j; k < 2 * n2; k++)
            uj[k] *= inv;
        for (int i = j + 1; i < n2; i++) {
            double *ui = &U[2 * (size_t)i * n2];
            // row i -= conj(U[j][i]) * row j
            const double fr = uj[2 * i], fi = -uj[2 * i + 1];
            for (int k = i; k < n2; k++) {
                const double xr = uj[2 * k], xi = uj[2 * k + 1];
                ui[2 * k] -= fr * xr - fi * xi;
                ui[2 * k + 1] -= fr * xi + fi * xr;
            }
        }
    }
    return true;
}

// sqrt(det(I - O)) of the Hermitian completion of the lower triangle of
// I - O (2M x 2M, O row-major with leading dimension ld, complex
// interleaved), by a Cholesky factorisation in long double: the product of
// the diagonal of L.  Returns a negative value when I - O is not positive
// definite.
double host_sqrt_det(int M, const double *O, long ld)
{
    const int m2 = 2 * M;
    std::vector<long double> Cr((size_t)m2 * m2), Ci((size_t)m2 * m2);
    for (int a = 0; a < m2; a++)
        for (int b = 0; b <= a; b++) {
            const long double orr = O[2 * ((size_t)a * ld + b)], oi = O[2 * ((size_t)a * ld + b) + 1];
            const long double cr = (a == b ? 1.0L : 0.0L) - orr, ci = (a == b) ? 0.0L : -oi;
            Cr[(size_t)a * m2 + b] = cr;
            Ci[(size_t)a * m2 + b] = ci;
        }
    long double prod = 1.0L;
    for (int j = 0; j < m2; j++) {
        long double d = Cr[(size_t)j * m2 + j];
        for (int k = 0; k < j; k++)
            d -= Cr[(size_t)j * m2 + k] * Cr[(size_t)j * m2 + k] + Ci[(size_t)j * m2 + k] * Ci[(size_t)j * m2 + k];
        if (!(d > 0.0L))
            return -1.0;
        const long double ljj = std::sqrt(d);
        prod *= ljj;
        Cr[(size_t)j * m2 + j] = ljj;
        Ci[(size_t)j * m2 + j] = 0.0L;
        for (int i = j + 1; i < m2; i++) {
            long double sr = Cr[(size_t)i * m2 + j], si = Ci[(size_t)i * m2 + j];
            for (int k = 0; k < j; k++) {
                // L[i][k] conj(L[j][k])
                const long double ar = Cr[(size_t)i * m2 + k], ai = Ci[(size_t)i * m2 + k];
                const long double br = Cr[(size_t)j * m2 + k], bi = Ci[(size_t)j * m2 + k];
                sr -= ar * br + ai * bi;
                si -= ai * br - ar * bi;
            }
            Cr[(size_t)i * m2 + j] = sr / ljj;
            Ci[(size_t)i * m2 + j] = si / ljj;
        }
    }
    return (double)prod;
}

// Gaussian-state structure.  The sampling matrix of a Gaussian state in
// block order has the form [[P, Q], [conj Q, conj P]] (Sec. 1: A = I - Sigma^-1
// from the Husimi covariance), and so has C = I - O.  For such C the unitary
// w = [[1, 1], [-i, i]] / sqrt(2) applied to every mode pair turns each 2x2
// mode block [[p, q], [conj q, conj p]] into the real block
// [[Re p + Re q, Im q - Im p], [Im p + Im q, Re p - Re q]]; the result is real
// symmetric and every principal mode-submatrix keeps its determinant
// (w is unitary and acts inside each mode), so the Torontonian is unchanged.
// C is taken as structured when both defining relations hold to 64 units of
// roundoff of max |C|; it is then symmetrised exactly (P <- (P + conj P')/2,
// Q <- (Q + Q^T)/2) before the transform.  With quad set the form is built in
// double-double from O itself (1 - O_ii and every sum of the transform are
// exact or rounded to 2^-106), for the double-double factor.
// Host double-double helpers: exact sum by TwoSum, renormalised sum.
struct hdd {
    double hi, lo;
};
hdd h_two_sum(double a, double b)
{
    const double s = a + b, bb = s - a;
    return hdd{s, (a - (s - bb)) + (b - bb)};
}
hdd h_add(hdd a, hdd b)
{
    hdd s = h_two_sum(a.hi, b.hi);
    const hdd t = h_two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = h_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return h_two_sum(s.hi, s.lo);
}
hdd h_neg(hdd a) { return hdd{-a.hi, -a.lo}; }

// Gaussian-state structure test of C (full Hermitian storage, block order):
// both defining relations hold to 64 units of roundoff of max |C| (cmax2 =
// max |C|^2).  Squared magnitudes are compared, so no square root is taken.
bool gaussian_structure(int n, const std::vector<double> &C, double cmax2)
{
    const int n2 = 2 * n;
    auto cre = [&](int a, int b) { return C[2 * ((size_t)a * n2 + b)]; };
    auto cim = [&](int a, int b) { return C[2 * ((size_t)a * n2 + b) + 1]; };
    double dev2 = 0.0;
    auto sq = [](double x, double y) { return x * x + y * y; };
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            // lower-right block = conj(upper-left); lower-left block symmetric
            dev2 = std::max(dev2, sq(cre(i + n, j + n) - cre(i, j), cim(i + n, j + n) + cim(i, j)));
            dev2 = std::max(dev2, sq(cre(i + n, j) - cre(j + n, i), cim(i + n, j) - cim(j + n, i)));
        }
    const double tol = 64.0 * kU * std::max(std::sqrt(cmax2), 1.0);
    return dev2 <= tol * tol;
}

// The real form of the symmetrised C, dense (2n x 2n, row-major, row 2 i + c
// for component c of mode i).
void real_form(int n, const std::vector<double> &C, std::vector<double> &R)
{
    const int n2 = 2 * n;
    auto cre = [&](int a, int b) { return C[2 * ((size_t)a * n2 + b)]; };
    auto cim = [&](int a, int b) { return C[2 * ((size_t)a * n2 + b) + 1]; };
    R.assign((size_t)n2 * n2, 0.0);
    for (int mi = 0; mi < n; mi++)
        for (int mj = 0; mj < n; mj++) {
            const double pr = 0.5 * (cre(mi, mj) + cre(mi + n, mj + n));
            const double pi = 0.5 * (cim(mi, mj) - cim(mi + n, mj + n));
            // Q = upper-right block, symmetrised: (Q + Q^T)/2, with Q[i][j] = C[i][j+n]
            const double qr = 0.5 * (cre(mi, mj + n) + cre(mj, mi + n));
            const double qi = 0.5 * (cim(mi, mj + n) + cim(mj, mi + n));
            double *r0 = &R[(size_t)(2 * mi) * n2 + 2 * mj], *r1 = r0 + n2;
            r0[0] = pr + qr;
            r0[1] = qi - pi;
            r1[0] = pi + qi;
            r1[1] = pr - qr;
        }
}

// Cholesky of the real symmetric m x m matrix R (row-major, full storage),
// FP64, in a scratch copy, in the row form of hpd_check: true when every
// pivot is positive.
bool spd_check(int m, const std::vector<double> &R)
{
    std::vector<double> U(R);
    for (int j = 0; j < m; j++) {
        double *uj = &U[(size_t)j * m];
        const double d = uj[j];
        if (!(d > 0.0))
            return false;
        const double inv = 1.0 / std::sqrt(d);
        for (int k = j; k < m; k++)
            uj[k] *= inv;
        for (int i = j + 1; i < m; i++) {
            double *ui = &U[(size_t)i * m];
            const double f = uj[i];
            for (int k = i; k < m; k++)
                ui[k] -= f * uj[k];
        }
    }
    return true;
}

// Pack the real form R (dense, from real_form) for the real path, or, with
// quad set, the same form rebuilt in double-double from O for the
// double-double factor.
void stage_real(int n, const std::vector<double> &R, const double *O, long ld, bool quad, Staged &st)
{
    const int n2 = 2 * n;
    const int N = std::max(n, quad ? QUAD_R : REAL_R);
    st.Nr = N;
    if (quad) {
        // entry (a, b) of I - O from the lower triangle of O, in double-double
        auto cdd = [&](int a, int b, hdd &re_, hdd &im_) {
            const bool up = a < b;
            const int i = up ? b : a, j = up ? a : b;
            const double orr = O[2 * ((size_t)i * ld + j)], oi = O[2 * ((size_t)i * ld + j) + 1];
            re_ = h_two_sum(i == j ? 1.0 : 0.0, -orr);
            im_ = hdd{i == j ? 0.0 : (up ? oi : -oi), 0.0};
        };
        auto qblk = [&](int mi, int mj, int ci, int cj) -> hdd {
            if (mi >= n || mj >= n)
                return hdd{(mi == mj && ci == cj) ? 0.5 : 0.0, 0.0};
            hdd p1r, p1i, p2r, p2i, q1r, q1i, q2r, q2i;
            cdd(mi, mj, p1r, p1i);
            cdd(mi + n, mj + n, p2r, p2i);
            cdd(mi, mj + n, q1r, q1i);
            cdd(mj, mi + n, q2r, q2i);
            auto half = [](hdd v) { return hdd{0.5 * v.hi, 0.5 * v.lo}; };
            const hdd pr = half(h_add(p1r, p2r)), pi = half(h_add(p1i, h_neg(p2i)));
            const hdd qr = half(h_add(q1r, q2r)), qi = half(h_add(q1i, q2i));
            if (ci == 0 && cj == 0) return h_add(pr, qr);
            if (ci == 0 && cj == 1) return h_add(qi, h_neg(pi));
            if (ci == 1 && cj == 0) return h_add(pi, qi);
            return h_add(pr, h_neg(qr));
        };
        st.packed_q.assign((size_t)NSZ(N), ddr{0.0, 0.0});
        for (int a = 0; a < N; a++)
            for (int b = 0; b <= a; b++)
                for (int e = 0; e < 4; e++) {
                    const int qi = 2 * N - 1 - (2 * a + (e >> 1)), qj = 2 * N - 1 - (2 * b + (e & 1));
                    const hdd v = qblk(qi / 2, qj / 2, qi % 2, qj % 2);
                    st.packed_q[(size_t)gpos((int)sizeof(ddr), NB(N), bidx(a, b), e)] = ddr{v.hi, v.lo};
                }
        st.path = PATH_QUAD;
        return;
    }
    st.packed_r.assign((size_t)NSZ(N), 0.0);
    // entry (qi, qj) of the form, interleaved order; modes >= n are padding
    auto rel = [&](int qi, int qj) -> double {
        if (qi >= n2 || qj >= n2)
            return qi == qj ? 0.5 : 0.0;
        return R[(size_t)qi * n2 + qj];
    };
    for (int a = 0; a < N; a++)
        for (int b = 0; b <= a; b++)
            for (int e = 0; e < 4; e++) {
                const int qi = 2 * N - 1 - (2 * a + (e >> 1)), qj = 2 * N - 1 - (2 * b + (e & 1));
                st.packed_r[(size_t)gpos((int)sizeof(double), NB(N), bidx(a, b), e)] = rel(qi, qj);
            }
    st.path = PATH_REAL;
}

// Validate, check, pack one matrix.  O is host memory.
int stage_matrix(int n, const double *O, long ld, unsigned flags, int min_modes, Staged &st)
{
    st.n = n;
    if (n < 0)
        return TOR_E_INVAL;
    if (n > 0 && (!O || ld < 2L * n))
        return TOR_E_INVAL;
    const int n2 = 2 * n;
    // Hermitian completion of the lower triangle of C = I - O
    std::vector<double> C((size_t)n2 * n2 * 2);
    double cmax2 = 0.0;  // max |C|^2
    for (int a = 0; a < n2; a++)
        for (int b = 0; b <= a; b++) {
            double orr = O[2 * ((size_t)a * ld + b)], oi = O[2 * ((size_t)a * ld + b) + 1];
            if (!std::isfinite(orr) || !std::isfinite(oi))
                return TOR_E_INVAL;
            double cr = (a == b ? 1.0 : 0.0) - orr;
            double ci = (a == b) ? 0.0 : -oi;
            cmax2 = std::max(cmax2, cr * cr + ci * ci);
            C[2 * ((size_t)a * n2 + b)] = cr;
            C[2 * ((size_t)a * n2 + b) + 1] = ci;
            C[2 * ((size_t)b * n2 + a)] = cr;
            C[2 * ((size_t)b * n2 + a) + 1] = -ci;
        }
    if (flags & TOR_CHECK_HERMITIAN) {
        double scale = 0.0, diff = 0.0;
        for (int a = 0; a < n2; a++)
            for (int b = 0; b < n2; b++) {
                double orr = O[2 * ((size_t)a * ld + b)], oi = O[2 * ((size_t)a * ld + b) + 1];
                double tr = O[2 * ((size_t)b * ld + a)], ti = -O[2 * ((size_t)b * ld + a) + 1];
                if (!std::isfinite(orr) || !std::isfinite(oi))
                    return TOR_E_INVAL;
                scale = std::max(scale, std::hypot(orr, oi));
                diff = std::max(diff, std::hypot(orr - tr, oi - ti));
            }
        if (diff > 1e-12 * std::max(scale, 1.0))
            return TOR_E_INVAL;
    }
    // The real path when the Gaussian-state structure holds: positive
    // definiteness is checked on the real symmetric form the kernel factors
    // (it has the eigenvalues of the symmetrised C), and the complex layout
    // is not built.  The empty matrix stays on the complex path unless the
    // double-double factor is asked for.
    const bool dd = (flags & TOR_FACTOR_DD) != 0;
    st.N = std::max(n, min_modes);
    if ((dd || (n > 0 && !(flags & TOR_FORCE_COMPLEX))) && gaussian_structure(n, C, cmax2)) {
        std::vector<double> R;
        real_form(n, C, R);
        if (n > 0 && !spd_check(n2, R))
            return TOR_E_NOT_PD;
        stage_real(n, R, O, ld, dd, st);
        return TOR_OK;
    }
    // the double-double factor runs on the real form only
    if (dd)
        return TOR_E_INVAL;
    if (n > 0 && !hpd_check(n2, C))
        return TOR_E_NOT_PD;
    // pack: N modes, reversed interleaved rows; row q (interleaved) of mode q/2,
    // component q%2 -> block-order row (q/2) + (q%2) n; modes >= n are padding
    const int N = st.N;
    st.packed.assign((size_t)NSZ(N), c64{0.0, 0.0});
    auto elem = [&](int qi, int qj) -> c64 {
        int mi = qi / 2, ci = qi % 2, mj = qj / 2, cj = qj % 2;
        if (mi >= n || mj >= n)
            return (qi == qj) ? c64{0.5, 0.0} : c64{0.0, 0.0};
        int a = mi + ci * n, b = mj + cj * n;
        return c64{C[2 * ((size_t)a * n2 + b)], C[2 * ((size_t)a * n2 + b) + 1]};
    };
    for (int a = 0; a < N; a++)
        for (int b = 0; b <= a; b++)
            for (int e = 0; e < 4; e++) {
                const int x = 2 * a + (e >> 1), y = 2 * b + (e & 1);
                c64 v = elem(2 * N - 1 - x, 2 * N - 1 - y);
                if (x == y)
                    v.y = 0.0;
                st.packed[(size_t)gpos((int)sizeof(c64), NB(N), bidx(a, b), e)] = v;
            }
    st.path = PATH_CPLX;
    return TOR_OK;
}


int path_R(int path) { return path == PATH_QUAD ? QUAD_R : path == PATH_REAL ? REAL_R : CPLX_R; }
int modes_of(const Staged &m, int path) { return path == PATH_CPLX ? m.N : m.Nr; }
// bytes per scalar of the device layout (c64 and ddr are both 16)
size_t path_esz(int path) { return path == PATH_REAL ? sizeof(double) : sizeof(c64); }
const void *packed_of(const Staged &m, int path)
{
    return path == PATH_QUAD ? (const void *)m.packed_q.data()
                             : path == PATH_REAL ? (const void *)m.packed_r.data() : (const void *)m.packed.data();
}
// tor_result.path: 1 real, 2 complex, 3 real with a double-double factor
int api_path(int path) { return path == PATH_REAL ? 1 : path == PATH_QUAD ? 3 : 2; }
const char *path_name(int path) { return path == PATH_REAL ? "real" : path == PATH_QUAD ? "quad" : "complex"; }

int default_grid(const tor_ctx *ctx, int path) { return ctx->grid[path]; }

// launch grid for a set of matrices: the tuned waves/CU of the largest one,
// else as many one-wave workgroups as the LDS allows (at most 8 per CU)
int launch_grid(const tor_ctx *ctx, int path, int Nmax)
{
    const int n = std::min(Nmax, MAX_N);
    const TuneEntry &t = ctx->tune[path][n];
    if (ctx->opt.waves_per_cu <= 0 && t.valid)
        return ctx->num_cu * std::min(t.waves, ctx->fit[path]);
    return default_grid(ctx, path);
}

// split depth: the tuned value for this size, else about four subtree roots
// per persistent wave, never deeper than the levels above the last R modes
int choose_k(const tor_ctx *ctx, int N, int path)
{
    const int LA = N - path_R(path);
    if (LA <= 0)
        return 0;
    if (ctx->opt.split_k > 0)
        return std::min(ctx->opt.split_k, LA);
    const TuneEntry &t = ctx->tune[path][std::min(N, MAX_N)];
    if (t.valid)
        return std::min(t.k, LA);
    int g = 1;
    while ((1 << g) < default_grid(ctx, path))
        ++g;
    return std::min(LA, g + 2);
}

int ensure_ws(tor_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->ws_bytes)
        return TOR_OK;
    if (!ctx->own_ws)
        return TOR_E_NOMEM;
    if (ctx->ws) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    size_t want = align_up(bytes + (bytes >> 3), 1 << 20);
    if (hipMalloc((void **)&ctx->ws, want) != hipSuccess) {
        ctx->ws = nullptr;
        return TOR_E_NOMEM;
    }
    ctx->ws_bytes = want;
    return TOR_OK;
}

// Workspace bytes a launch needs after its matrices and slots: descriptors,
// reduction descriptors, queue counter, results, per-wave tier-A stacks.
struct LaunchLayout {
    size_t b_probs, b_red, b_counter, b_res;
    long long stride;
    size_t total(int grid) const { return b_probs + b_red + b_counter + b_res + (size_t)stride * grid; }
};

LaunchLayout launch_layout(int path, int count, int nred, int Nmax)
{
    const size_t esz = path_esz(path);
    LaunchLayout L;
    L.b_probs = align_up(sizeof(ProblemDesc) * std::max(count, 1), 256);
    L.b_red = align_up(sizeof(ProblemDesc) * std::max(nred, 1), 256);
    L.b_counter = 256;
    L.b_res = align_up(sizeof(double) * 4 * std::max(nred, 1), 256);
    L.stride = (long long)align_up(esz * (size_t)std::max(Gsum(Nmax - 1) - Gsum(path_R(path) - 1), 1ll), 256);
    return L;
}

// One persistent launch over the root ranges in descs (C, slots, N, k,
// root_begin, nroots filled in), followed by the reduction of the matrices
// listed in reduce (indices into descs, or none), into results (4 doubles
// each).  The workspace from byte ws_off on holds descriptors, counter,
// results and the per-wave tier-A stacks.  When ws_off > 0 the bytes below it
// hold data the descriptors point to, and the caller has already sized the
// workspace (a reallocation here would move that data).
int run_launch(tor_ctx *ctx, int path, std::vector<ProblemDesc> &descs, const std::vector<int> &reduce,
               size_t ws_off, int grid, std::vector<double> *results, float *ms)
{
    const int count = (int)descs.size();
    long long total = 0;
    int Nmax = 0;
    for (auto &d : descs) {
        d.item_begin = total;
        total += d.nroots;
        Nmax = std::max(Nmax, d.N);
    }
    std::vector<ProblemDesc> red;
    for (int i : reduce)
        red.push_back(descs[i]);
    const int nred = (int)red.size();
    const LaunchLayout Lo = launch_layout(path, count, nred, Nmax);
    const size_t need = ws_off + Lo.total(grid);
    if (ws_off > 0 && need > ctx->ws_bytes)
        return TOR_E_NOMEM;  // the caller sizes the workspace first
    int rc = ensure_ws(ctx, need);
    if (rc != TOR_OK)
        return rc;
    char *dProbs = ctx->ws + ws_off;
    char *dRed = dProbs + Lo.b_probs;
    unsigned long long *dCounter = (unsigned long long *)(dRed + Lo.b_red);
    double *dRes = (double *)((char *)dCounter + Lo.b_counter);
    char *dScr = (char *)dRes + Lo.b_res;
    const long long stride = Lo.stride;
    // descriptors and reduction descriptors at their exact byte offsets
    std::vector<char> hdesc(Lo.b_probs + Lo.b_red, 0);
    std::memcpy(hdesc.data(), descs.data(), sizeof(ProblemDesc) * count);
    if (nred)
        std::memcpy(hdesc.data() + Lo.b_probs, red.data(), sizeof(ProblemDesc) * nred);

    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dProbs, hdesc.data(), hdesc.size(), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = launch_zero(dCounter, 1, ctx->stream);
    MainParams mp{};
    mp.probs = (const ProblemDesc *)dProbs;
    mp.nprob = count;
    mp.total_items = total;
    mp.counter = dCounter;
    mp.scratch = dScr;
    mp.scratch_stride = stride;
    // the double-double factor always sums in double-double
    const bool dd = ctx->opt.accum != TOR_ACCUM_FP64 || path == PATH_QUAD;
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev0, ctx->stream);
    if (e == hipSuccess && total > 0)
        e = launch_main(path, dd, mp, grid, ctx->stream);
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev1, ctx->stream);  // device_ms: the main kernel alone
    std::vector<double> hres(4 * (size_t)std::max(nred, 1));
    if (e == hipSuccess && nred > 0) {
        e = launch_reduce((const ProblemDesc *)dRed, nred, dRes, dd, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hres.data(), dRes, sizeof(double) * 4 * nred, hipMemcpyDeviceToHost, ctx->stream);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess)
        return hip_status(e);
    if (ms)
        (void)hipEventElapsedTime(ms, ctx->ev0, ctx->ev1);
    if (results)
        results->assign(hres.begin(), hres.begin() + 4 * nred);
    return TOR_OK;
}

// Synchronous path: all roots of every matrix in one launch, matrices with
// more modes first.  results: 4 doubles per matrix (input order).
int run_recursive(tor_ctx *ctx, int path, std::vector<Staged *> &mats, std::vector<int> &ks,
                  std::vector<double> &results, float *ms, std::vector<double> *slots_out)
{
    const size_t esz = path_esz(path);
    const int count = (int)mats.size();
    std::vector<int> order(count);
    for (int i = 0; i < count; i++)
        order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return modes_of(*mats[a], path) > modes_of(*mats[b], path); });
    // workspace: matrices, then slots, then what run_launch needs
    std::vector<size_t> c_off(count), s_off(count);
    size_t off = 0;
    long long nslots = 0;
    int Nmax = 0;
    for (int s = 0; s < count; s++) {
        const Staged *m = mats[order[s]];
        c_off[s] = off;
        off = align_up(off + esz * (size_t)NSZ(modes_of(*m, path)), 256);
        Nmax = std::max(Nmax, modes_of(*m, path));
    }
    for (int s = 0; s < count; s++) {
        s_off[s] = off + sizeof(double) * 4 * (size_t)nslots;
        nslots += 1ll << ks[order[s]];
    }
    off = align_up(off + sizeof(double) * 4 * (size_t)nslots, 256);
    const int grid = launch_grid(ctx, path, Nmax);
    // size the workspace for everything before placing data in it
    int rc = ensure_ws(ctx, off + launch_layout(path, count, count, Nmax).total(grid));
    if (rc != TOR_OK)
        return rc;
    std::vector<char> hbuf(s_off.empty() ? 0 : s_off[0], 0);
    std::vector<ProblemDesc> descs(count);
    std::vector<int> red(count);
    for (int s = 0; s < count; s++) {
        const Staged *m = mats[order[s]];
        std::memcpy(hbuf.data() + c_off[s], packed_of(*m, path), esz * (size_t)NSZ(modes_of(*m, path)));
        ProblemDesc &d = descs[s];
        d.C = ctx->ws + c_off[s];
        d.slots = (double *)(ctx->ws + s_off[s]);
        d.N = modes_of(*m, path);
        d.k = ks[order[s]];
        d.root_begin = 0;
        d.nroots = 1ll << d.k;
        red[s] = s;
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess && !hbuf.empty())
        e = hipMemcpyAsync(ctx->ws, hbuf.data(), hbuf.size(), hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess)
        return hip_status(e);
    std::vector<double> res;
    rc = run_launch(ctx, path, descs, red, off, grid, &res, ms);
    if (rc != TOR_OK)
        return rc;
    results.assign(4 * (size_t)count, 0.0);
    for (int s = 0; s < count; s++)
        for (int j = 0; j < 4; j++)
            results[4 * (size_t)order[s] + j] = res[4 * (size_t)s + j];
    if (slots_out) {
        slots_out->resize(4 * (size_t)nslots);
        e = hipMemcpy(slots_out->data(), ctx->ws + s_off[0], sizeof(double) * 4 * nslots, hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            return hip_status(e);
    }
    return TOR_OK;
}

void fill_result(const Staged &st, int path, const double *r, float ms, tor_result *out)
{
    std::memset(out, 0, sizeof(*out));
    out->tor = r[0];
    out->tor_lo = r[1];
    // a padding mode (its block of I - O is I/2) turns each term t into the
    // pair -t, +2t: Tor is unchanged and the padded sum of |t| is 3 times the
    // input's, so it is scaled back (3^pad is exact for pad < 34)
    const int pad = modes_of(st, path) - st.n;
    out->sum_abs = pad > 0 ? r[2] / std::pow(3.0, pad) : r[2];
    const double v = std::fabs(r[0] + r[1]);
    // each term carries a relative rounding error of a few units of roundoff
    // (FP64, or 2^-104 for the double-double factor) per factorisation step;
    // independent errors add in quadrature
    const double R = v > 0.0 ? out->sum_abs / v : INFINITY;
    const double u = path == PATH_QUAD ? kUdd : kU;
    out->err_est = u * (double)std::max(st.n, 1) * R / std::sqrt(std::ldexp(1.0, st.n));
    out->subsets = 1ull << st.n;
    out->status = (r[3] != 0.0 || !std::isfinite(r[0])) ? TOR_E_NUMERIC : TOR_OK;
    out->path = api_path(path);
    out->device_ms = ms;
}

int copy_input_to_host(int n, const double *O, long ld, unsigned flags, std::vector<double> &tmp, const double *&host)
{
    host = O;
    if (!(flags & TOR_INPUT_DEVICE) || n == 0)
        return TOR_OK;
    if (!O || ld < 2L * n)
        return TOR_E_INVAL;
    tmp.resize((size_t)2 * n * ld * 2);
    hipError_t e = hipMemcpy(tmp.data(), O, sizeof(double) * tmp.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_status(e);
    host = tmp.data();
    return TOR_OK;
}

// Split depths for a launch of several matrices: roots of about equal work,
// about four per persistent wave over the whole launch (a lone matrix keeps
// its own tuned or default depth).
void batch_ks(const tor_ctx *ctx, int path, const std::vector<Staged *> &grp, std::vector<int> &ks)
{
    if (grp.size() == 1 || ctx->opt.split_k > 0) {
        for (size_t j = 0; j < grp.size(); j++)
            ks[j] = choose_k(ctx, modes_of(*grp[j], path), path);
        return;
    }
    double work = 0.0;
    int Nmax = 0;
    for (Staged *m : grp) {
        work += std::ldexp(1.0, modes_of(*m, path));
        Nmax = std::max(Nmax, modes_of(*m, path));
    }
    const double per_root = std::max(work / (4.0 * launch_grid(ctx, path, Nmax)), 1.0);
    const int lg = (int)std::floor(std::log2(per_root) + 0.5);
    for (size_t j = 0; j < grp.size(); j++) {
        const int N = modes_of(*grp[j], path);
        ks[j] = std::max(0, std::min(N - lg, N - path_R(path)));
    }
}

// Launch the staged matrices, one launch per arithmetic path.
int run_staged(tor_ctx *ctx, std::vector<Staged *> &mats, const std::vector<int> &idx, int fixed_k,
               tor_result *out, std::vector<double> *slots_out, int *k_out)
{
    int first_err = TOR_OK;
    const int order[NPATH] = {PATH_REAL, PATH_CPLX, PATH_QUAD};
    for (int path : order) {
        std::vector<Staged *> grp;
        std::vector<int> gidx, ks;
        for (size_t j = 0; j < mats.size(); j++)
            if (mats[j]->path == path) {
                grp.push_back(mats[j]);
                gidx.push_back(idx[j]);
                const int N = modes_of(*mats[j], path);
                ks.push_back(std::min(std::max(fixed_k, 0), std::max(N - path_R(path), 0)));
            }
        if (grp.empty())
            continue;
        if (fixed_k < 0)
            batch_ks(ctx, path, grp, ks);
        std::vector<double> res;
        float ms = 0.f;
        int rc = run_recursive(ctx, path, grp, ks, res, &ms, slots_out);
        if (rc != TOR_OK)
            return rc;
        for (size_t j = 0; j < grp.size(); j++) {
            fill_result(*grp[j], path, &res[4 * j], ms, &out[gidx[j]]);
            if (out[gidx[j]].status != TOR_OK && first_err == TOR_OK)
                first_err = out[gidx[j]].status;
        }
        if (k_out)
            *k_out = ks[0];
    }
    return first_err;
}

int eval_many(tor_ctx *ctx, int count, const int *n, const double *const *O, const long *ld, tor_result *out,
              int fixed_k, std::vector<double> *slots_out, int *k_out, unsigned flags)
{
    std::vector<Staged> st(count);
    std::vector<int> rcs(count, TOR_OK);
    // host staging (validation, HPD check, packing) of a batch on a few threads
    auto stage_one = [&](int i) {
        if (n[i] > ctx->opt.max_n) {
            rcs[i] = TOR_E_INVAL;
            return;
        }
        std::vector<double> tmp;
        const double *host;
        int rc = copy_input_to_host(n[i], O ? O[i] : nullptr, ld ? ld[i] : 0, flags, tmp, host);
        if (rc == TOR_OK)
            rc = stage_matrix(n[i], host, ld ? ld[i] : 0, flags, CPLX_R, st[i]);
        rcs[i] = rc;
    };
    const int nthr = (count >= 8 && !(flags & TOR_INPUT_DEVICE))
                         ? (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()))
                         : 1;
    if (nthr <= 1) {
        for (int i = 0; i < count; i++)
            stage_one(i);
    } else {
        std::vector<std::thread> pool;
        for (int t = 0; t < nthr; t++)
            pool.emplace_back([&, t] {
                for (int i = t; i < count; i += nthr)
                    stage_one(i);
            });
        for (auto &th : pool)
            th.join();
    }
    std::vector<Staged *> ok;
    std::vector<int> idx;
    int first_err = TOR_OK;
    for (int i = 0; i < count; i++) {
        if (rcs[i] != TOR_OK) {
            out[i] = tor_result{};
            out[i].status = rcs[i];
            if (first_err == TOR_OK)
                first_err = rcs[i];
            continue;
        }
        ok.push_back(&st[i]);
        idx.push_back(i);
    }
    if (!ok.empty()) {
        int rc = run_staged(ctx, ok, idx, fixed_k, out, slots_out, k_out);
        if (rc != TOR_OK && first_err == TOR_OK)
            first_err = rc;
    }
    return first_err;
}

// ---- serving: device pool ----------------------------------------------------

bool pool_alloc(tor_ctx *ctx, size_t len, size_t &off)
{
    len = align_up(len, 256);
    for (auto it = ctx->pool_free.begin(); it != ctx->pool_free.end(); ++it)
        if (it->second >= len) {
            off = it->first;
            const size_t rest = it->second - len;
            ctx->pool_free.erase(it);
            if (rest)
                ctx->pool_free[off + len] = rest;
            return true;
        }
    return false;
}

void pool_release(tor_ctx *ctx, size_t off, size_t len)
{
    len = align_up(len, 256);
    auto it = ctx->pool_free.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != ctx->pool_free.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        ctx->pool_free.erase(nx);
    }
    if (it != ctx->pool_free.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            ctx->pool_free.erase(it);
        }
    }
}

// Split depth of a served request: roots of at most a quarter-wave share of
// one launch's budget, so that no single root outlasts the launch it is in.
int serve_k(const tor_ctx *ctx, const Request &r)
{
    const int LA = std::max(r.N - path_R(r.path), 0);
    const double per_root = std::max((double)ctx->chunk_subsets / (4.0 * launch_grid(ctx, r.path, r.N)), 1.0);
    const int lg = (int)std::floor(std::log2(per_root));
    const int k = std::max(choose_k(ctx, r.N, r.path), r.N - lg);
    return std::max(0, std::min(k, std::min(LA, 20)));
}

size_t request_bytes(const Request &r)
{
    const size_t esz = path_esz(r.path);
    return align_up(esz * (size_t)NSZ(r.N), 256) + align_up(sizeof(double) * 4 * (size_t)r.nroots, 256);
}

// One scheduling round for one path: pick root ranges for a launch, run it,
// retire the finished requests.  Called with ctx->mu held.
int serve_round(tor_ctx *ctx, int path, std::vector<Request *> &active, std::vector<Request *> &finished)
{
    std::vector<Request *> cand;
    for (Request *r : active)
        if (r->path == path && r->next_root < r->nroots)
            cand.push_back(r);
    if (cand.empty())
        return TOR_OK;
    // the oldest request always gets its share of the budget (oldest_share);
    // the rest goes to the requests with the least remaining work
    Request *oldest = *std::min_element(cand.begin(), cand.end(),
                                        [](Request *a, Request *b) { return a->ticket < b->ticket; });
    std::stable_sort(cand.begin(), cand.end(), [](Request *a, Request *b) {
        return (a->nroots - a->next_root) * a->root_work < (b->nroots - b->next_root) * b->root_work;
    });
    long long budget = ctx->chunk_subsets;
    std::vector<ProblemDesc> descs;
    std::vector<Request *> used;
    auto take = [&](Request *r, long long share) {
        long long n = std::max(1ll, share / std::max(r->root_work, 1ll));
        n = std::min(n, r->nroots - r->next_root);
        ProblemDesc d{};
        d.C = r->dC;
        d.slots = r->dSlots;
        d.N = r->N;
        d.k = r->k;
        d.root_begin = r->next_root;
        d.nroots = n;
        descs.push_back(d);
        used.push_back(r);
        r->next_root += n;
        budget -= n * r->root_work;
    };
    take(oldest, (long long)(ctx->oldest_share * (double)budget));
    for (Request *r : cand) {
        if (budget <= 0)
            break;
        if (r->next_root < r->nroots)
            take(r, budget);
    }
    int Nmax = 0;
    for (auto &d : descs)
        Nmax = std::max(Nmax, d.N);
    // reduce the requests that this launch completes
    std::vector<int> red;
    for (size_t i = 0; i < used.size(); i++)
        if (used[i]->next_root == used[i]->nroots && std::find(used.begin(), used.begin() + i, used[i]) == used.begin() + i)
            red.push_back((int)i);
    std::vector<ProblemDesc> rdesc;
    for (int i : red) {
        ProblemDesc d = descs[i];
        rdesc.push_back(d);
    }
    std::vector<double> res;
    float ms = 0.f;
    int rc = run_launch(ctx, path, descs, red, 0, launch_grid(ctx, path, Nmax), &res, &ms);
    for (Request *r : used)
        r->device_ms += ms / (float)used.size();
    if (rc != TOR_OK) {
        for (Request *r : used) {
            r->res = tor_result{};
            r->res.status = rc;
            r->next_root = r->nroots;
            if (std::find(finished.begin(), finished.end(), r) == finished.end())
                finished.push_back(r);
        }
        return rc;
    }
    for (size_t j = 0; j < red.size(); j++) {
        Request *r = used[red[j]];
        fill_result(r->st, path, &res[4 * j], r->device_ms, &r->res);
        finished.push_back(r);
    }
    return TOR_OK;
}

void serve_loop(tor_ctx *ctx)
{
    std::vector<Request *> active;
    for (;;) {
        std::vector<Request *> admit;
        {
            std::unique_lock<std::mutex> lk(ctx->smu);
            ctx->scv.wait(lk, [&] { return ctx->stop || !ctx->pending.empty() || !active.empty(); });
            if (ctx->stop)
                return;
            // admission by device footprint, in arrival order
            while (!ctx->pending.empty()) {
                Request *r = ctx->pending.front();
                r->k = serve_k(ctx, *r);
                r->nroots = 1ll << r->k;
                r->root_work = 1ll << (r->N - r->k);
                if (!ctx->pool) {
                    if (hipSetDevice(ctx->device) != hipSuccess ||
                        hipMalloc((void **)&ctx->pool, ctx->pool_bytes) != hipSuccess) {
                        ctx->pool = nullptr;
                        break;
                    }
                    ctx->pool_free.clear();
                    ctx->pool_free[0] = ctx->pool_bytes;
                }
                size_t off;
                const size_t len = request_bytes(*r);
                if (!pool_alloc(ctx, len, off))
                    break;
                r->pool_off = off;
                r->pool_len = len;
                r->dC = ctx->pool + off;
                r->dSlots = (double *)(ctx->pool + off + align_up(path_esz(r->path) * (size_t)NSZ(r->N), 256));
                ctx->pending.pop_front();
                admit.push_back(r);
                ++ctx->admitted;
            }
        }
        std::vector<Request *> finished;
        {
            std::lock_guard<std::mutex> g(ctx->mu);
            hipError_t e = hipSetDevice(ctx->device);
            for (Request *r : admit) {
                const void *src = packed_of(r->st, r->path);
                const size_t bytes = path_esz(r->path) * (size_t)NSZ(r->N);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(r->dC, src, bytes, hipMemcpyHostToDevice, ctx->stream);
                active.push_back(r);
            }
            if (e != hipSuccess) {
                for (Request *r : admit) {
                    r->res = tor_result{};
                    r->res.status = hip_status(e);
                    r->next_root = r->nroots;
                    finished.push_back(r);
                }
            } else {
                for (int path : {PATH_REAL, PATH_CPLX, PATH_QUAD})
                    serve_round(ctx, path, active, finished);
            }
        }
        if (finished.empty() && admit.empty() && active.empty())
            continue;
        {
            std::lock_guard<std::mutex> g(ctx->smu);
            for (Request *r : finished) {
                pool_release(ctx, r->pool_off, r->pool_len);
                r->done = true;
                --ctx->admitted;
                active.erase(std::remove(active.begin(), active.end(), r), active.end());
            }
        }
        ctx->scv.notify_all();
    }
}

// ---- autotuning ------------------------------------------------------------

int tune_one(tor_ctx *ctx, int path, int n, TuneEntry &best)
{
    // timing does not depend on the values: I - O = I/2 has the Gaussian-state
    // structure (real path) and is well inside the positive-definite cone
    std::vector<double> O((size_t)2 * n * 2 * n * 2, 0.0);
    for (int i = 0; i < 2 * n; i++)
        O[2 * ((size_t)i * 2 * n + i)] = 0.5;
    Staged st;
    const unsigned fl = path == PATH_CPLX ? (unsigned)TOR_FORCE_COMPLEX : path == PATH_QUAD ? (unsigned)TOR_FACTOR_DD : 0u;
    int rc = stage_matrix(n, O.data(), 2 * n, fl, CPLX_R, st);
    if (rc != TOR_OK)
        return rc;
    if (st.path != path)
        return TOR_E_INVAL;
    const int N = modes_of(st, path);
    const int LA = std::max(N - path_R(path), 0);
    best = TuneEntry{};
    const int wave_opts[5] = {2, 4, 6, 8, ctx->fit[path]};
    for (int wi = 0; wi < 5; wi++) {
        const int w = wave_opts[wi];
        if (w > ctx->fit[path] || (wi == 4 && (w == 2 || w == 4 || w == 6 || w == 8)))
            continue;
        const int grid = ctx->num_cu * w;
        int g = 1;
        while ((1 << g) < grid)
            ++g;
        const int klo = std::min(LA, std::max(0, g - 1)), khi = std::min(LA, g + 3);
        for (int k = klo; k <= khi; ++k) {
            float tmin = 1e30f;
            for (int rep = 0; rep < 3; rep++) {
                std::vector<Staged *> mats{&st};
                std::vector<int> ks{k};
                // run with this grid: temporarily pin the table entry
                TuneEntry save = ctx->tune[path][std::min(N, MAX_N)];
                ctx->tune[path][std::min(N, MAX_N)] = TuneEntry{true, k, w, 0.f};
                std::vector<double> res;
                float ms = 0.f;
                rc = run_recursive(ctx, path, mats, ks, res, &ms, nullptr);
                ctx->tune[path][std::min(N, MAX_N)] = save;
                if (rc != TOR_OK)
                    return rc;
                if (rep > 0)
                    tmin = std::min(tmin, ms);
            }
            if (!best.valid || tmin < best.ms)
                best = TuneEntry{true, k, w, tmin};
        }
    }
    return TOR_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

void tor_default_options(tor_options *opt)
{
    if (!opt)
        return;
    std::memset(opt, 0, sizeof(*opt));
    opt->max_n = 40;
    opt->accum = TOR_ACCUM_DD;
}

const char *tor_strerror(int code)
{
    switch (code) {
    case TOR_OK: return "ok";
    case TOR_PENDING: return "pending";
    case TOR_E_INVAL: return "invalid argument";
    case TOR_E_NOT_PD: return "I - O is not Hermitian positive definite";
    case TOR_E_NUMERIC: return "numerical failure (non-positive pivot) inside the walk";
    case TOR_E_BUSY: return "admission refused: serving queue full";
    case TOR_E_NOMEM: return "out of memory";
    case TOR_E_DEVICE: return "device error or no usable GPU";
    case TOR_E_TIMEOUT: return "timed out";
    case TOR_E_UNKNOWN: return "unknown ticket";
    default: return "unrecognised status code";
    }
}

size_t tor_workspace_size(int max_n, int split_k, int max_inflight)
{
    if (max_n < 0 || max_n > MAX_N)
        return 0;
    // bounds over all paths: the smaller R has more roots and a deeper
    // tier-A stack; 16-byte scalars; at most MAX_FIT waves on each of 256 CUs
    const int Rmin = std::min(std::min(REAL_R, CPLX_R), QUAD_R);
    const int N = std::max(max_n, std::max(std::max(REAL_R, CPLX_R), QUAD_R));
    const int k = split_k > 0 ? split_k : 14;
    const int cnt = std::max(max_inflight, 1);
    const long long items = (1ll << std::min(k, std::max(N - Rmin, 0))) * cnt;
    const size_t grid = 256 * MAX_FIT;
    const size_t scr = align_up(sizeof(c64) * (size_t)std::max(Gsum(N - 1) - Gsum(Rmin - 1), 1ll), 256) * grid;
    return align_up(sizeof(c64) * (size_t)NSZ(N), 256) * cnt + 2 * align_up(sizeof(ProblemDesc) * cnt, 256) + 256 +
           align_up(32 * (size_t)items, 256) + align_up(32 * (size_t)cnt, 256) + scr + (1 << 20);
}

int tor_create(tor_ctx **out, const tor_options *opt)
{
    if (!out)
        return TOR_E_INVAL;
    *out = nullptr;
    tor_options o;
    tor_default_options(&o);
    if (opt)
        o = *opt;
    if (o.max_n <= 0)
        o.max_n = 40;
    if (o.max_n > MAX_N || o.split_k < 0 || o.split_k > 40 || o.waves_per_cu < 0 || o.waves_per_cu > 16 ||
        (o.accum != TOR_ACCUM_DD && o.accum != TOR_ACCUM_FP64) ||
        ((o.flags & TOR_FACTOR_DD) && (o.flags & TOR_FORCE_COMPLEX)))
        return TOR_E_INVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0 || o.device < 0 || o.device >= ndev)
        return TOR_E_DEVICE;
    tor_ctx *ctx = new (std::nothrow) tor_ctx();
    if (!ctx)
        return TOR_E_NOMEM;
    ctx->opt = o;
    ctx->device = o.device;
    if (hipSetDevice(o.device) != hipSuccess) {
        delete ctx;
        return TOR_E_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, o.device) != hipSuccess) {
        delete ctx;
        return TOR_E_DEVICE;
    }
    ctx->num_cu = prop.multiProcessorCount;
    ctx->arch = prop.gcnArchName;
    // persistent grid: as many one-wave workgroups per CU as the kernel's
    // registers and LDS allow
    for (int path = 0; path < NPATH; path++) {
        int fit = main_occupancy(path);
        if (fit <= 0) {
            delete ctx;
            return TOR_E_DEVICE;
        }
        fit = std::min(fit, MAX_FIT);
        ctx->fit[path] = fit;
        const int w = o.waves_per_cu > 0 ? std::min(o.waves_per_cu, fit) : fit;
        ctx->grid[path] = ctx->num_cu * w;
    }
    if (o.stream) {
        ctx->stream = (hipStream_t)o.stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return TOR_E_DEVICE;
        }
        ctx->own_stream = true;
    }
    if (o.workspace) {
        ctx->ws = (char *)o.workspace;
        ctx->ws_bytes = o.workspace_bytes;
        ctx->own_ws = false;
    } else {
        ctx->own_ws = true;
    }
    if (hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess) {
        tor_destroy(ctx);
        return TOR_E_DEVICE;
    }
    ctx->worker = std::thread(serve_loop, ctx);
    *out = ctx;
    return TOR_OK;
}

void tor_destroy(tor_ctx *ctx)
{
    if (!ctx)
        return;
    {
        std::unique_lock<std::mutex> lk(ctx->smu);
        ctx->stop = true;
    }
    ctx->scv.notify_all();
    if (ctx->worker.joinable())
        ctx->worker.join();  // the scheduler finishes its current launch first
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        (void)hipSetDevice(ctx->device);
        if (ctx->stream)
            (void)hipStreamSynchronize(ctx->stream);
        if (ctx->own_ws && ctx->ws)
            (void)hipFree(ctx->ws);
        if (ctx->pool)
            (void)hipFree(ctx->pool);
        if (ctx->ev0)
            (void)hipEventDestroy(ctx->ev0);
        if (ctx->ev1)
            (void)hipEventDestroy(ctx->ev1);
        if (ctx->own_stream && ctx->stream)
            (void)hipStreamDestroy(ctx->stream);
    }
    ctx->pending.clear();  // every pending request is also in live
    for (auto &kv : ctx->live)
        delete kv.second;
    delete ctx;
}

int tor_eval(tor_ctx *ctx, int n, const double *O, long ld, tor_result *out)
{
    if (!ctx || !out)
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    const double *Op[1] = {O};
    long lds[1] = {ld};
    int ns[1] = {n};
    tor_result r{};
    int rc = eval_many(ctx, 1, ns, Op, lds, &r, -1, nullptr, nullptr, ctx->opt.flags);
    if (rc == TOR_E_INVAL && r.status == TOR_E_INVAL)
        return rc;
    *out = r;
    return rc;
}

int tor_eval_batch(tor_ctx *ctx, int count, const int *n, const double *const *O, const long *ld, tor_result *out)
{
    if (!ctx || count < 0 || (count > 0 && (!n || !O || !ld || !out)))
        return TOR_E_INVAL;
    if (count == 0)
        return TOR_OK;
    std::lock_guard<std::mutex> g(ctx->mu);
    return eval_many(ctx, count, n, O, ld, out, -1, nullptr, nullptr, ctx->opt.flags);
}

int tor_eval_partials(tor_ctx *ctx, int n, const double *O, long ld, int k_max, int *k_out, double *partials,
                      tor_result *out)
{
    if (!ctx || !out || !k_out || !partials || k_max < 0 || k_max > 30)
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    const double *Op[1] = {O};
    long lds[1] = {ld};
    int ns[1] = {n};
    std::vector<double> slots;
    int k = 0;
    tor_result r{};
    int rc = eval_many(ctx, 1, ns, Op, lds, &r, k_max, &slots, &k, ctx->opt.flags);
    if (rc != TOR_OK && rc != TOR_E_NUMERIC)
        return rc;
    *out = r;
    *k_out = k;
    // padding modes scale each partial's sum of |t| by 3 (see fill_result)
    const int pad = std::max(n, path_R(r.path == 1)) - n;
    const double p3 = std::pow(3.0, pad);
    for (long long i = 0; i < (1ll << k); i++) {
        partials[3 * i] = slots[4 * i];
        partials[3 * i + 1] = slots[4 * i + 1];
        partials[3 * i + 2] = pad > 0 ? slots[4 * i + 2] / p3 : slots[4 * i + 2];
    }
    return rc;
}
int tor_click_probs(tor_ctx *ctx, int M, const double *O, long ld, int count, const unsigned long long *patterns,
                    double *probs, tor_result *results)
{
    if (!ctx || M < 0 || M > 64 || count < 0 || (count > 0 && (!patterns || !probs)) || (M > 0 && !O) ||
        (M > 0 && ld < 2L * M))
        return TOR_E_INVAL;
    for (int i = 0; i < count; i++) {
        if (M < 64 && (patterns[i] >> M) != 0)
            return TOR_E_INVAL;
        if (__builtin_popcountll(patterns[i]) > ctx->opt.max_n)
            return TOR_E_INVAL;
    }
    std::lock_guard<std::mutex> g(ctx->mu);
    std::vector<double> tmp;
    const double *host = O;
    int rc = copy_input_to_host(M, O, ld, ctx->opt.flags, tmp, host);
    if (rc != TOR_OK)
        return rc;
    const double sq = M > 0 ? host_sqrt_det(M, host, ld) : 1.0;
    if (!(sq > 0.0))
        return TOR_E_NOT_PD;
    // the principal submatrix of every pattern: rows and columns {s, s + M}
    std::vector<std::vector<double>> subs(count);
    std::vector<int> ns(count);
    std::vector<const double *> ptrs(count);
    std::vector<long> lds(count);
    for (int i = 0; i < count; i++) {
        std::vector<int> sel;
        for (int q = 0; q < M; q++)
            if ((patterns[i] >> q) & 1ull)
                sel.push_back(q);
        const int k = (int)sel.size();
        std::vector<int> idx(2 * k);
        for (int a = 0; a < k; a++) {
            idx[a] = sel[a];
            idx[k + a] = sel[a] + M;
        }
        subs[i].assign((size_t)2 * k * 2 * k * 2, 0.0);
        for (int a = 0; a < 2 * k; a++)
            for (int b = 0; b < 2 * k; b++) {
                subs[i][2 * ((size_t)a * 2 * k + b)] = host[2 * ((size_t)idx[a] * ld + idx[b])];
                subs[i][2 * ((size_t)a * 2 * k + b) + 1] = host[2 * ((size_t)idx[a] * ld + idx[b]) + 1];
            }
        ns[i] = k;
        ptrs[i] = subs[i].data();
        lds[i] = std::max(2 * k, 1);
    }
    std::vector<tor_result> res(std::max(count, 1));
    // the submatrices are host copies even when O was on the device
    rc = count > 0 ? eval_many(ctx, count, ns.data(), ptrs.data(), lds.data(), res.data(), -1, nullptr, nullptr,
                               ctx->opt.flags & ~(unsigned)TOR_INPUT_DEVICE)
                   : TOR_OK;
    for (int i = 0; i < count; i++) {
        probs[i] = res[i].status == TOR_OK ? (res[i].tor + res[i].tor_lo) * sq : NAN;
        if (results)
            results[i] = res[i];
    }
    return rc;
}

int tor_eval_plain(tor_ctx *ctx, int n, const double *O, long ld, unsigned long long mask_begin,
                   unsigned long long mask_end, tor_result *out)
{
    if (!ctx || !out || n < 1 || n > 34 || mask_begin > mask_end || mask_end > (1ull << n))
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    std::vector<double> tmp;
    const double *host;
    int rc = copy_input_to_host(n, O, ld, ctx->opt.flags, tmp, host);
    Staged st;
    if (rc == TOR_OK)  // the comparison kernels run on the complex matrix
        rc = stage_matrix(n, host, ld, (ctx->opt.flags & ~(unsigned)TOR_FACTOR_DD) | TOR_FORCE_COMPLEX, 0, st);
    if (rc != TOR_OK)
        return rc;
    const int chunk = 16;
    const size_t bC = align_up(sizeof(c64) * st.packed.size(), 256);
    const int pgrid = ctx->grid[PATH_CPLX];
    const size_t bParts = align_up(sizeof(double) * 4 * pgrid, 256);
    rc = ensure_ws(ctx, bC + 256 + bParts + 256);
    if (rc != TOR_OK)
        return rc;
    char *dC = ctx->ws;
    unsigned long long *dCounter = (unsigned long long *)(dC + bC);
    double *dParts = (double *)((char *)dCounter + 256);
    double *dRes = (double *)((char *)dParts + bParts);
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dC, st.packed.data(), sizeof(c64) * st.packed.size(), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = launch_zero(dCounter, 1, ctx->stream);
    PlainParams pp{};
    pp.C = dC;
    pp.n = n;
    pp.mask_begin = mask_begin;
    pp.mask_end = mask_end;
    pp.counter = dCounter;
    pp.partials = dParts;
    pp.chunk = chunk;
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev0, ctx->stream);
    if (e == hipSuccess)
        e = launch_plain(pp, pgrid, ctx->stream);
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev1, ctx->stream);
    if (e == hipSuccess)
        e = launch_plain_reduce(dParts, pgrid, dRes, ctx->stream);
    double h[4] = {0, 0, 0, 0};
    if (e == hipSuccess)
        e = hipMemcpyAsync(h, dRes, sizeof(h), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess)
        return hip_status(e);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    st.N = n;
    fill_result(st, PATH_CPLX, h, ms, out);
    out->subsets = mask_end - mask_begin;
    return out->status;
}

int tor_eval_removal(tor_ctx *ctx, int n, const double *O, long ld, tor_result *out)
{
    if (!ctx || !out || n < 0 || n > REMOVAL_MAX_N || n > ctx->opt.max_n)
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    std::vector<double> tmp;
    const double *host;
    int rc = copy_input_to_host(n, O, ld, ctx->opt.flags, tmp, host);
    Staged st;
    if (rc == TOR_OK)  // validation and the positive-definiteness check
        rc = stage_matrix(n, host, ld, (ctx->opt.flags & ~(unsigned)TOR_FACTOR_DD) | TOR_FORCE_COMPLEX, 0, st);
    if (rc != TOR_OK)
        return rc;
    // I - O in the interleaved order a_0, a_0^dag, a_1, ... (the ordering of
    // Sec. 2), the Hermitian completion of its lower triangle, packed by rows
    std::vector<c64> Ci((size_t)E(std::max(n, 1)), c64{0.0, 0.0});
    for (int x = 0; x < 2 * n; x++)
        for (int y = 0; y <= x; y++) {
            const int bx = (x >> 1) + (x & 1) * n, by = (y >> 1) + (y & 1) * n;
            const bool lower = bx >= by;
            const int i = lower ? bx : by, j = lower ? by : bx;
            const double orr = host[2 * ((size_t)i * ld + j)], oi = host[2 * ((size_t)i * ld + j) + 1];
            c64 v{(i == j ? 1.0 : 0.0) - orr, i == j ? 0.0 : -oi};
            if (!lower)
                v.y = -v.y;
            Ci[(size_t)pidx(x, y)] = v;
        }
    const int grid = ctx->num_cu * MAX_FIT;
    int k = 0;
    while (k < n && (1ll << k) < 4ll * grid)
        ++k;
    const size_t bC = align_up(sizeof(c64) * Ci.size(), 256);
    const size_t bParts = align_up(sizeof(double) * 4 * grid, 256);
    const long long stride = (long long)align_up(sizeof(c64) * (size_t)(n - k + 1) * (size_t)NSZ(n), 256);
    const size_t bScr = (size_t)stride * grid;
    rc = ensure_ws(ctx, bC + 256 + bParts + 256 + bScr);
    if (rc != TOR_OK)
        return rc;
    char *dC = ctx->ws;
    unsigned long long *dCounter = (unsigned long long *)(dC + bC);
    double *dParts = (double *)((char *)dCounter + 256);
    double *dRes = (double *)((char *)dParts + bParts);
    char *dScr = (char *)dRes + 256;
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dC, Ci.data(), sizeof(c64) * Ci.size(), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = launch_zero(dCounter, 1, ctx->stream);
    RemovalParams rp{};
    rp.C = dC;
    rp.n = n;
    rp.k = k;
    rp.counter = dCounter;
    rp.scratch = dScr;
    rp.scratch_stride = stride;
    rp.partials = dParts;
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev0, ctx->stream);
    if (e == hipSuccess)
        e = launch_removal(rp, grid, ctx->stream);
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev1, ctx->stream);
    if (e == hipSuccess)
        e = launch_plain_reduce(dParts, grid, dRes, ctx->stream);
    double h[4] = {0, 0, 0, 0};
    if (e == hipSuccess)
        e = hipMemcpyAsync(h, dRes, sizeof(h), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess)
        return hip_status(e);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    st.N = n;
    fill_result(st, PATH_CPLX, h, ms, out);
    return out->status;
}

int tor_debug_math(tor_ctx *ctx, int count, const double *x, double *out)
{
    if (!ctx || count <= 0 || !x || !out)
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    const size_t bx = align_up(sizeof(double) * count, 256);
    int rc = ensure_ws(ctx, 5 * bx);
    if (rc != TOR_OK)
        return rc;
    double *dx = (double *)ctx->ws;
    double *dout = (double *)(ctx->ws + bx);
    hipError_t e = hipMemcpyAsync(dx, x, sizeof(double) * count, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = launch_math_probe(dx, dout, count, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, dout, sizeof(double) * 4 * count, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    return hip_status(e);
}

// ---- serving ---------------------------------------------------------------

int tor_submit(tor_ctx *ctx, int n, const double *O, long ld, unsigned long long *ticket)
{
    if (!ctx || !ticket)
        return TOR_E_INVAL;
    if (n < 0 || n > ctx->opt.max_n)
        return TOR_E_INVAL;
    Request *r = new (std::nothrow) Request();
    if (!r)
        return TOR_E_NOMEM;
    std::vector<double> tmp;
    const double *host;
    int rc = copy_input_to_host(n, O, ld, ctx->opt.flags, tmp, host);
    if (rc == TOR_OK)
        rc = stage_matrix(n, host, ld, ctx->opt.flags, CPLX_R, r->st);
    if (rc != TOR_OK) {
        delete r;
        return rc;
    }
    r->path = r->st.path;
    r->N = modes_of(r->st, r->path);
    r->k = std::min(std::max(r->N - path_R(r->path), 0), 20);  // largest split admission may choose
    r->nroots = 1ll << r->k;
    if (request_bytes(*r) > ctx->pool_bytes) {
        delete r;
        return TOR_E_NOMEM;
    }
    {
        std::lock_guard<std::mutex> g(ctx->smu);
        if ((int)ctx->live.size() >= ctx->max_queue) {
            delete r;
            return TOR_E_BUSY;
        }
        r->ticket = ctx->next_ticket++;
        ctx->live[r->ticket] = r;
        ctx->pending.push_back(r);
        *ticket = r->ticket;
    }
    ctx->scv.notify_all();
    return TOR_OK;
}

int tor_poll(tor_ctx *ctx, unsigned long long ticket, tor_result *out)
{
    if (!ctx || !out)
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->smu);
    auto it = ctx->live.find(ticket);
    if (it == ctx->live.end())
        return TOR_E_UNKNOWN;
    if (!it->second->done)
        return TOR_PENDING;
    *out = it->second->res;
    delete it->second;
    ctx->live.erase(it);
    return TOR_OK;
}

int tor_drain(tor_ctx *ctx, int timeout_ms)
{
    if (!ctx)
        return TOR_E_INVAL;
    std::unique_lock<std::mutex> lk(ctx->smu);
    auto pred = [&] { return ctx->pending.empty() && ctx->admitted == 0; };
    if (timeout_ms < 0) {
        ctx->scv.wait(lk, pred);
        return TOR_OK;
    }
    return ctx->scv.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred) ? TOR_OK : TOR_E_TIMEOUT;
}

int tor_serve_config(tor_ctx *ctx, long long chunk_subsets, double oldest_share, int max_queue)
{
    if (!ctx || chunk_subsets < 1024 || !(oldest_share >= 0.0 && oldest_share <= 1.0) || max_queue < 1)
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->smu);
    ctx->chunk_subsets = chunk_subsets;
    ctx->oldest_share = oldest_share;
    ctx->max_queue = max_queue;
    return TOR_OK;
}

// ---- autotuning ---------------------------------------------------------------

int tor_autotune(tor_ctx *ctx, int n_min, int n_max, unsigned paths)
{
    if (!ctx || n_min < 1 || n_max > ctx->opt.max_n || n_min > n_max || (paths & ~7u) || !paths)
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    const unsigned bit[NPATH] = {TOR_TUNE_COMPLEX, TOR_TUNE_REAL, TOR_TUNE_QUAD};
    for (int path : {PATH_REAL, PATH_CPLX, PATH_QUAD}) {
        if (!(paths & bit[path]))
            continue;
        for (int n = n_min; n <= n_max; n++) {
            TuneEntry best;
            int rc = tune_one(ctx, path, n, best);
            if (rc != TOR_OK)
                return rc;
            const int N = std::max(n, path_R(path));
            ctx->tune[path][std::min(N, MAX_N)] = best;
        }
    }
    return TOR_OK;
}

int tor_tune_save(tor_ctx *ctx, const char *path)
{
    if (!ctx || !path)
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    FILE *f = std::fopen(path, "w");
    if (!f)
        return TOR_E_INVAL;
    std::fprintf(f, "{\"arch\": \"%s\", \"cus\": %d, \"entries\": [", ctx->arch.c_str(), ctx->num_cu);
    bool first = true;
    for (int path = 0; path < NPATH; path++)
        for (int N = 0; N <= MAX_N; N++) {
            const TuneEntry &t = ctx->tune[path][N];
            if (!t.valid)
                continue;
            std::fprintf(f, "%s\n  {\"path\": \"%s\", \"modes\": %d, \"k\": %d, \"waves_per_cu\": %d, \"ms\": %.4f}",
                         first ? "" : ",", path_name(path), N, t.k, t.waves, (double)t.ms);
            first = false;
        }
    std::fprintf(f, "\n]}\n");
    std::fclose(f);
    return TOR_OK;
}

int tor_tune_load(tor_ctx *ctx, const char *path)
{
    if (!ctx || !path)
        return TOR_E_INVAL;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return TOR_E_INVAL;
    std::string txt;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0)
        txt.append(buf, got);
    std::fclose(f);
    // entries written by tor_tune_save; the cache is only taken for the same
    // architecture and CU count
    char arch[64] = {0};
    int cus = 0;
    const char *a = std::strstr(txt.c_str(), "\"arch\": \"");
    const char *c = std::strstr(txt.c_str(), "\"cus\": ");
    if (!a || !c || std::sscanf(a + 9, "%63[^\"]", arch) != 1 || std::sscanf(c + 7, "%d", &cus) != 1)
        return TOR_E_INVAL;
    if (ctx->arch != arch || cus != ctx->num_cu)
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    const char *p = txt.c_str();
    while ((p = std::strstr(p, "{\"path\": \"")) != nullptr) {
        char kind[16] = {0};
        int N = 0, k = 0, w = 0;
        double ms = 0.0;
        if (std::sscanf(p, "{\"path\": \"%15[^\"]\", \"modes\": %d, \"k\": %d, \"waves_per_cu\": %d, \"ms\": %lf}",
                        kind, &N, &k, &w, &ms) != 5)
            return TOR_E_INVAL;
        if (N < 0 || N > MAX_N || k < 0 || w < 1 || w > 16)
            return TOR_E_INVAL;
        int path = -1;
        for (int q = 0; q < NPATH; q++)
            if (std::strcmp(kind, path_name(q)) == 0)
                path = q;
        if (path < 0)
            return TOR_E_INVAL;
        ctx->tune[path][N] = TuneEntry{true, k, w, (float)ms};
        ++p;
    }
    return TOR_OK;
}

}  // extern "C"
