// tor_runtime.cpp -- host runtime and C ABI of libtor (see include/tor.h).
//
// Host side of one evaluation:
//   1. validate the arguments and every value of the lower triangle;
//   2. form I - O from its lower triangle (Hermitian completion) and run one
//      FP64 Cholesky of the full matrix: positive definiteness of I - O
//      implies it for every principal submatrix (Cauchy interlacing), so
//      this single check covers all 2^n subsets;
//   3. pack the matrix in the device layout (mode-interleaved, reversed,
//      lower-packed; see tor_device.hpp), padded to the kernel's minimum size
//      with decoupled modes of (I - O) block I/2 -- such a mode multiplies
//      the Torontonian by 1/sqrt(1/4) - 1 = 1 exactly;
//   4. one persistent launch over all (matrix, subtree root) items, then the
//      fixed-order per-matrix reduction, one device-to-host copy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/tor.h"
#include "tor_internal.hpp"

using namespace tor;

namespace {

constexpr double kU = 1.1102230246251565e-16;  // FP64 unit roundoff

struct Staged {
    int n = 0;        // modes of the input
    int N = 0;        // modes after padding (complex path)
    std::vector<c64> packed;
    bool real = false;            // Gaussian-state structure found: real path
    int Nr = 0;                   // modes after padding (real path)
    std::vector<double> packed_r; // real symmetric form, same layout
    int status = TOR_OK;
};

struct Request {
    unsigned long long ticket;
    Staged st;
    tor_result res;
    bool done = false;
    std::chrono::steady_clock::time_point t_submit;
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
    int waves_per_cu = 4;
    int grid = 0;    // complex-path persistent grid
    int grid_r = 0;  // real-path persistent grid
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::mutex mu;  // serialises device work on this context

    // serving
    std::mutex smu;
    std::condition_variable scv;
    std::deque<Request *> pending;
    std::unordered_map<unsigned long long, Request *> live;
    unsigned long long next_ticket = 1;
    std::thread worker;
    bool stop = false;
    int inflight = 0;
    int max_queue = 65536;
};

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? TOR_OK : (e == hipErrorOutOfMemory ? TOR_E_NOMEM : TOR_E_DEVICE); }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Cholesky of the Hermitian 2n x 2n matrix C (full storage), FP64.
bool hpd_check(int n2, const std::vector<double> &C)
{
    std::vector<double> L((size_t)n2 * n2 * 2, 0.0);
    for (int i = 0; i < n2; i++) {
        for (int j = 0; j <= i; j++) {
            double sr = C[2 * ((size_t)i * n2 + j)], si = C[2 * ((size_t)i * n2 + j) + 1];
            for (int k = 0; k < j; k++) {
                double ar = L[2 * ((size_t)i * n2 + k)], ai = L[2 * ((size_t)i * n2 + k) + 1];
                double br = L[2 * ((size_t)j * n2 + k)], bi = L[2 * ((size_t)j * n2 + k) + 1];
                sr -= ar * br + ai * bi;
                si -= ai * br - ar * bi;
            }
            if (i == j) {
                if (!(sr > 0.0))
                    return false;
                L[2 * ((size_t)i * n2 + i)] = std::sqrt(sr);
            } else {
                double d = L[2 * ((size_t)j * n2 + j)];
                L[2 * ((size_t)i * n2 + j)] = sr / d;
                L[2 * ((size_t)i * n2 + j) + 1] = si / d;
            }
        }
    }
    return true;
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
// Q <- (Q + Q^T)/2) before the transform.
void stage_real(int n, const std::vector<double> &C, Staged &st)
{
    const int n2 = 2 * n;
    auto cre = [&](int a, int b) { return C[2 * ((size_t)a * n2 + b)]; };
    auto cim = [&](int a, int b) { return C[2 * ((size_t)a * n2 + b) + 1]; };
    double cmax = 0.0, dev = 0.0;
    for (int a = 0; a < n2; a++)
        for (int b = 0; b < n2; b++)
            cmax = std::max(cmax, std::hypot(cre(a, b), cim(a, b)));
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            // lower-right block = conj(upper-left); lower-left block symmetric
            dev = std::max(dev, std::hypot(cre(i + n, j + n) - cre(i, j), cim(i + n, j + n) + cim(i, j)));
            dev = std::max(dev, std::hypot(cre(i + n, j) - cre(j + n, i), cim(i + n, j) - cim(j + n, i)));
        }
    if (!(dev <= 64.0 * kU * std::max(cmax, 1.0)))
        return;
    const int N = std::max(n, REAL_R);
    st.Nr = N;
    st.packed_r.assign((size_t)NSZ(N), 0.0);
    // real 2x2 block of modes (mi, mj), row component ci, column component cj
    auto rblk = [&](int mi, int mj, int ci, int cj) -> double {
        if (mi >= n || mj >= n)
            return (mi == mj && ci == cj) ? 0.5 : 0.0;
        const double pr = 0.5 * (cre(mi, mj) + cre(mi + n, mj + n));
        const double pi = 0.5 * (cim(mi, mj) - cim(mi + n, mj + n));
        // Q = upper-right block, symmetrised: (Q + Q^T)/2, with Q[i][j] = C[i][j+n]
        const double qr = 0.5 * (cre(mi, mj + n) + cre(mj, mi + n));
        const double qi = 0.5 * (cim(mi, mj + n) + cim(mj, mi + n));
        if (ci == 0 && cj == 0) return pr + qr;
        if (ci == 0 && cj == 1) return qi - pi;
        if (ci == 1 && cj == 0) return pi + qi;
        return pr - qr;
    };
    for (int a = 0; a < N; a++)
        for (int b = 0; b <= a; b++)
            for (int e = 0; e < 4; e++) {
                const int qi = 2 * N - 1 - (2 * a + (e >> 1)), qj = 2 * N - 1 - (2 * b + (e & 1));
                st.packed_r[(size_t)4 * bidx(a, b) + e] = rblk(qi / 2, qj / 2, qi % 2, qj % 2);
            }
    st.real = true;
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
    for (int a = 0; a < n2; a++)
        for (int b = 0; b <= a; b++) {
            double orr = O[2 * ((size_t)a * ld + b)], oi = O[2 * ((size_t)a * ld + b) + 1];
            if (!std::isfinite(orr) || !std::isfinite(oi))
                return TOR_E_INVAL;
            double cr = (a == b ? 1.0 : 0.0) - orr;
            double ci = (a == b) ? 0.0 : -oi;
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
    if (n > 0 && !hpd_check(n2, C))
        return TOR_E_NOT_PD;
    // pack: N modes, reversed interleaved rows; row q (interleaved) of mode q/2,
    // component q%2 -> block-order row (q/2) + (q%2) n; modes >= n are padding
    const int N = std::max(n, min_modes);
    st.N = N;
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
                st.packed[(size_t)4 * bidx(a, b) + e] = v;
            }
    st.real = false;
    if (!(flags & TOR_FORCE_COMPLEX) && n > 0)
        stage_real(n, C, st);
    return TOR_OK;
}

struct LaunchPlan {
    std::vector<int> order;  // problem index (input order) for each launch slot
    std::vector<ProblemDesc> probs;
    std::vector<size_t> c_off;
    long long total_items = 0;
    long long max_scratch_entries = 0;
    size_t bytes_C = 0;
};

int path_R(bool real) { return real ? REAL_R : CPLX_R; }
int path_grid(const tor_ctx *ctx, bool real) { return real ? ctx->grid_r : ctx->grid; }
int modes_of(const Staged &m, bool real) { return real ? m.Nr : m.N; }

// split depth: about four subtree roots per persistent wave, never deeper than
// the levels above the last R modes
int choose_k(const tor_ctx *ctx, int N, bool real)
{
    const int LA = N - path_R(real);
    if (LA <= 0)
        return 0;
    if (ctx->opt.split_k > 0)
        return std::min(ctx->opt.split_k, LA);
    int g = 1;
    while ((1 << g) < path_grid(ctx, real))
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

// Run the recursive path over already staged matrices that all take the same
// path.  results: 4 doubles per matrix (input order).  slots_out (optional)
// receives the raw slots.
int run_recursive(tor_ctx *ctx, bool real, std::vector<Staged *> &mats, std::vector<int> &ks,
                  std::vector<double> &results, float *ms, std::vector<double> *slots_out)
{
    const int R = path_R(real);
    const size_t esz = real ? sizeof(double) : sizeof(c64);
    const int grid = path_grid(ctx, real);
    const int count = (int)mats.size();
    LaunchPlan plan;
    plan.order.resize(count);
    for (int i = 0; i < count; i++)
        plan.order[i] = i;
    std::stable_sort(plan.order.begin(), plan.order.end(),
                     [&](int a, int b) { return modes_of(*mats[a], real) > modes_of(*mats[b], real); });
    size_t off = 0;
    for (int s = 0; s < count; s++) {
        Staged *m = mats[plan.order[s]];
        ProblemDesc d{};
        d.N = modes_of(*m, real);
        d.k = ks[plan.order[s]];
        d.item_begin = plan.total_items;
        plan.total_items += 1ll << d.k;
        plan.c_off.push_back(off);
        off = align_up(off + esz * (size_t)NSZ(d.N), 256);
        plan.probs.push_back(d);
        long long se = Gsum(d.N - 1) - Gsum(R - 1);
        plan.max_scratch_entries = std::max(plan.max_scratch_entries, se);
    }
    plan.bytes_C = off;
    const size_t b_probs = align_up(sizeof(ProblemDesc) * count, 256);
    const size_t b_counter = 256;
    const size_t b_slots = align_up(sizeof(double) * 4 * (size_t)plan.total_items, 256);
    const size_t b_res = align_up(sizeof(double) * 4 * (size_t)count, 256);
    const long long stride = (long long)align_up(esz * (size_t)std::max(plan.max_scratch_entries, 1ll), 256);
    const size_t b_scr = (size_t)stride * grid;
    const size_t total = plan.bytes_C + b_probs + b_counter + b_slots + b_res + b_scr;
    int rc = ensure_ws(ctx, total);
    if (rc != TOR_OK)
        return rc;
    char *base = ctx->ws;
    char *dC = base;
    ProblemDesc *dProbs = (ProblemDesc *)(dC + plan.bytes_C);
    unsigned long long *dCounter = (unsigned long long *)((char *)dProbs + b_probs);
    double *dSlots = (double *)((char *)dCounter + b_counter);
    double *dRes = (double *)((char *)dSlots + b_slots);
    char *dScr = (char *)dRes + b_res;

    // host staging buffer for C and descriptors
    std::vector<char> hbuf(plan.bytes_C + b_probs, 0);
    for (int s = 0; s < count; s++) {
        Staged *m = mats[plan.order[s]];
        if (real)
            std::memcpy(hbuf.data() + plan.c_off[s], m->packed_r.data(), esz * m->packed_r.size());
        else
            std::memcpy(hbuf.data() + plan.c_off[s], m->packed.data(), esz * m->packed.size());
        plan.probs[s].C = dC + plan.c_off[s];
    }
    std::memcpy(hbuf.data() + plan.bytes_C, plan.probs.data(), sizeof(ProblemDesc) * count);

    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dC, hbuf.data(), hbuf.size(), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = launch_zero(dCounter, 1, ctx->stream);
    MainParams mp{};
    mp.probs = dProbs;
    mp.nprob = count;
    mp.total_items = plan.total_items;
    mp.counter = dCounter;
    mp.slots = dSlots;
    mp.scratch = dScr;
    mp.scratch_stride = stride;
    const bool dd = ctx->opt.accum != TOR_ACCUM_FP64;
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev0, ctx->stream);
    if (e == hipSuccess)
        e = launch_main(real, dd, mp, grid, ctx->stream);
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev1, ctx->stream);  // device_ms: the main kernel alone
    if (e == hipSuccess)
        e = launch_reduce(dProbs, count, dSlots, dRes, dd, ctx->stream);
    std::vector<double> hres(4 * (size_t)count);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hres.data(), dRes, sizeof(double) * 4 * count, hipMemcpyDeviceToHost, ctx->stream);
    if (slots_out && e == hipSuccess) {
        slots_out->resize(4 * (size_t)plan.total_items);
        e = hipMemcpyAsync(slots_out->data(), dSlots, sizeof(double) * 4 * plan.total_items,
                           hipMemcpyDeviceToHost, ctx->stream);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess)
        return hip_status(e);
    if (ms)
        (void)hipEventElapsedTime(ms, ctx->ev0, ctx->ev1);
    results.assign(4 * (size_t)count, 0.0);
    for (int s = 0; s < count; s++)
        for (int j = 0; j < 4; j++)
            results[4 * (size_t)plan.order[s] + j] = hres[4 * (size_t)s + j];
    return TOR_OK;
}

void fill_result(const Staged &st, bool real, const double *r, float ms, tor_result *out)
{
    std::memset(out, 0, sizeof(*out));
    out->tor = r[0];
    out->tor_lo = r[1];
    out->sum_abs = r[2];
    const double v = std::fabs(r[0] + r[1]);
    // each term carries a relative rounding error of a few units of roundoff
    // per factorisation step; independent errors add in quadrature
    const double R = v > 0.0 ? r[2] / v : INFINITY;
    out->err_est = kU * (double)std::max(st.n, 1) * R / std::sqrt(std::ldexp(1.0, st.n));
    out->subsets = 1ull << st.n;
    out->status = (r[3] != 0.0 || !std::isfinite(r[0])) ? TOR_E_NUMERIC : TOR_OK;
    out->path = real ? 1 : 2;
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

// Launch the staged matrices, one launch per arithmetic path.  done[j] and
// out[idx[j]] are filled for every staged matrix.
int run_staged(tor_ctx *ctx, std::vector<Staged *> &mats, const std::vector<int> &idx, int fixed_k,
               tor_result *out, std::vector<double> *slots_out, int *k_out)
{
    int first_err = TOR_OK;
    for (int pass = 0; pass < 2; pass++) {
        const bool real = pass == 0;
        std::vector<Staged *> grp;
        std::vector<int> gidx, ks;
        for (size_t j = 0; j < mats.size(); j++)
            if (mats[j]->real == real) {
                grp.push_back(mats[j]);
                gidx.push_back(idx[j]);
                const int N = modes_of(*mats[j], real);
                ks.push_back(fixed_k >= 0 ? std::min(fixed_k, std::max(N - path_R(real), 0)) : choose_k(ctx, N, real));
            }
        if (grp.empty())
            continue;
        std::vector<double> res;
        float ms = 0.f;
        int rc = run_recursive(ctx, real, grp, ks, res, &ms, slots_out);
        if (rc != TOR_OK)
            return rc;
        for (size_t j = 0; j < grp.size(); j++) {
            fill_result(*grp[j], real, &res[4 * j], ms, &out[gidx[j]]);
            if (out[gidx[j]].status != TOR_OK && first_err == TOR_OK)
                first_err = out[gidx[j]].status;
        }
        if (k_out)
            *k_out = ks[0];
    }
    return first_err;
}

int eval_many(tor_ctx *ctx, int count, const int *n, const double *const *O, const long *ld, tor_result *out,
              int fixed_k, std::vector<double> *slots_out, int *k_out)
{
    std::vector<Staged> st(count);
    std::vector<Staged *> ok;
    std::vector<int> idx;
    int first_err = TOR_OK;
    for (int i = 0; i < count; i++) {
        if (n[i] > ctx->opt.max_n) {
            out[i] = tor_result{};
            out[i].status = TOR_E_INVAL;
            if (first_err == TOR_OK)
                first_err = TOR_E_INVAL;
            continue;
        }
        std::vector<double> tmp;
        const double *host;
        int rc = copy_input_to_host(n[i], O ? O[i] : nullptr, ld ? ld[i] : 0, ctx->opt.flags, tmp, host);
        if (rc == TOR_OK)
            rc = stage_matrix(n[i], host, ld ? ld[i] : 0, ctx->opt.flags, CPLX_R, st[i]);
        if (rc != TOR_OK) {
            out[i] = tor_result{};
            out[i].status = rc;
            if (first_err == TOR_OK)
                first_err = rc;
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

void serve_loop(tor_ctx *ctx);

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
    const int N = std::max(max_n, CPLX_R);
    const int k = split_k > 0 ? split_k : 14;
    const long long items = (1ll << std::min(k, std::max(N - CPLX_R, 0))) * std::max(max_inflight, 1);
    const size_t grid = 256 * 8;
    const size_t scr = align_up(sizeof(c64) * (size_t)std::max(Gsum(N - 1) - Gsum(CPLX_R - 1), 1ll), 256) * grid;
    return align_up(sizeof(c64) * (size_t)NSZ(N), 256) * std::max(max_inflight, 1) + 4096 * (size_t)std::max(max_inflight, 1) +
           256 + align_up(32 * (size_t)items, 256) + scr + (1 << 20);
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
    if (o.max_n > MAX_N || o.split_k < 0 || o.split_k > 40 || o.waves_per_cu < 0 || o.waves_per_cu > 16)
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
    // persistent grid: as many one-wave workgroups per CU as the LDS allows
    for (int real = 0; real < 2; real++) {
        const int lds = main_lds_bytes(real != 0);
        int fit = (int)(prop.maxSharedMemoryPerMultiProcessor / (size_t)std::max(lds, 1));
        fit = std::max(1, std::min(fit, 8));
        const int w = o.waves_per_cu > 0 ? o.waves_per_cu : fit;
        (real ? ctx->grid_r : ctx->grid) = ctx->num_cu * w;
        if (!real)
            ctx->waves_per_cu = w;
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
        ctx->worker.join();
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        (void)hipSetDevice(ctx->device);
        if (ctx->stream)
            (void)hipStreamSynchronize(ctx->stream);
        if (ctx->own_ws && ctx->ws)
            (void)hipFree(ctx->ws);
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
    int rc = eval_many(ctx, 1, ns, Op, lds, &r, -1, nullptr, nullptr);
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
    return eval_many(ctx, count, n, O, ld, out, -1, nullptr, nullptr);
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
    int rc = eval_many(ctx, 1, ns, Op, lds, &r, k_max, &slots, &k);
    if (rc != TOR_OK && rc != TOR_E_NUMERIC)
        return rc;
    *out = r;
    *k_out = k;
    for (long long i = 0; i < (1ll << k); i++)
        for (int j = 0; j < 3; j++)
            partials[3 * i + j] = slots[4 * i + j];
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
    if (rc == TOR_OK)
        rc = stage_matrix(n, host, ld, ctx->opt.flags, 0, st);
    if (rc != TOR_OK)
        return rc;
    const int chunk = 16;
    const size_t bC = align_up(sizeof(c64) * st.packed.size(), 256);
    const size_t bParts = align_up(sizeof(double) * 4 * ctx->grid, 256);
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
        e = launch_plain(pp, ctx->grid, ctx->stream);
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev1, ctx->stream);
    if (e == hipSuccess)
        e = launch_plain_reduce(dParts, ctx->grid, dRes, ctx->stream);
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
    fill_result(st, false, h, ms, out);
    out->subsets = mask_end - mask_begin;
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
    r->t_submit = std::chrono::steady_clock::now();
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
    auto pred = [&] { return ctx->pending.empty() && ctx->inflight == 0; };
    if (timeout_ms < 0) {
        ctx->scv.wait(lk, pred);
        return TOR_OK;
    }
    return ctx->scv.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred) ? TOR_OK : TOR_E_TIMEOUT;
}

}  // extern "C"

namespace {

// Continuous batching at launch granularity: whatever is pending when the
// device becomes free goes into the next persistent launch; requests that
// arrive meanwhile wait for the launch after it.
void serve_loop(tor_ctx *ctx)
{
    for (;;) {
        std::vector<Request *> batch;
        {
            std::unique_lock<std::mutex> lk(ctx->smu);
            ctx->scv.wait(lk, [&] { return ctx->stop || !ctx->pending.empty(); });
            if (ctx->pending.empty() && ctx->stop)
                return;
            while (!ctx->pending.empty()) {
                batch.push_back(ctx->pending.front());
                ctx->pending.pop_front();
            }
            ctx->inflight += (int)batch.size();
        }
        std::vector<Staged *> mats;
        std::vector<int> idx;
        std::vector<tor_result> res(batch.size());
        for (size_t i = 0; i < batch.size(); i++) {
            mats.push_back(&batch[i]->st);
            idx.push_back((int)i);
        }
        int rc;
        {
            std::lock_guard<std::mutex> g(ctx->mu);
            rc = run_staged(ctx, mats, idx, -1, res.data(), nullptr, nullptr);
        }
        {
            std::lock_guard<std::mutex> g(ctx->smu);
            for (size_t i = 0; i < batch.size(); i++) {
                Request *r = batch[i];
                if (rc == TOR_OK || rc == TOR_E_NUMERIC) {
                    r->res = res[i];
                } else {
                    r->res = tor_result{};
                    r->res.status = rc;
                }
                r->done = true;
            }
            ctx->inflight -= (int)batch.size();
        }
        ctx->scv.notify_all();
    }
}

}  // namespace
