// tor_runtime.cpp -- host runtime and C ABI of libtor (see include/tor.h).
//
// One evaluation:
//   1. the host checks the arguments (sizes, pointers, leading dimensions);
//   2. a host input is copied to the device as it is (a device input is read
//      in place); the staging kernel (tor_stage.hip) validates every value,
//      forms I - O from its lower triangle, tests the Gaussian-state
//      structure and packs the matrix in the layout of its path, straight
//      into the workspace; the host reads back only the path and status;
//   3. one persistent launch over all (matrix, subtree root) items, then the
//      fixed-order per-matrix reduction of the root slots, one copy back.
//      Positive definiteness is the kernel's own test: it checks the pivots
//      of every subset, I - O itself among them, and a failed pivot is
//      reported as TOR_E_NOT_PD.
//
// Serving (tor_submit / tor_poll) keeps each admitted request's matrix and
// root slots in a device pool and runs them in chunked launches: every launch
// takes a bounded number of subsets from the admitted requests, smallest
// remaining work first, so requests that arrive while others run join the
// next launch instead of waiting for the longest one to finish.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

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
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/tor.h"
#include "tor_internal.hpp"

using namespace tor;

namespace {

constexpr double kU = 1.1102230246251565e-16;  // FP64 unit roundoff
constexpr double kUdd = 1.9721522630525295e-31; // 2^-102: a few units of 2^-104 per double-double step

// A matrix staged on the device: its form lives in the workspace at ws_off,
// or at pool (serving).
struct Mat {
    int n = 0;             // modes of the input
    int N = 0;             // modes of the staged form (padded to the path's minimum)
    int path = PATH_CPLX;  // PATH_REAL when the Gaussian-state structure is found
    int status = TOR_OK;
    size_t ws_off = 0;
    char *pool = nullptr;
};

struct Request {
    unsigned long long ticket = 0;
    int n = 0;
    std::vector<double> raw;  // the input, 2n x 2n complex128, compact rows
    Mat st;
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
    int launches = 0;       // serving launches that ran part of it
    int flights = 0;            // serving launches in flight that hold some of its roots
    bool quick_flight = false;  // one of them is an express launch
    bool failed = false;        // a launch of it failed: retired with that status
};

// Serving policy (tor_serve_config).  Written under the serving lock; the
// scheduler takes a copy under the same lock before each round.
struct ServeCfg {
    long long chunk_subsets = 1ll << 30;   // work per chunked serving launch
    long long express_subsets = 1ll << 24; // requests this small run ahead, whole (0: none)
    double oldest_share = 0.5;             // of a chunk, guaranteed to the oldest request
};

// A set of launch resources of its own: serving runs its launches on two
// of these.  `stream` is limited by a CU mask to `cus` CUs (0: no mask could
// be set, and it runs on every CU); `side`, when made, has the same mask
// (serving stages requests there, beside the lane's launches); `wide`, when
// made, runs on every CU; `cur` is the one the lane's current launch goes to.
// Two slots of pinned buffers and events let a second launch be queued on
// the lane's stream behind the one running (both share the workspace, which
// the second launch's first copy rewrites only after the first launch's
// last copy, in stream order); `slot` is the one the next launch uses.
struct LaunchLane {
    hipStream_t stream = nullptr, side = nullptr, wide = nullptr, cur = nullptr;
    int cus = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int slot = 0;
    char *hup[2] = {}, *hdown[2] = {};
    size_t hup_bytes[2] = {}, hdown_bytes[2] = {};
    hipEvent_t ev0[2] = {}, ev1[2] = {}, done[2] = {};
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
    // pinned host staging for uploads and read-backs (grown on demand)
    char *hup = nullptr, *hdown = nullptr;
    size_t hup_bytes = 0, hdown_bytes = 0;
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
    ServeCfg serve;  // guarded by smu
    // debug (tor_debug_fail_root): root dbg_root of the next synchronous
    // evaluation's first matrix reports a numeric failure in its first
    // dbg_runs launches
    long long dbg_root = -1;
    int dbg_runs = 0;
    char *pool = nullptr;
    size_t pool_bytes = 256ull << 20;
    std::map<size_t, size_t> pool_free;  // offset -> length
    LaunchLane chunk;  // serving's chunked launches (created on first use)
    LaunchLane quick;  // serving's express launches (created on first use)
};

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? TOR_OK : (e == hipErrorOutOfMemory ? TOR_E_NOMEM : TOR_E_DEVICE); }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int path_R(int path) { return path == PATH_QUAD ? QUAD_R : path == PATH_REAL ? REAL_R : CPLX_R; }
// bytes per scalar of the device layout (c64 and ddr are both 16)
size_t path_esz(int path) { return path == PATH_REAL ? sizeof(double) : sizeof(c64); }
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
    // Every root first recomputes its k eliminations in global memory, which a
    // short root does not amortise, so no more roots than leave each about
    // 64 tier-A leaves on the real path (k <= LA - 6) and 32 on the 16-byte
    // paths (k <= LA - 5), within [g, g + 2] on the real path (one to four
    // roots per wave of the 2^g grid) and [g - 1, g + 3] on the 16-byte
    // paths, whose leaves are a quarter the size and whose launches end more
    // evenly with more roots.  The autotuner's picks this follows:
    // real n = 26 k = 11 (0.26 ms against 0.34 at k = 13), n = 30 k = 13;
    // complex n = 24 k = 10 (0.26 against 0.33 at 13), n = 30 k = 14 (10.1
    // against 10.9 at 13); double-double n = 30 k = 14 (24.1 against 24.9).
    const int lo = path == PATH_REAL ? g : g - 1;
    const int hi = path == PATH_REAL ? g + 2 : g + 3;
    // real path, LA from g - 1 to g + 2 (n = 21..24 on the 2048-wave grid):
    // the grid cannot be filled with roots of many leaves, and one leaf per
    // root leaves each wave's root set-up unshared; roots of two to eight
    // leaves at g - 1 measured fastest (n = 22: 0.052 ms against 0.079 at
    // k = g = LA, n = 23: 0.069 against 0.078)
    if (path == PATH_REAL && LA >= g - 1 && LA <= g + 2)
        return std::min(LA - 1, g - 1);
    // the 16-byte paths' leaves are a quarter the size: 32 leaves per root
    // (n = 26: complex 0.73 ms against 0.83 with 64, double-double 1.85
    // against 2.07; n = 27 double-double 3.23 against 3.64)
    const int leaves = path == PATH_REAL ? 6 : 5;
    const int k = std::min(LA, std::max(lo, std::min(hi, LA - leaves)));
    // real path: two roots per wave end the launch worst (the two waves of a
    // SIMD run at different speeds, and the faster ones run dry with half
    // their share left to the others): n = 29 1.61 ms at k = g + 1 against
    // 1.37 at g + 2, n = 28 0.84 against 0.73
    if (path == PATH_REAL && k == g + 1)
        return std::min(LA, g + 2);
    return k;
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

// Grow the workspace to at least bytes, keeping its first `keep` bytes.
int ensure_ws_keep(tor_ctx *ctx, size_t bytes, size_t keep)
{
    if (bytes <= ctx->ws_bytes)
        return TOR_OK;
    if (!ctx->own_ws)
        return TOR_E_NOMEM;
    const size_t want = align_up(bytes + (bytes >> 3), 1 << 20);
    char *nw = nullptr;
    if (hipMalloc((void **)&nw, want) != hipSuccess)
        return TOR_E_NOMEM;
    hipError_t e = hipSuccess;
    if (ctx->ws && keep > 0)
        e = hipMemcpyAsync(nw, ctx->ws, keep, hipMemcpyDeviceToDevice, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(nw);
        return hip_status(e);
    }
    if (ctx->ws)
        (void)hipFree(ctx->ws);
    ctx->ws = nw;
    ctx->ws_bytes = want;
    return TOR_OK;
}

// Pinned host buffer of at least need bytes.  Only grown between
// synchronised calls, so no copy is in flight from the old one.
int pin_grow(char *&buf, size_t &cap, size_t need)
{
    if (need <= cap)
        return TOR_OK;
    if (buf)
        (void)hipHostFree(buf);
    buf = nullptr;
    cap = 0;
    const size_t want = align_up(std::max(need + (need >> 2), (size_t)1 << 16), 4096);
    if (hipHostMalloc((void **)&buf, want, hipHostMallocDefault) != hipSuccess) {
        buf = nullptr;
        return TOR_E_NOMEM;
    }
    cap = want;
    return TOR_OK;
}

const char *mat_ptr(const tor_ctx *ctx, const Mat &m) { return m.pool ? m.pool : ctx->ws + m.ws_off; }

unsigned stage_flags(unsigned api_flags)
{
    return ((api_flags & TOR_CHECK_HERMITIAN) ? STAGE_CHECK_HERM : 0u) |
           ((api_flags & TOR_FORCE_COMPLEX) ? STAGE_FORCE_CPLX : 0u) | ((api_flags & TOR_FACTOR_DD) ? STAGE_DD : 0u);
}

// Device bytes of the staged form of an n-mode matrix: the largest form the
// staging kernel may choose under these flags.
size_t staged_bytes(int n, unsigned sflags, int min_cplx)
{
    if (sflags & STAGE_INTERLEAVED)
        return sizeof(c64) * (size_t)E(std::max(n, 1));
    if (sflags & STAGE_DD)
        return sizeof(ddr) * (size_t)NSZ(std::max(n, QUAD_R));
    size_t b = sizeof(c64) * (size_t)NSZ(std::max(n, min_cplx));
    if (!(sflags & STAGE_FORCE_CPLX))
        b = std::max(b, sizeof(double) * (size_t)NSZ(std::max(n, REAL_R)));
    return b;
}

// One matrix to stage: n modes of O (host or device memory, leading
// dimension ld in complex elements); with sel (host, n increasing modes) the
// principal submatrix of an M-mode O on rows {s, s + M}.  dst: where the
// staged form goes when not in the workspace (the serving pool).
struct StageIn {
    int n = 0;
    const double *O = nullptr;
    long ld = 0;
    const int *sel = nullptr;
    int M = 0;
    char *dst = nullptr;
};

// Enqueue one staging launch for in[0..count) on the context's stream: the
// descriptors, the pattern lists and (for host inputs) the raw matrices go
// up in one copy into the workspace from byte base on; the staged forms
// follow them.  The kernel's status records are copied back into ctx->hdown
// (StageInfo each, from byte 0); *end receives the first workspace byte
// after the staging area and *down_end the first free byte of ctx->hdown.
// stage_collect reads them after the stream has been synchronised.
// Workspace layout of a staging launch (offsets from its base).  A host
// matrix given several times (the same pointer, leading dimension and size,
// as for click patterns) is uploaded once: raw_first[i] is set for the input
// that carries each distinct copy.
struct StageLayout {
    size_t b_desc = 0, b_info = 0, b_sel = 0, b_raw = 0, up_bytes = 0, total = 0;
    std::vector<size_t> raw_off, out_off;
    std::vector<char> raw_first;
};

StageLayout stage_layout(const std::vector<StageIn> &in, bool on_device, unsigned sflags, int min_cplx)
{
    const int count = (int)in.size();
    StageLayout L;
    L.b_desc = align_up(sizeof(StageDesc) * count, 256);
    L.b_info = align_up(sizeof(StageInfo) * count, 256);
    size_t nsel = 0;
    for (const StageIn &x : in)
        if (x.sel)
            nsel += (size_t)x.n;
    L.b_sel = align_up(sizeof(int) * std::max(nsel, (size_t)1), 256);
    // raw inputs: one compact copy per distinct host matrix
    L.raw_off.assign(count, 0);
    L.raw_first.assign(count, 0);
    std::map<std::tuple<const double *, long, int>, size_t> seen;
    if (!on_device)
        for (int i = 0; i < count; i++) {
            const int rows = 2 * (in[i].sel ? in[i].M : in[i].n);
            if (rows == 0)
                continue;
            const auto key = std::make_tuple(in[i].O, in[i].ld, rows);
            auto it = seen.find(key);
            if (it == seen.end()) {
                it = seen.emplace(key, L.b_raw).first;
                L.raw_first[i] = 1;
                L.b_raw += align_up(sizeof(c64) * (size_t)rows * rows, 256);
            }
            L.raw_off[i] = it->second;
        }
    L.up_bytes = L.b_desc + L.b_info + L.b_sel + L.b_raw;
    size_t out_bytes = 0;
    L.out_off.assign(count, 0);
    for (int i = 0; i < count; i++)
        if (!in[i].dst) {
            L.out_off[i] = L.up_bytes + out_bytes;
            out_bytes += align_up(staged_bytes(in[i].n, sflags, min_cplx), 256);
        }
    L.total = L.up_bytes + out_bytes;
    return L;
}

int stage_enqueue(tor_ctx *ctx, const std::vector<StageIn> &in, bool on_device, unsigned sflags, int min_cplx,
                  size_t base, std::vector<Mat> &mats, size_t *end, size_t *down_end, hipStream_t stream = nullptr)
{
    if (!stream)
        stream = ctx->stream;
    const int count = (int)in.size();
    mats.assign(count, Mat{});
    *end = base;
    *down_end = 0;
    if (count == 0)
        return TOR_OK;
    const StageLayout L = stage_layout(in, on_device, sflags, min_cplx);
    const size_t b_desc = L.b_desc, b_info = L.b_info, b_sel = L.b_sel, up_bytes = L.up_bytes;
    const std::vector<size_t> &raw_off = L.raw_off, &out_off = L.out_off;
    // device inputs that live in the workspace must already fit (growing
    // it would move them)
    int rc = ensure_ws_keep(ctx, base + L.total, base);
    if (rc == TOR_OK)
        rc = pin_grow(ctx->hup, ctx->hup_bytes, up_bytes);
    if (rc == TOR_OK)  // 256 spare bytes for a caller's own read-back
        rc = pin_grow(ctx->hdown, ctx->hdown_bytes, b_info + 256);
    if (rc != TOR_OK)
        return rc;
    char *dbase = ctx->ws + base;
    char *h = ctx->hup;
    StageDesc *hd = (StageDesc *)h;
    int *hsel = (int *)(h + b_desc + b_info);
    size_t sel_at = 0;
    struct RawCopy {
        char *dst;
        const double *src;
        long ld;
        int rows;
    };
    std::vector<RawCopy> copies;
    for (int i = 0; i < count; i++) {
        const StageIn &x = in[i];
        StageDesc d{};
        d.n = x.n;
        d.M = x.sel ? x.M : x.n;
        d.flags = sflags;
        d.min_cplx = min_cplx;
        d.info = (StageInfo *)(dbase + b_desc) + i;
        d.out = x.dst ? (void *)x.dst : (void *)(dbase + out_off[i]);
        if (x.sel) {
            std::memcpy(hsel + sel_at, x.sel, sizeof(int) * (size_t)x.n);
            d.sel = (const int *)(dbase + b_desc + b_info) + sel_at;
            sel_at += (size_t)x.n;
        }
        const int rows = 2 * d.M;
        if (rows > 0 && !on_device) {
            if (L.raw_first[i])
                copies.push_back(RawCopy{h + b_desc + b_info + b_sel + raw_off[i], x.O, x.ld, rows});
            d.O = (const double *)(dbase + b_desc + b_info + b_sel + raw_off[i]);
            d.ld = rows;
        } else {
            d.O = x.O;
            d.ld = x.ld;
        }
        hd[i] = d;
        mats[i].n = x.n;
        mats[i].pool = x.dst;
        mats[i].ws_off = x.dst ? 0 : base + out_off[i];
    }
    // compact the host inputs into the pinned image, on a few threads for a
    // large batch
    auto do_copies = [&](size_t first, size_t step) {
        for (size_t c = first; c < copies.size(); c += step) {
            const RawCopy &rc_ = copies[c];
            for (int r = 0; r < rc_.rows; r++)
                std::memcpy(rc_.dst + sizeof(c64) * (size_t)r * rc_.rows, rc_.src + 2 * (size_t)r * (size_t)rc_.ld,
                            sizeof(c64) * (size_t)rc_.rows);
        }
    };
    const size_t nthr = L.b_raw > ((size_t)4 << 20) && copies.size() >= 16
                            ? std::min<size_t>(8, std::max(1u, std::thread::hardware_concurrency()))
                            : 1;
    if (nthr <= 1) {
        do_copies(0, 1);
    } else {
        std::vector<std::thread> pool;
        for (size_t t = 0; t < nthr; t++)
            pool.emplace_back(do_copies, t, nthr);
        for (auto &th : pool)
            th.join();
    }
    hipError_t e = hipSetDevice(ctx->device);
    // the infos' bytes are part of the copy (their values do not matter)
    if (e == hipSuccess)
        e = hipMemcpyAsync(dbase, h, up_bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = launch_stage((const StageDesc *)dbase, count, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->hdown, dbase + b_desc, sizeof(StageInfo) * count, hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess)
        return hip_status(e);
    *end = base + L.total;
    *down_end = b_info;
    return TOR_OK;
}

// After the stream has been synchronised: each matrix's path, modes and
// status from the staging kernel's records.
void stage_collect(const tor_ctx *ctx, std::vector<Mat> &mats)
{
    const StageInfo *info = (const StageInfo *)ctx->hdown;
    for (size_t i = 0; i < mats.size(); i++) {
        mats[i].status = info[i].status == 0 ? TOR_OK : TOR_E_INVAL;
        mats[i].path = info[i].path;
        mats[i].N = info[i].N;
    }
}

// Stage, wait, collect (on the context's stream unless one is given).
int stage_sync(tor_ctx *ctx, const std::vector<StageIn> &in, bool on_device, unsigned sflags, int min_cplx,
               size_t base, std::vector<Mat> &mats, size_t *end, hipStream_t stream = nullptr)
{
    size_t down_end = 0;
    int rc = stage_enqueue(ctx, in, on_device, sflags, min_cplx, base, mats, end, &down_end, stream);
    if (rc != TOR_OK || in.empty())
        return rc;
    hipError_t e = hipStreamSynchronize(stream ? stream : ctx->stream);
    if (e != hipSuccess)
        return hip_status(e);
    stage_collect(ctx, mats);
    return TOR_OK;
}


// Bytes of one persistent wave's stack for a matrix of N modes split at
// depth k (tslot_off): the root node, the tier-A slots, the determinants.
long long wave_stack_bytes(int path, int N, int k)
{
    const int rsz = path == PATH_QUAD ? (int)sizeof(ddr) : (int)sizeof(double);
    return (long long)align_up((size_t)stack_bytes(N, k, path_R(path), (int)path_esz(path), rsz), 256);
}

// Workspace bytes a launch needs after its matrices and slots: descriptors,
// reduction descriptors, queue counter, results, per-wave stacks (stride:
// the largest wave_stack_bytes of the launch's matrices).
struct LaunchLayout {
    size_t b_probs, b_red, b_counter, b_res;
    long long stride;
    size_t total(int grid) const { return b_probs + b_red + b_counter + b_res + (size_t)stride * grid; }
};

LaunchLayout launch_layout(int count, int nred, long long stride)
{
    LaunchLayout L;
    L.b_probs = align_up(sizeof(ProblemDesc) * std::max(count, 1), 256);
    L.b_red = align_up(sizeof(ProblemDesc) * std::max(nred, 1), 256);
    L.b_counter = 256;
    L.b_res = align_up(sizeof(double) * 4 * std::max(nred, 1), 256);
    L.stride = std::max(stride, 256ll);
    return L;
}

// Workspace of a launch lane: grown (never shrunk) between launches, when
// nothing is in flight on its stream.
int lane_ws(LaunchLane &L, size_t bytes)
{
    if (bytes <= L.ws_bytes)
        return TOR_OK;
    if (L.ws) {
        for (hipStream_t st : {L.stream, L.side, L.wide})
            if (st)
                (void)hipStreamSynchronize(st);
        (void)hipFree(L.ws);
        L.ws = nullptr;
        L.ws_bytes = 0;
    }
    const size_t want = align_up(bytes + (bytes >> 3), 1 << 20);
    if (hipMalloc((void **)&L.ws, want) != hipSuccess) {
        L.ws = nullptr;
        return TOR_E_NOMEM;
    }
    L.ws_bytes = want;
    return TOR_OK;
}

// One persistent launch over the root ranges in descs (C, slots, N, k,
// root_begin, nroots filled in), followed by the reduction of the matrices
// listed in reduce (indices into descs, or none), into results (4 doubles
// each).  The workspace from byte ws_off on holds descriptors, counter,
// results and the per-wave tier-A stacks.  When ws_off > 0 the bytes below it
// hold data the descriptors point to, and the caller has already sized the
// workspace (a reallocation here would move that data).
// With a lane, the launch goes to the lane's current stream, its workspace
// and the pinned buffers of its current slot, and the call returns once it
// is enqueued: the slot's done event follows the read-back of the results,
// which lane_collect then takes.
int run_launch(tor_ctx *ctx, int path, std::vector<ProblemDesc> &descs, const std::vector<int> &reduce,
               size_t ws_off, int grid, std::vector<double> *results, float *ms, long long fail_item1 = 0,
               double *terms = nullptr, LaunchLane *lane = nullptr)
{
    const int count = (int)descs.size();
    long long total = 0, stack = 0;
    for (auto &d : descs) {
        d.item_begin = total;
        total += d.nroots;
        stack = std::max(stack, wave_stack_bytes(path, d.N, d.k));
    }
    std::vector<ProblemDesc> red;
    for (int i : reduce)
        red.push_back(descs[i]);
    const int nred = (int)red.size();
    const LaunchLayout Lo = launch_layout(count, nred, stack);
    const size_t need = ws_off + Lo.total(grid);
    if (ws_off > 0 && need > (lane ? lane->ws_bytes : ctx->ws_bytes))
        return TOR_E_NOMEM;  // the caller sizes the workspace first
    int rc = lane ? lane_ws(*lane, need) : ensure_ws(ctx, need);
    if (rc != TOR_OK)
        return rc;
    const hipStream_t stream = lane ? lane->cur : ctx->stream;
    const int sl = lane ? lane->slot : 0;
    char *&hup = lane ? lane->hup[sl] : ctx->hup;
    char *&hdown = lane ? lane->hdown[sl] : ctx->hdown;
    size_t &hup_bytes = lane ? lane->hup_bytes[sl] : ctx->hup_bytes;
    size_t &hdown_bytes = lane ? lane->hdown_bytes[sl] : ctx->hdown_bytes;
    const hipEvent_t ev0 = lane ? lane->ev0[sl] : ctx->ev0, ev1 = lane ? lane->ev1[sl] : ctx->ev1;
    char *dProbs = (lane ? lane->ws : ctx->ws) + ws_off;
    char *dRed = dProbs + Lo.b_probs;
    unsigned long long *dCounter = (unsigned long long *)(dRed + Lo.b_red);
    double *dRes = (double *)((char *)dCounter + Lo.b_counter);
    char *dScr = (char *)dRes + Lo.b_res;
    const long long stride = Lo.stride;
    // descriptors and reduction descriptors at their exact byte offsets and
    // the zeroed queue counter after them: one copy from pinned memory (the
    // previous use of the buffer has been synchronised)
    const size_t up = Lo.b_probs + Lo.b_red + sizeof(unsigned long long);
    rc = pin_grow(hup, hup_bytes, up);
    if (rc == TOR_OK)
        rc = pin_grow(hdown, hdown_bytes, sizeof(double) * 4 * (size_t)std::max(nred, 1));
    if (rc != TOR_OK)
        return rc;
    std::memset(hup, 0, up);
    std::memcpy(hup, descs.data(), sizeof(ProblemDesc) * count);
    if (nred)
        std::memcpy(hup + Lo.b_probs, red.data(), sizeof(ProblemDesc) * nred);

    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dProbs, hup, up, hipMemcpyHostToDevice, stream);
    MainParams mp{};
    mp.probs = (const ProblemDesc *)dProbs;
    mp.nprob = count;
    mp.total_items = total;
    mp.counter = dCounter;
    mp.scratch = dScr;
    mp.scratch_stride = stride;
    mp.fail_item1 = fail_item1;
    mp.terms = terms;
    // the double-double factor always sums in double-double
    const bool dd = ctx->opt.accum != TOR_ACCUM_FP64 || path == PATH_QUAD;
    if (e == hipSuccess)
        e = hipEventRecord(ev0, stream);
    // no more persistent waves than queue items: a launch of few roots (a
    // small matrix) does not pay for starting the whole grid
    if (e == hipSuccess && total > 0)
        e = terms ? launch_main_store(mp, (int)std::min<long long>(grid, total), stream)
                  : launch_main(path, dd, mp, (int)std::min<long long>(grid, total), stream);
    if (e == hipSuccess)
        e = hipEventRecord(ev1, stream);  // device_ms: the main kernel alone
    const double *hres = (const double *)hdown;
    if (e == hipSuccess && nred > 0) {
        e = launch_reduce((const ProblemDesc *)dRed, nred, dRes, dd, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hdown, dRes, sizeof(double) * 4 * nred, hipMemcpyDeviceToHost, stream);
    }
    if (lane) {
        if (e == hipSuccess)
            e = hipEventRecord(lane->done[sl], stream);
        if (e != hipSuccess)
            (void)hipStreamSynchronize(stream);  // nothing still reads the pinned buffers
        return hip_status(e);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(stream);
    if (e != hipSuccess)
        return hip_status(e);
    if (ms)
        (void)hipEventElapsedTime(ms, ev0, ev1);
    if (results)
        results->assign(hres, hres + 4 * (size_t)nred);
    return TOR_OK;
}

// Results (4 doubles per reduced matrix) and main-kernel time of a lane's
// launch in slot sl, once its done event has been reached.
void lane_collect(const LaunchLane &L, int sl, int nred, std::vector<double> &results, float *ms)
{
    if (ms)
        (void)hipEventElapsedTime(ms, L.ev0[sl], L.ev1[sl]);
    const double *h = (const double *)L.hdown[sl];
    results.assign(h, h + 4 * (size_t)nred);
}

void lane_close(LaunchLane &L)
{
    for (hipStream_t st : {L.stream, L.side, L.wide})
        if (st)
            (void)hipStreamSynchronize(st);
    if (L.ws)
        (void)hipFree(L.ws);
    for (int sl = 0; sl < 2; sl++) {
        if (L.hup[sl])
            (void)hipHostFree(L.hup[sl]);
        if (L.hdown[sl])
            (void)hipHostFree(L.hdown[sl]);
        for (hipEvent_t ev : {L.ev0[sl], L.ev1[sl], L.done[sl]})
            if (ev)
                (void)hipEventDestroy(ev);
    }
    for (hipStream_t st : {L.stream, L.side, L.wide})
        if (st)
            (void)hipStreamDestroy(st);
    L = LaunchLane{};
}

// Streams and events of a lane, made on its first use: `stream` limited to
// the ncu CUs from bit `first` of the device's CU mask on (the runtime spreads
// the mask's bits over the dies), a plain stream if the mask is refused;
// with `side` a second stream of the same mask (only if the mask is set),
// with `wide` a plain stream beside them.  Every stream has the default
// priority.
int lane_open(LaunchLane &L, int num_cu, int first, int ncu, bool side, bool wide)
{
    if (L.stream)
        return TOR_OK;
    uint32_t mask[32] = {};
    const uint32_t words = (uint32_t)((num_cu + 31) / 32);
    hipError_t e = hipErrorInvalidValue;
    if (ncu > 0 && first >= 0 && first + ncu <= num_cu && num_cu <= 1024) {
        for (int c = first; c < first + ncu; c++)
            mask[c / 32] |= 1u << (c % 32);
        e = hipExtStreamCreateWithCUMask(&L.stream, words, mask);
    }
    L.cus = e == hipSuccess ? ncu : 0;
    if (e != hipSuccess && hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess)
        L.stream = nullptr;
    bool ok = L.stream != nullptr;
    if (ok && side && L.cus > 0)
        ok = hipExtStreamCreateWithCUMask(&L.side, words, mask) == hipSuccess;
    if (ok && wide)
        ok = hipStreamCreateWithFlags(&L.wide, hipStreamNonBlocking) == hipSuccess;
    for (int sl = 0; sl < 2; sl++)
        ok = ok && hipEventCreate(&L.ev0[sl]) == hipSuccess && hipEventCreate(&L.ev1[sl]) == hipSuccess &&
             hipEventCreateWithFlags(&L.done[sl], hipEventDisableTiming) == hipSuccess;
    if (ok) {
        L.cur = L.stream;
        return TOR_OK;
    }
    lane_close(L);
    return TOR_E_DEVICE;
}

// Synchronous path: all roots of every staged matrix in one launch, matrices
// with more modes first; their root slots and the launch's own data go into
// the workspace from byte base on.  results: 4 doubles per matrix (input
// order).
int run_recursive(tor_ctx *ctx, int path, std::vector<Mat *> &mats, std::vector<int> &ks,
                  std::vector<double> &results, float *ms, std::vector<double> *slots_out, size_t base,
                  std::vector<int> *launches)
{
    const int count = (int)mats.size();
    std::vector<int> order(count);
    for (int i = 0; i < count; i++)
        order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return mats[a]->N > mats[b]->N; });
    // workspace: slots, then what run_launch needs
    std::vector<size_t> s_off(count);
    long long nslots = 0, stack = 0;
    int Nmax = 0;
    for (int s = 0; s < count; s++) {
        s_off[s] = base + sizeof(double) * 4 * (size_t)nslots;
        nslots += 1ll << ks[order[s]];
        Nmax = std::max(Nmax, mats[order[s]]->N);
        stack = std::max(stack, wave_stack_bytes(path, mats[order[s]]->N, ks[order[s]]));
    }
    const size_t off = align_up(base + sizeof(double) * 4 * (size_t)nslots, 256);
    const int grid = launch_grid(ctx, path, Nmax);
    // size the workspace for everything, keeping the staged matrices below base
    int rc = ensure_ws_keep(ctx, off + launch_layout(count, count, stack).total(grid), base);
    if (rc != TOR_OK)
        return rc;
    std::vector<ProblemDesc> descs(count);
    std::vector<int> red(count);
    for (int s = 0; s < count; s++) {
        const Mat *m = mats[order[s]];
        ProblemDesc &d = descs[s];
        d.C = mat_ptr(ctx, *m);
        d.slots = (double *)(ctx->ws + s_off[s]);
        d.N = m->N;
        d.k = ks[order[s]];
        d.root_begin = 0;
        d.nroots = 1ll << d.k;
        red[s] = s;
    }
    // debug: the queue item of root dbg_root of the first input matrix
    int dbg_s = 0;
    while (order[dbg_s] != 0)
        ++dbg_s;
    long long dbg_item1 = 0;
    const bool use_dbg = launches != nullptr;  // evaluations only, not the autotuner
    if (use_dbg && ctx->dbg_runs > 0 && ctx->dbg_root >= 0 && ctx->dbg_root < descs[dbg_s].nroots) {
        for (int s = 0; s < dbg_s; s++)
            dbg_item1 += descs[s].nroots;
        dbg_item1 += ctx->dbg_root + 1;
    }
    const long long dbg_root = ctx->dbg_root;
    int dbg_runs = dbg_item1 ? ctx->dbg_runs : 0;
    if (use_dbg)
        ctx->dbg_runs = 0;
    std::vector<double> res;
    rc = run_launch(ctx, path, descs, red, off, grid, &res, ms, dbg_item1);
    if (rc != TOR_OK)
        return rc;
    --dbg_runs;
    std::vector<int> runs(count, 1);
    // Recovery: a matrix whose roots report numeric failures and no failed
    // pivot runs the range of its failed roots once more.  Root slots are
    // overwritten, not accumulated, so a root that runs again (or a good one
    // inside the range) leaves exactly the value a clean launch leaves, and
    // the reduction sums the slots in the same fixed order.
    std::vector<int> redo;
    for (int s = 0; s < count; s++)
        if (res[4 * (size_t)s + 3] == SLOT_NUMERIC)
            redo.push_back(s);
    if (!redo.empty()) {
        std::vector<double> hs(4 * (size_t)nslots);
        hipError_t e = hipMemcpy(hs.data(), ctx->ws + s_off[0], sizeof(double) * 4 * nslots, hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            return hip_status(e);
        std::vector<ProblemDesc> rd;
        std::vector<int> rred;
        long long item1 = 0, items = 0;
        for (int s : redo) {
            const long long first = (long long)(s_off[s] - s_off[0]) / (4 * (long long)sizeof(double));
            long long lo = -1, hi = -1;
            for (long long r = 0; r < descs[s].nroots; r++)
                if (hs[4 * (first + r) + 3] == SLOT_NUMERIC) {
                    if (lo < 0)
                        lo = r;
                    hi = r;
                }
            ProblemDesc d = descs[s];
            d.root_begin = lo;
            d.nroots = hi - lo + 1;
            if (s == dbg_s && dbg_runs > 0 && dbg_root >= lo && dbg_root <= hi)
                item1 = items + (dbg_root - lo) + 1;
            items += d.nroots;
            rred.push_back((int)rd.size());
            rd.push_back(d);
        }
        std::vector<double> res2;
        rc = run_launch(ctx, path, rd, rred, off, grid, &res2, nullptr, item1);
        if (rc != TOR_OK)
            return rc;
        for (size_t i = 0; i < redo.size(); i++) {
            for (int j = 0; j < 4; j++)
                res[4 * (size_t)redo[i] + j] = res2[4 * i + j];
            ++runs[redo[i]];
        }
    }
    if (launches) {
        launches->assign(count, 1);
        for (int s = 0; s < count; s++)
            (*launches)[order[s]] = runs[s];
    }
    results.assign(4 * (size_t)count, 0.0);
    for (int s = 0; s < count; s++)
        for (int j = 0; j < 4; j++)
            results[4 * (size_t)order[s] + j] = res[4 * (size_t)s + j];
    if (slots_out) {
        slots_out->resize(4 * (size_t)nslots);
        hipError_t e = hipMemcpy(slots_out->data(), ctx->ws + s_off[0], sizeof(double) * 4 * nslots,
                                 hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            return hip_status(e);
    }
    return TOR_OK;
}

void fill_result(const Mat &st, int path, const double *r, float ms, tor_result *out)
{
    std::memset(out, 0, sizeof(*out));
    out->tor = r[0];
    out->tor_lo = r[1];
    // a padding mode (its block of I - O is I/2) turns each term t into the
    // pair -t, +2t: Tor is unchanged and the padded sum of |t| is 3 times the
    // input's, so it is scaled back (3^pad is exact for pad < 34)
    const int pad = st.N - st.n;
    out->sum_abs = pad > 0 ? r[2] / std::pow(3.0, pad) : r[2];
    const double v = std::fabs(r[0] + r[1]);
    // each term carries a small relative rounding error of either sign,
    // independent between subsets, so the sum's error is about
    // u sqrt(sum t^2), of which R / sqrt(2^n) is the value for terms of equal
    // size; measured against the extended-precision and __float128 oracles
    // (n = 20, 24, 30) the FP64 path's error is 0.1 to 3.5 times
    // u R / sqrt(2^n), so twice that is the typical size
    const double R = v > 0.0 ? out->sum_abs / v : INFINITY;
    const double u = path == PATH_QUAD ? kUdd : kU;
    out->err_est = 2.0 * u * R / std::sqrt(std::ldexp(1.0, st.n));
    out->subsets = 1ull << st.n;
    // a pivot that is not positive in some subset: I - O is not positive
    // definite (the all-include subset is I - O itself)
    out->status = r[3] >= SLOT_NOT_PD ? TOR_E_NOT_PD : (r[3] > 0.0 || !std::isfinite(r[0])) ? TOR_E_NUMERIC : TOR_OK;
    out->path = api_path(path);
    out->device_ms = ms;
    out->launches = 1;
}

// Split depths for a launch of several matrices: roots of about equal work,
// about eight per persistent wave over the whole launch (a lone matrix keeps
// its own tuned or default depth).  With four, the waves that draw the last
// roots still run one when the others have none left; eight such roots
// shorten that end by about as much as their extra root set-ups cost, and
// sixteen or thirty-two gain nothing more.
void batch_ks(const tor_ctx *ctx, int path, const std::vector<Mat *> &grp, std::vector<int> &ks)
{
    if (grp.size() == 1 || ctx->opt.split_k > 0) {
        for (size_t j = 0; j < grp.size(); j++)
            ks[j] = choose_k(ctx, grp[j]->N, path);
        return;
    }
    double work = 0.0;
    int Nmax = 0;
    for (Mat *m : grp) {
        work += std::ldexp(1.0, m->N);
        Nmax = std::max(Nmax, m->N);
    }
    const double per_root = std::max(work / (8.0 * launch_grid(ctx, path, Nmax)), 1.0);
    const int lg = (int)std::floor(std::log2(per_root) + 0.5);
    for (size_t j = 0; j < grp.size(); j++) {
        const int N = grp[j]->N;
        ks[j] = std::max(0, std::min(N - lg, N - path_R(path)));
    }
}

// Launch the staged matrices, one launch per arithmetic path; the launches
// use the workspace from byte base on.
int run_staged(tor_ctx *ctx, std::vector<Mat *> &mats, const std::vector<int> &idx, int fixed_k, tor_result *out,
               std::vector<double> *slots_out, int *k_out, size_t base)
{
    int first_err = TOR_OK;
    const int order[NPATH] = {PATH_REAL, PATH_CPLX, PATH_QUAD};
    for (int path : order) {
        std::vector<Mat *> grp;
        std::vector<int> gidx, ks;
        for (size_t j = 0; j < mats.size(); j++)
            if (mats[j]->path == path) {
                grp.push_back(mats[j]);
                gidx.push_back(idx[j]);
                ks.push_back(std::min(std::max(fixed_k, 0), std::max(mats[j]->N - path_R(path), 0)));
            }
        if (grp.empty())
            continue;
        if (fixed_k < 0)
            batch_ks(ctx, path, grp, ks);
        std::vector<double> res;
        std::vector<int> runs;
        float ms = 0.f;
        int rc = run_recursive(ctx, path, grp, ks, res, &ms, slots_out, base, &runs);
        if (rc != TOR_OK)
            return rc;
        for (size_t j = 0; j < grp.size(); j++) {
            fill_result(*grp[j], path, &res[4 * j], ms, &out[gidx[j]]);
            out[gidx[j]].launches = runs[j];
            if (out[gidx[j]].status != TOR_OK && first_err == TOR_OK)
                first_err = out[gidx[j]].status;
        }
        if (k_out)
            *k_out = ks[0];
    }
    return first_err;
}

// Check the arguments of one matrix on the host.
bool args_ok(const tor_ctx *ctx, int n, const double *O, long ld)
{
    return n >= 0 && n <= ctx->opt.max_n && (n == 0 || (O && ld >= 2L * n));
}

// Evaluate the matrices in: argument checks, device staging, then one
// launch per path.  Matrices that fail a check or the staging get that
// status; the call returns the first error of any matrix.
int eval_many(tor_ctx *ctx, const std::vector<StageIn> &in, tor_result *out, int fixed_k,
              std::vector<double> *slots_out, int *k_out, unsigned flags)
{
    const int count = (int)in.size();
    std::vector<StageIn> good;
    std::vector<int> gi;
    int first_err = TOR_OK;
    for (int i = 0; i < count; i++) {
        const StageIn &x = in[i];
        const bool ok = x.sel ? (x.n >= 0 && x.n <= ctx->opt.max_n && x.n <= x.M && (x.M == 0 || (x.O && x.ld >= 2L * x.M)))
                              : args_ok(ctx, x.n, x.O, x.ld);
        if (!ok) {
            out[i] = tor_result{};
            out[i].status = TOR_E_INVAL;
            if (first_err == TOR_OK)
                first_err = TOR_E_INVAL;
            continue;
        }
        good.push_back(x);
        gi.push_back(i);
    }
    std::vector<Mat> mats;
    size_t end = 0;
    int rc = stage_sync(ctx, good, (flags & TOR_INPUT_DEVICE) != 0, stage_flags(flags), CPLX_R, 0, mats, &end);
    if (rc != TOR_OK)
        return rc;
    std::vector<Mat *> ok;
    std::vector<int> idx;
    for (size_t j = 0; j < mats.size(); j++) {
        if (mats[j].status != TOR_OK) {
            out[gi[j]] = tor_result{};
            out[gi[j]].status = mats[j].status;
            if (first_err == TOR_OK)
                first_err = mats[j].status;
            continue;
        }
        ok.push_back(&mats[j]);
        idx.push_back(gi[j]);
    }
    if (!ok.empty()) {
        rc = run_staged(ctx, ok, idx, fixed_k, out, slots_out, k_out, end);
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
int serve_k(const tor_ctx *ctx, const ServeCfg &cfg, const Request &r)
{
    const int LA = std::max(r.N - path_R(r.path), 0);
    const double per_root = std::max((double)cfg.chunk_subsets / (4.0 * launch_grid(ctx, r.path, r.N)), 1.0);
    const int lg = (int)std::floor(std::log2(per_root));
    const int k = std::max(choose_k(ctx, r.N, r.path), r.N - lg);
    return std::max(0, std::min(k, std::min(LA, 20)));
}

// Pool bytes of a request of n modes: the largest staged form its flags
// allow, then root slots for the deepest split any of its possible paths
// may take (serve_k never goes beyond 20).
size_t request_form_bytes(int n, unsigned sflags) { return align_up(staged_bytes(n, sflags, CPLX_R), 256); }
size_t request_bytes(int n, unsigned sflags)
{
    auto slots_for = [&](int R) {
        const int k = std::min(std::max(std::max(n, R) - R, 0), 20);
        return align_up(sizeof(double) * 4 * ((size_t)1 << k), 256);
    };
    size_t slots = (sflags & STAGE_DD) ? slots_for(QUAD_R) : slots_for(CPLX_R);
    if (!(sflags & (STAGE_DD | STAGE_FORCE_CPLX)))
        slots = std::max(slots, slots_for(REAL_R));
    return request_form_bytes(n, sflags) + slots;
}

// CUs that the chunked serving launches leave to the express launches beside
// them (two per die of an eight-die part, 6 % of its 256; 8 and 12 gave a
// higher median latency at the same saturated rate).  The express launches there fill each CU
// to half the waves it holds, so that staging (a 1024-thread workgroup with
// 52 KB of LDS, on a stream of the same CU mask) finds room beside them and
// never waits for a chunk.  Half, not just enough LDS: a staging workgroup
// puts waves on every SIMD of its CU, so none may hold two express waves
// (5 waves per CU let staging wait in 1-2 % of rounds, p99 0.47 ms).
constexpr int SERVE_QUICK_CUS = 16;
// How long before the running chunk's expected end the next one is queued
// behind it: the scheduler's polling interval and a launch's host time,
// with room to spare.
constexpr double SERVE_QUEUE_LEAD_S = 200e-6;

// A serving launch in flight on one of the context's serving lanes.
struct ServeLaunch {
    bool busy = false;
    bool quick = false;  // on the express lane
    int path = PATH_REAL;
    int slot = 0;                 // the lane slot of its buffers and events
    long long subsets = 0;        // its work
    double end_est = 0.0;         // when it should end (steady-clock seconds; 0: unknown)
    std::vector<Request *> used;  // one entry per root range (a request may hold two)
    std::vector<int> red;         // entries of used whose request the launch completes
};

// Book a finished serving launch (rc its status; res 4 doubles per entry of
// red): every request in it counts the launch once and takes its share of
// the kernel time; the ones it completed, or all of them on failure, move
// to finished, once (a request that failed in an earlier launch is not
// reported again).  A failed launch is booked only once nothing still runs
// on its lane, since the requests' memory goes back to the pool.
void retire_launch(const ServeLaunch &L, int rc, const std::vector<double> &res, float ms,
                   std::vector<Request *> &finished)
{
    std::vector<Request *> uniq;
    for (Request *r : L.used)
        if (std::find(uniq.begin(), uniq.end(), r) == uniq.end())
            uniq.push_back(r);
    for (Request *r : uniq) {
        --r->flights;
        if (L.quick)
            r->quick_flight = false;
        r->device_ms += ms / (float)uniq.size();
        ++r->launches;
    }
    if (rc != TOR_OK) {
        for (Request *r : uniq) {
            if (r->failed)
                continue;
            r->failed = true;
            r->res = tor_result{};
            r->res.status = rc;
            r->next_root = r->nroots;
            finished.push_back(r);
        }
        return;
    }
    for (size_t j = 0; j < L.red.size(); j++) {
        Request *r = L.used[L.red[j]];
        if (r->failed)
            continue;
        fill_result(r->st, L.path, &res[4 * j], r->device_ms, &r->res);
        r->res.launches = r->launches;
        finished.push_back(r);
    }
}

enum { TAKE_SMALL, TAKE_LARGE, TAKE_ANY };  // which requests a serving round takes

// One scheduling round for one path: pick root ranges of about `budget`
// subsets, the oldest request's share first, then the requests with the
// least remaining work (the small ones whole), and enqueue a launch of them
// on lane's current stream and slot, with the tuned waves per CU of their
// largest size (at most wpc_max when positive) on `cus` CUs; rec records
// it.  TAKE_SMALL takes only the requests whose remaining work is at most
// cfg.express_subsets, TAKE_LARGE only the others.  An express launch (quick
// set) leaves out every request with roots in flight; a chunked one only
// those in an express launch, since chunks run one after another on their
// lane's stream, so a request may hold roots in two queued chunks (and the
// later one reduces it).  Called with ctx->mu held.
int serve_round(tor_ctx *ctx, const ServeCfg &cfg, int path, std::vector<Request *> &active,
                std::vector<Request *> &finished, int take_kind, long long budget, int cus, int wpc_max,
                LaunchLane &lane, bool quick, ServeLaunch &rec)
{
    std::vector<Request *> cand;
    for (Request *r : active) {
        if (r->path != path || r->failed || r->next_root >= r->nroots || r->quick_flight || (quick && r->flights > 0))
            continue;
        const bool small = (r->nroots - r->next_root) * r->root_work <= cfg.express_subsets;
        if (take_kind == TAKE_ANY || small == (take_kind == TAKE_SMALL))
            cand.push_back(r);
    }
    if (cand.empty())
        return TOR_OK;
    Request *oldest = *std::min_element(cand.begin(), cand.end(),
                                        [](Request *a, Request *b) { return a->ticket < b->ticket; });
    std::stable_sort(cand.begin(), cand.end(), [](Request *a, Request *b) {
        return (a->nroots - a->next_root) * a->root_work < (b->nroots - b->next_root) * b->root_work;
    });
    std::vector<ProblemDesc> descs;
    std::vector<Request *> used;
    long long work = 0;
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
        work += n * r->root_work;
    };
    // a small request is taken whole or not at all, so that it takes one
    // launch; a large one's share may end anywhere
    auto left = [](const Request *r) { return (r->nroots - r->next_root) * r->root_work; };
    auto small = [&](const Request *r) { return left(r) <= cfg.express_subsets; };
    take(oldest, small(oldest) ? left(oldest) : (long long)(cfg.oldest_share * (double)budget));
    for (Request *r : cand) {
        if (budget <= 0)
            break;
        if (r->next_root >= r->nroots)
            continue;
        if (!small(r))
            take(r, budget);
        else if (left(r) <= budget)
            take(r, left(r));
    }
    int Nmax = 0;
    for (auto &d : descs)
        Nmax = std::max(Nmax, d.N);
    int wpc = launch_grid(ctx, path, Nmax) / ctx->num_cu;
    if (wpc_max > 0)
        wpc = std::min(wpc, wpc_max);
    const int grid = wpc * cus;
    // reduce the requests that this launch completes
    std::vector<int> red;
    for (size_t i = 0; i < used.size(); i++)
        if (used[i]->next_root == used[i]->nroots && std::find(used.begin(), used.begin() + i, used[i]) == used.begin() + i)
            red.push_back((int)i);
    rec = ServeLaunch{};
    rec.quick = quick;
    rec.path = path;
    rec.slot = lane.slot;
    rec.subsets = work;
    rec.used = std::move(used);
    rec.red = std::move(red);
    for (size_t i = 0; i < rec.used.size(); i++)
        if (std::find(rec.used.begin(), rec.used.begin() + i, rec.used[i]) == rec.used.begin() + i) {
            ++rec.used[i]->flights;
            rec.used[i]->quick_flight |= quick;
        }
    const int rc = run_launch(ctx, path, descs, rec.red, 0, grid, nullptr, nullptr, 0, nullptr, &lane);
    if (rc != TOR_OK) {
        // its requests may hold roots in a launch queued before it
        for (hipStream_t st : {lane.stream, lane.side, lane.wide})
            if (st)
                (void)hipStreamSynchronize(st);
        retire_launch(rec, rc, {}, 0.f, finished);
        rec = ServeLaunch{};
        return rc;
    }
    lane.slot ^= 1;
    rec.busy = true;
    return TOR_OK;
}

// Retire the launch if its done event has been reached, or on a failed
// query, once its lane has drained.  Called with ctx->mu held.
bool poll_launch(const LaunchLane &lane, ServeLaunch &rec, std::vector<Request *> &finished, double *ms_per_subset)
{
    if (!rec.busy)
        return false;
    const hipError_t q = hipEventQuery(lane.done[rec.slot]);
    if (q == hipErrorNotReady)
        return false;
    std::vector<double> res;
    float ms = 0.f;
    const int rc = hip_status(q);
    if (rc == TOR_OK) {
        lane_collect(lane, rec.slot, (int)rec.red.size(), res, &ms);
        if (ms_per_subset && rec.subsets > 0 && ms > 0.f) {
            const double x = ms / (double)rec.subsets;
            *ms_per_subset = *ms_per_subset > 0.0 ? 0.75 * *ms_per_subset + 0.25 * x : x;
        }
    } else {
        for (hipStream_t st : {lane.stream, lane.side, lane.wide})
            if (st)
                (void)hipStreamSynchronize(st);
    }
    retire_launch(rec, rc, res, ms, finished);
    rec = ServeLaunch{};
    return true;
}

// The scheduler.  Two launch lanes, each with at most one launch in flight:
// the chunk lane runs chunked launches of at most cfg.chunk_subsets on all
// CUs but SERVE_QUICK_CUS of them; the quick lane runs express launches of
// small requests, on those SERVE_QUICK_CUS CUs while a chunk is in flight
// (half full, with about as much work as they do in a chunk's time), on the
// whole device otherwise.  Staging runs on those CUs too while a chunk is in
// flight, on the context's stream otherwise.
// Each round retires the launches that have ended, enqueues the next chunk,
// stages the newly admitted requests, enqueues an express launch, and
// publishes the finished requests; while launches are in flight it polls
// their events.  A chunk takes the requests too large for express launches,
// and small ones only while the express lane is busy.  So a small request
// waits for neither the chunk in flight nor a large request: only for the
// express launch before it.
void serve_loop(tor_ctx *ctx)
{
    std::vector<Request *> active;
    std::deque<ServeLaunch> chunks;  // in flight on the chunk lane, in stream order (at most two)
    ServeLaunch quick;               // in flight on the express lane
    double rate[NPATH] = {};         // kernel ms per subset of the recent chunks, per path
    int next_chunk = 0, next_quick = 0;  // each lane takes the paths in turn
    auto now_s = [] {
        return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
    };
    static const int kPaths[NPATH] = {PATH_REAL, PATH_CPLX, PATH_QUAD};
    (void)prctl(PR_SET_TIMERSLACK, 1000ul, 0ul, 0ul, 0ul);  // polling sleeps of tens of microseconds
    // retire finished requests: release their pool memory and wake pollers
    auto publish = [&](std::vector<Request *> &fin) {
        if (fin.empty())
            return;
        {
            std::lock_guard<std::mutex> g(ctx->smu);
            for (Request *r : fin) {
                pool_release(ctx, r->pool_off, r->pool_len);
                r->done = true;
                --ctx->admitted;
                active.erase(std::remove(active.begin(), active.end(), r), active.end());
            }
        }
        ctx->scv.notify_all();
        fin.clear();
    };
    for (;;) {
        std::vector<Request *> admit;
        ServeCfg cfg;
        {
            std::unique_lock<std::mutex> lk(ctx->smu);
            auto ready = [&] {
                return ctx->stop || !ctx->pending.empty() || (chunks.empty() && !quick.busy && !active.empty());
            };
            if (!chunks.empty() || quick.busy)  // poll the events, waking early for new requests
                ctx->scv.wait_for(lk, std::chrono::microseconds(20), ready);
            else
                ctx->scv.wait(lk, ready);
            if (ctx->stop)
                return;  // tor_destroy drains the serving lanes
            cfg = ctx->serve;  // this round's policy
            // admission by device footprint, in arrival order
            const unsigned sfl = stage_flags(ctx->opt.flags);
            while (!ctx->pending.empty()) {
                Request *r = ctx->pending.front();
                if (!ctx->pool) {
                    if (hipSetDevice(ctx->device) != hipSuccess ||
                        hipMalloc((void **)&ctx->pool, ctx->pool_bytes) != hipSuccess) {
                        // no device memory for the pool: every waiting
                        // request completes with TOR_E_NOMEM (the next
                        // submission tries again)
                        ctx->pool = nullptr;
                        for (Request *q : ctx->pending) {
                            q->res = tor_result{};
                            q->res.status = TOR_E_NOMEM;
                            q->done = true;
                        }
                        ctx->pending.clear();
                        ctx->scv.notify_all();
                        break;
                    }
                    ctx->pool_free.clear();
                    ctx->pool_free[0] = ctx->pool_bytes;
                }
                size_t off;
                const size_t len = request_bytes(r->n, sfl);
                if (!pool_alloc(ctx, len, off))
                    break;
                r->pool_off = off;
                r->pool_len = len;
                r->dC = ctx->pool + off;
                ctx->pending.pop_front();
                admit.push_back(r);
                ++ctx->admitted;
            }
        }
        std::vector<Request *> finished;
        {
            std::lock_guard<std::mutex> g(ctx->mu);
            int rc = hipSetDevice(ctx->device) == hipSuccess ? TOR_OK : TOR_E_DEVICE;
            if (rc == TOR_OK)
                rc = lane_open(ctx->chunk, ctx->num_cu, 0, ctx->num_cu - SERVE_QUICK_CUS, false, false);
            if (rc == TOR_OK)
                rc = lane_open(ctx->quick, ctx->num_cu, ctx->num_cu - SERVE_QUICK_CUS, SERVE_QUICK_CUS, true, true);
            // express launches beside a chunk need both masks
            const bool beside = rc == TOR_OK && ctx->chunk.cus > 0 && ctx->quick.cus > 0;
            if (rc == TOR_OK) {
                while (!chunks.empty() && poll_launch(ctx->chunk, chunks.front(), finished, &rate[chunks.front().path]))
                    chunks.pop_front();
                poll_launch(ctx->quick, quick, finished, nullptr);
            }
            // the next chunk: the large requests, or, while the express lane
            // is busy, any (the paths in turn).  It is queued behind the one
            // running when that one is due to end within SERVE_QUEUE_LEAD_S
            // (by the rate of recent chunks), so the lane does not sit idle
            // while the host sees the end and launches the next.
            auto start_chunk = [&] {
                if (chunks.size() >= 2 ||
                    (chunks.size() == 1 && !(chunks.back().end_est > 0.0 && now_s() >= chunks.back().end_est - SERVE_QUEUE_LEAD_S)))
                    return;
                ServeLaunch rec;
                for (int kind : {TAKE_LARGE, TAKE_ANY}) {
                    if (kind == TAKE_ANY && cfg.express_subsets > 0 && !quick.busy)
                        break;
                    for (int i = 0; i < NPATH && !rec.busy; i++) {
                        const int path = kPaths[(next_chunk + i) % NPATH];
                        serve_round(ctx, cfg, path, active, finished, kind, cfg.chunk_subsets,
                                    ctx->chunk.cus > 0 ? ctx->chunk.cus : ctx->num_cu, 0, ctx->chunk, false, rec);
                        if (rec.busy)
                            next_chunk = (next_chunk + i + 1) % NPATH;
                    }
                    if (rec.busy)
                        break;
                }
                if (!rec.busy)
                    return;
                const double t = now_s();
                const bool known = rate[rec.path] > 0.0 && (chunks.empty() || chunks.back().end_est > 0.0);
                const double start = chunks.empty() ? t : std::max(t, chunks.back().end_est);
                rec.end_est = known ? start + 1e-3 * rate[rec.path] * (double)rec.subsets : 0.0;
                chunks.push_back(std::move(rec));
            };
            if (rc == TOR_OK)
                start_chunk();
            // stage the admitted requests on the device, straight into their
            // pool slots; the path and size of each are known from here on
            const unsigned sfl = stage_flags(ctx->opt.flags);
            std::vector<StageIn> in(admit.size());
            for (size_t j = 0; j < admit.size(); j++) {
                in[j].n = admit[j]->n;
                in[j].O = admit[j]->raw.empty() ? nullptr : admit[j]->raw.data();
                in[j].ld = 2L * admit[j]->n;
                in[j].dst = admit[j]->dC;
            }
            std::vector<Mat> mats;
            size_t end = 0;
            // on the express CUs while a chunk holds the others (an unmasked
            // workgroup can be handed to a shader engine whose CUs the chunk
            // fills, and wait there for the whole chunk)
            const hipStream_t sst = !chunks.empty() && ctx->quick.side ? ctx->quick.side : ctx->stream;
            const int src = admit.empty() ? TOR_OK : stage_sync(ctx, in, false, sfl, CPLX_R, 0, mats, &end, sst);
            for (size_t j = 0; j < admit.size(); j++) {
                Request *r = admit[j];
                const int st = src != TOR_OK ? src : mats[j].status;
                if (st != TOR_OK) {
                    r->res = tor_result{};
                    r->res.status = st;
                    finished.push_back(r);
                    continue;
                }
                r->st = mats[j];
                r->path = r->st.path;
                r->N = r->st.N;
                r->k = serve_k(ctx, cfg, *r);
                r->nroots = 1ll << r->k;
                r->next_root = 0;
                r->root_work = 1ll << (r->N - r->k);
                r->dSlots = (double *)(r->dC + request_form_bytes(r->n, sfl));
                std::vector<double>().swap(r->raw);
                active.push_back(r);
            }
            if (rc != TOR_OK) {
                // no serving lanes: every admitted request fails
                for (Request *r : active)
                    if (r->flights == 0 && !r->failed) {
                        r->failed = true;
                        r->res = tor_result{};
                        r->res.status = rc;
                        finished.push_back(r);
                    }
            } else {
                // small requests: beside the chunk in flight on the express
                // lane's own CUs, with about the work those CUs do in a
                // chunk's time, or on the whole device when no chunk runs
                const bool chunk_busy = !chunks.empty();
                if (cfg.express_subsets > 0 && !quick.busy && (!chunk_busy || beside)) {
                    ctx->quick.cur = chunk_busy ? ctx->quick.stream : ctx->quick.wide;
                    const int cus = chunk_busy ? ctx->quick.cus : ctx->num_cu;
                    const long long budget =
                        chunk_busy ? std::max(1ll, cfg.chunk_subsets / ctx->num_cu * cus) : (1ll << 62);
                    for (int i = 0; i < NPATH && !quick.busy; i++) {
                        const int path = kPaths[(next_quick + i) % NPATH];
                        serve_round(ctx, cfg, path, active, finished, TAKE_SMALL, budget, cus,
                                    chunk_busy ? std::max(1, ctx->fit[path] / 2) : 0, ctx->quick, true, quick);
                        if (quick.busy)
                            next_quick = (next_quick + i + 1) % NPATH;
                    }
                }
                start_chunk();
            }
        }
        publish(finished);
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
    const unsigned sfl = path == PATH_CPLX ? STAGE_FORCE_CPLX : path == PATH_QUAD ? STAGE_DD : 0u;
    std::vector<StageIn> in(1);
    in[0].n = n;
    in[0].O = O.data();
    in[0].ld = 2L * n;
    std::vector<Mat> mats;
    size_t base = 0;
    int rc = stage_sync(ctx, in, false, sfl, CPLX_R, 0, mats, &base);
    if (rc != TOR_OK)
        return rc;
    if (mats[0].status != TOR_OK || mats[0].path != path)
        return TOR_E_INVAL;
    const int N = mats[0].N;
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
                std::vector<Mat *> ms{&mats[0]};
                std::vector<int> ks{k};
                // run with this grid: temporarily pin the table entry
                TuneEntry save = ctx->tune[path][std::min(N, MAX_N)];
                ctx->tune[path][std::min(N, MAX_N)] = TuneEntry{true, k, w, 0.f};
                std::vector<double> res;
                float ms_ = 0.f;
                rc = run_recursive(ctx, path, ms, ks, res, &ms_, nullptr, base, nullptr);
                ctx->tune[path][std::min(N, MAX_N)] = save;
                if (rc != TOR_OK)
                    return rc;
                if (rep > 0)
                    tmin = std::min(tmin, ms_);
            }
            if (!best.valid || tmin < best.ms)
                best = TuneEntry{true, k, w, tmin};
        }
    }
    return TOR_OK;
}

// ---- the allocation-free evaluation (tor_eval_static) -----------------------
// A file-scope device array: every GPU the library runs on holds its own copy,
// at its own address, once a context has been created on it, until the
// process ends.  Host code never uses the array's name as an address (on the
// host it only stands for the symbol): tor_create resolves the device
// address with hipGetSymbolAddress, with that device current, and keeps it
// per device; kernels receive that address as an argument.
__device__ __align__(256) char scratch[TOR_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
struct StaticScratch {
    std::mutex mu;          // one tor_eval_static at a time on a device
    char *ptr = nullptr;    // the device address of `scratch` on that device
    bool resolved = false;
    hipError_t err = hipSuccess;
};
StaticScratch g_static[kMaxDevices];
std::mutex g_static_init;

// Resolve the array's address on `device` (the current device) once.
void resolve_static(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return;
    std::lock_guard<std::mutex> g(g_static_init);
    StaticScratch &ss = g_static[device];
    if (ss.resolved)
        return;
    void *p = nullptr;
    ss.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    ss.ptr = ss.err == hipSuccess ? (char *)p : nullptr;
    ss.resolved = true;
}

// Byte layout of one tor_eval_static call in the device array: the staging
// descriptor and record, the launch descriptor, queue counter and result,
// then (from kStaticData on) the host input's copy, the staged form, the
// root slots and the per-wave stacks.
constexpr size_t kStaticDesc = 0, kStaticInfo = 256, kStaticProb = 512, kStaticCounter = 1024,
                 kStaticRes = 1280, kStaticData = 4096;

int eval_static(tor_ctx *ctx, char *base, int n, const double *O, long ld, tor_result *out)
{
    const bool dev_in = (ctx->opt.flags & TOR_INPUT_DEVICE) != 0;
    const unsigned sfl = stage_flags(ctx->opt.flags);
    const int n2 = 2 * n;
    size_t at = kStaticData;
    char *dRaw = nullptr;
    if (!dev_in && n > 0) {
        dRaw = base + at;
        at += align_up(sizeof(c64) * (size_t)n2 * n2, 256);
    }
    char *dForm = base + at;
    at += align_up(staged_bytes(n, sfl, CPLX_R), 256);
    if (at > TOR_STATIC_SCRATCH_BYTES)
        return TOR_E_SCRATCH;
    StageDesc *dDesc = (StageDesc *)(base + kStaticDesc);
    StageInfo *dInfo = (StageInfo *)(base + kStaticInfo);
    ProblemDesc *dProb = (ProblemDesc *)(base + kStaticProb);
    unsigned long long *dCounter = (unsigned long long *)(base + kStaticCounter);
    double *dRes = (double *)(base + kStaticRes);

    // staging: the host matrix (compact rows) and the descriptor go up from
    // host memory the caller or this frame owns, both alive until the
    // synchronisations below
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess && dRaw)
        e = hipMemcpy2DAsync(dRaw, sizeof(c64) * n2, O, sizeof(c64) * (size_t)ld, sizeof(c64) * n2, n2,
                             hipMemcpyHostToDevice, ctx->stream);
    StageDesc d{};
    d.O = dRaw ? (const double *)dRaw : O;
    d.ld = dRaw ? n2 : ld;
    d.sel = nullptr;
    d.n = n;
    d.M = n;
    d.flags = sfl;
    d.min_cplx = CPLX_R;
    d.out = dForm;
    d.info = dInfo;
    StageInfo info{};
    if (e == hipSuccess)
        e = hipMemcpyAsync(dDesc, &d, sizeof(d), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = launch_stage(dDesc, 1, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&info, dInfo, sizeof(info), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess)
        return hip_status(e);
    if (info.status != 0) {
        *out = tor_result{};
        out->status = TOR_E_INVAL;
        return TOR_E_INVAL;
    }
    Mat m;
    m.n = n;
    m.N = info.N;
    m.path = info.path;
    const int path = info.path, N = info.N;
    const int k = choose_k(ctx, N, path);
    const long long nroots = 1ll << k;
    double *dSlots = (double *)(base + at);
    at += align_up(sizeof(double) * 4 * (size_t)nroots, 256);
    const long long stride = wave_stack_bytes(path, N, k);
    const int grid = (int)std::min<long long>(launch_grid(ctx, path, N), nroots);
    if (at + (size_t)stride * grid > TOR_STATIC_SCRATCH_BYTES)
        return TOR_E_SCRATCH;
    ProblemDesc pd{};
    pd.C = dForm;
    pd.slots = dSlots;
    pd.N = N;
    pd.k = k;
    pd.root_begin = 0;
    pd.item_begin = 0;
    pd.nroots = nroots;
    MainParams mp{};
    mp.probs = dProb;
    mp.nprob = 1;
    mp.total_items = nroots;
    mp.counter = dCounter;
    mp.scratch = base + at;
    mp.scratch_stride = stride;
    const bool dd = ctx->opt.accum != TOR_ACCUM_FP64 || path == PATH_QUAD;
    double h[4] = {0, 0, 0, 0};
    e = hipMemcpyAsync(dProb, &pd, sizeof(pd), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)  // the queue head starts at zero: a fill kernel, no memset
        e = launch_zero(dCounter, 1, ctx->stream);
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev0, ctx->stream);
    if (e == hipSuccess)
        e = launch_main(path, dd, mp, grid, ctx->stream);
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev1, ctx->stream);
    if (e == hipSuccess)
        e = launch_reduce(dProb, 1, dRes, dd, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h, dRes, sizeof(h), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess)
        return hip_status(e);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    fill_result(m, path, h, ms, out);
    return out->status;
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
    case TOR_E_SCRATCH: return "the problem exceeds the static scratch of tor_eval_static";
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
    // the largest per-wave stack: 16-byte scalars, the smallest R, k = 0
    const size_t scr = align_up((size_t)stack_bytes(N, 0, Rmin, 16, 16), 256) * grid;
    // staging: descriptors and status records, a raw copy of each input and its
    // staged form (16-byte scalars bound every path)
    const size_t n2 = 2 * (size_t)std::max(max_n, 1);
    const size_t stage = align_up(sizeof(StageDesc) * cnt, 256) + align_up(sizeof(StageInfo) * cnt, 256) + 256 +
                         (align_up(sizeof(c64) * n2 * n2, 256) + align_up(sizeof(c64) * (size_t)NSZ(N), 256)) * cnt;
    return stage + 2 * align_up(sizeof(ProblemDesc) * cnt, 256) + 256 + align_up(32 * (size_t)items, 256) +
           align_up(32 * (size_t)cnt, 256) + scr + (1 << 20);
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
        ((o.flags & TOR_FACTOR_DD) && (o.flags & TOR_FORCE_COMPLEX)) ||
        ((uintptr_t)o.workspace & 255))  // the kernels read 16-byte granules
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
    resolve_static(o.device);  // the device is current
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
        lane_close(ctx->chunk);  // each waits for a serving launch still in flight
        lane_close(ctx->quick);
        if (ctx->own_ws && ctx->ws)
            (void)hipFree(ctx->ws);
        if (ctx->pool)
            (void)hipFree(ctx->pool);
        if (ctx->hup)
            (void)hipHostFree(ctx->hup);
        if (ctx->hdown)
            (void)hipHostFree(ctx->hdown);
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

int tor_eval_static(tor_ctx *ctx, int n, const double *O, long ld, tor_result *out)
{
    if (!ctx || !out || !args_ok(ctx, n, O, ld))
        return TOR_E_INVAL;
    if (ctx->device < 0 || ctx->device >= kMaxDevices || !g_static[ctx->device].ptr)
        return TOR_E_DEVICE;
    StaticScratch &ss = g_static[ctx->device];
    std::lock_guard<std::mutex> g(ctx->mu);
    std::lock_guard<std::mutex> gs(ss.mu);
    return eval_static(ctx, ss.ptr, n, O, ld, out);
}

int tor_eval(tor_ctx *ctx, int n, const double *O, long ld, tor_result *out)
{
    if (!ctx || !out)
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    std::vector<StageIn> in(1);
    in[0].n = n;
    in[0].O = O;
    in[0].ld = ld;
    tor_result r{};
    int rc = eval_many(ctx, in, &r, -1, nullptr, nullptr, ctx->opt.flags);
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
    std::vector<StageIn> in(count);
    for (int i = 0; i < count; i++) {
        in[i].n = n[i];
        in[i].O = O[i];
        in[i].ld = ld[i];
    }
    return eval_many(ctx, in, out, -1, nullptr, nullptr, ctx->opt.flags);
}

int tor_eval_partials(tor_ctx *ctx, int n, const double *O, long ld, int k_max, int *k_out, double *partials,
                      tor_result *out)
{
    if (!ctx || !out || !k_out || !partials || k_max < 0 || k_max > 30)
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    std::vector<StageIn> in(1);
    in[0].n = n;
    in[0].O = O;
    in[0].ld = ld;
    std::vector<double> slots;
    int k = 0;
    tor_result r{};
    int rc = eval_many(ctx, in, &r, k_max, &slots, &k, ctx->opt.flags);
    if (rc != TOR_OK && rc != TOR_E_NUMERIC)
        return rc;
    *out = r;
    *k_out = k;
    // padding modes scale each partial's sum of |t| by 3 (see fill_result)
    const int path = r.path == 1 ? PATH_REAL : r.path == 3 ? PATH_QUAD : PATH_CPLX;
    const int pad = std::max(n, path_R(path)) - n;
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
    if (count == 0)
        return TOR_OK;
    std::lock_guard<std::mutex> g(ctx->mu);
    // O on the device (the caller's, or one copy in the workspace), then the
    // scratch and result of sqrt(det(I - O)), then the staged patterns
    const int m2 = 2 * M;
    const bool dev = (ctx->opt.flags & TOR_INPUT_DEVICE) != 0;
    const size_t bO = dev ? 0 : align_up(sizeof(c64) * (size_t)m2 * m2, 256);
    const size_t bScr = align_up(sizeof(c64) * (size_t)std::max(m2 * m2, 1), 256);
    const size_t base = bO + bScr + 256;
    // the principal submatrix of every pattern: rows and columns {s, s + M}
    std::vector<std::vector<int>> sels(count);
    std::vector<StageIn> in(count);
    for (int i = 0; i < count; i++) {
        for (int q = 0; q < M; q++)
            if ((patterns[i] >> q) & 1ull)
                sels[i].push_back(q);
        in[i].n = (int)sels[i].size();
        in[i].sel = sels[i].empty() ? nullptr : sels[i].data();
        in[i].M = M;
    }
    const unsigned sfl = stage_flags(ctx->opt.flags);
    // the workspace takes O and the staging area before O is placed in it
    int rc = ensure_ws_keep(ctx, base + stage_layout(in, true, sfl, CPLX_R).total, 0);
    if (rc != TOR_OK)
        return rc;
    hipError_t e = hipSetDevice(ctx->device);
    const double *dO = O;
    long dld = ld;
    if (!dev && M > 0) {
        e = hipMemcpy2DAsync(ctx->ws, sizeof(c64) * m2, O, sizeof(c64) * (size_t)ld, sizeof(c64) * m2, m2,
                             hipMemcpyHostToDevice, ctx->stream);
        dO = (const double *)ctx->ws;
        dld = m2;
    }
    double *dDet = (double *)(ctx->ws + bO + bScr);
    if (e == hipSuccess && M > 0)
        e = launch_sqrt_det(dO, dld, M, (c64 *)(ctx->ws + bO), dDet, ctx->stream);
    if (e != hipSuccess)
        return hip_status(e);
    for (int i = 0; i < count; i++) {
        in[i].O = dO;
        in[i].ld = dld;
    }
    std::vector<Mat> mats;
    size_t end = 0, down = 0;
    rc = stage_enqueue(ctx, in, true, sfl, CPLX_R, base, mats, &end, &down);
    if (rc != TOR_OK)
        return rc;
    // stage_enqueue leaves 256 spare bytes after the status records (a copy into
    // the buffer is pending, so it must not be regrown here)
    const size_t det_at = align_up(down, 16);
    if (det_at + 2 * sizeof(double) > ctx->hdown_bytes)
        return TOR_E_NOMEM;
    double *hDet = (double *)(ctx->hdown + det_at);
    hDet[0] = 1.0;
    hDet[1] = 0.0;
    e = hipSuccess;
    if (M > 0)
        e = hipMemcpyAsync(hDet, dDet, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess)
        return hip_status(e);
    stage_collect(ctx, mats);
    const double sq = hDet[0];
    if (hDet[1] != 0.0 || !(sq > 0.0))
        return TOR_E_NOT_PD;
    std::vector<tor_result> res(count);
    std::vector<Mat *> ok;
    std::vector<int> idx;
    int first_err = TOR_OK;
    for (int i = 0; i < count; i++) {
        if (mats[i].status != TOR_OK) {
            res[i] = tor_result{};
            res[i].status = mats[i].status;
            if (first_err == TOR_OK)
                first_err = mats[i].status;
            continue;
        }
        ok.push_back(&mats[i]);
        idx.push_back(i);
    }
    if (!ok.empty()) {
        rc = run_staged(ctx, ok, idx, -1, res.data(), nullptr, nullptr, end);
        if (rc != TOR_OK && first_err == TOR_OK)
            first_err = rc;
    }
    for (int i = 0; i < count; i++) {
        probs[i] = res[i].status == TOR_OK ? (res[i].tor + res[i].tor_lo) * sq : NAN;
        if (results)
            results[i] = res[i];
    }
    return first_err;
}

int tor_click_all(tor_ctx *ctx, int M, const double *O, long ld, double *probs, double *tor_hi, double *tor_lo,
                  tor_result *out)
{
    if (!ctx || M < 0 || M > TOR_CLICK_ALL_MAX_M || M > ctx->opt.max_n || (M > 0 && (!O || ld < 2L * M)) ||
        (!probs && !tor_hi && !out) || (!tor_hi != !tor_lo))
        return TOR_E_INVAL;
    const bool dev_out = (ctx->opt.flags & TOR_OUTPUT_DEVICE) != 0;
    // the terms are stored by the FP64 kernel of the real quadrature form
    if (ctx->opt.flags & (TOR_FORCE_COMPLEX | TOR_FACTOR_DD))
        return TOR_E_INVAL;
    if (M == 0) {  // the empty pattern of a 0-mode state: Tor = 1, p = 1
        const double one[2] = {1.0, 0.0};
        if (dev_out && (probs || tor_hi)) {
            std::lock_guard<std::mutex> g(ctx->mu);
            hipError_t e = hipSetDevice(ctx->device);
            if (e == hipSuccess && probs)
                e = hipMemcpyAsync(probs, &one[0], sizeof(double), hipMemcpyHostToDevice, ctx->stream);
            if (e == hipSuccess && tor_hi)
                e = hipMemcpyAsync(tor_hi, &one[0], sizeof(double), hipMemcpyHostToDevice, ctx->stream);
            if (e == hipSuccess && tor_lo)
                e = hipMemcpyAsync(tor_lo, &one[1], sizeof(double), hipMemcpyHostToDevice, ctx->stream);
            if (e == hipSuccess)
                e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess)
                return hip_status(e);
        } else {
            if (probs)
                probs[0] = 1.0;
            if (tor_hi)
                tor_hi[0] = 1.0;
            if (tor_lo)
                tor_lo[0] = 0.0;
        }
        if (out) {
            std::memset(out, 0, sizeof(*out));
            out->tor = 1.0;
            out->sum_abs = 1.0;
            out->subsets = 1;
            out->path = api_path(PATH_REAL);
        }
        return TOR_OK;
    }
    std::lock_guard<std::mutex> g(ctx->mu);
    const int m2 = 2 * M;
    const bool dev = (ctx->opt.flags & TOR_INPUT_DEVICE) != 0;
    const size_t bO = dev ? 0 : align_up(sizeof(c64) * (size_t)m2 * m2, 256);
    const size_t bScr = align_up(sizeof(c64) * (size_t)m2 * m2, 256);
    const size_t base = bO + bScr + 256;
    std::vector<StageIn> in(1);
    in[0].n = M;
    in[0].M = M;
    const unsigned sfl = stage_flags(ctx->opt.flags);
    int rc = ensure_ws_keep(ctx, base + stage_layout(in, true, sfl, CPLX_R).total, 0);
    if (rc != TOR_OK)
        return rc;
    hipError_t e = hipSetDevice(ctx->device);
    const double *dO = O;
    long dld = ld;
    if (e == hipSuccess && !dev) {
        e = hipMemcpy2DAsync(ctx->ws, sizeof(c64) * m2, O, sizeof(c64) * (size_t)ld, sizeof(c64) * m2, m2,
                             hipMemcpyHostToDevice, ctx->stream);
        dO = (const double *)ctx->ws;
        dld = m2;
    }
    double *dDet = (double *)(ctx->ws + bO + bScr);
    if (e == hipSuccess)
        e = launch_sqrt_det(dO, dld, M, (c64 *)(ctx->ws + bO), dDet, ctx->stream);
    if (e != hipSuccess)
        return hip_status(e);
    in[0].O = dO;
    in[0].ld = dld;
    std::vector<Mat> mats;
    size_t end = 0, down = 0;
    rc = stage_enqueue(ctx, in, true, sfl, CPLX_R, base, mats, &end, &down);
    if (rc != TOR_OK)
        return rc;
    const size_t det_at = align_up(down, 16);
    if (det_at + 2 * sizeof(double) > ctx->hdown_bytes)
        return TOR_E_NOMEM;
    double *hDet = (double *)(ctx->hdown + det_at);
    e = hipMemcpyAsync(hDet, dDet, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess)
        return hip_status(e);
    stage_collect(ctx, mats);
    if (hDet[1] != 0.0 || !(hDet[0] > 0.0))
        return TOR_E_NOT_PD;
    if (mats[0].status != TOR_OK)
        return mats[0].status;
    if (mats[0].path != PATH_REAL)
        return TOR_E_INVAL;  // O lacks the Gaussian-state block structure
    const int N = mats[0].N;
    const int k = choose_k(ctx, N, PATH_REAL);
    // after the staged matrix: root slots, the 2^N terms, their subset sums,
    // staging arrays for the outputs that go to the host (none with
    // TOR_OUTPUT_DEVICE), then what run_launch needs
    const long long nS = 1ll << N, nP = 1ll << M;
    const size_t oSlots = align_up(end, 256);
    const size_t oTerms = align_up(oSlots + sizeof(double) * 4 * ((size_t)1 << k), 256);
    const size_t oG = align_up(oTerms + sizeof(double) * (size_t)nS, 256);
    const size_t oOut = align_up(oG + sizeof(ddr) * (size_t)nS, 256);
    const int nstage = dev_out ? 0 : (probs ? 1 : 0) + (tor_hi ? 2 : 0);
    const size_t off = align_up(oOut + nstage * sizeof(double) * (size_t)nP, 256);
    const long long stack = wave_stack_bytes(PATH_REAL, N, k);
    const int fit = std::max(1, std::min(main_store_occupancy(), ctx->fit[PATH_REAL]));
    const int grid = ctx->num_cu * fit;
    rc = ensure_ws_keep(ctx, off + launch_layout(1, 1, stack).total(grid), end);
    if (rc != TOR_OK)
        return rc;
    double *dTerms = (double *)(ctx->ws + oTerms);
    ddr *dG = (ddr *)(ctx->ws + oG);
    double *dP = (double *)(ctx->ws + oOut), *dH = dP + (probs ? nP : 0), *dL = dH + nP;
    dDet = (double *)(ctx->ws + bO + bScr);  // the workspace may have moved
    std::vector<ProblemDesc> descs(1);
    ProblemDesc &d = descs[0];
    d.C = mat_ptr(ctx, mats[0]);
    d.slots = (double *)(ctx->ws + oSlots);
    d.N = N;
    d.k = k;
    d.root_begin = 0;
    d.nroots = 1ll << k;
    std::vector<double> res;
    float ms_main = 0.f, ms_zeta = 0.f;
    rc = run_launch(ctx, PATH_REAL, descs, std::vector<int>{0}, off, grid, &res, &ms_main, 0, dTerms);
    if (rc != TOR_OK)
        return rc;
    if (res[3] >= SLOT_NOT_PD)
        return TOR_E_NOT_PD;
    if (res[3] > 0.0)
        return TOR_E_NUMERIC;
    e = hipEventRecord(ctx->ev0, ctx->stream);
    if (e == hipSuccess)
        e = launch_zeta(dTerms, dG, N, ctx->stream);
    // where the kernel writes: the caller's device arrays, or the workspace
    // (then copied to the caller's host arrays)
    double *pP = probs ? (dev_out ? probs : dP) : nullptr;
    double *pH = tor_hi ? (dev_out ? tor_hi : dH) : nullptr;
    double *pL = tor_lo ? (dev_out ? tor_lo : dL) : nullptr;
    if (e == hipSuccess && (pP || pH))
        e = launch_click_out(dG, N, M, dDet, pP, pH, pL, ctx->stream);
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev1, ctx->stream);
    if (e == hipSuccess && probs && !dev_out)
        e = hipMemcpyAsync(probs, dP, sizeof(double) * nP, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess && tor_hi && !dev_out)
        e = hipMemcpyAsync(tor_hi, dH, sizeof(double) * nP, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess && tor_lo && !dev_out)
        e = hipMemcpyAsync(tor_lo, dL, sizeof(double) * nP, hipMemcpyDeviceToHost, ctx->stream);
    // the whole state's Tor for out: the subset sum of the pattern of every
    // mode (index bit N-1-q for mode q: the top M bits), with the sign
    // (-1)^(N-M) that turns a subset sum into a Torontonian
    ddr full{0.0, 0.0};
    if (e == hipSuccess && out)
        e = hipMemcpyAsync(&full, dG + ((nP - 1) << (N - M)), sizeof(ddr), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess)
        return hip_status(e);
    (void)hipEventElapsedTime(&ms_zeta, ctx->ev0, ctx->ev1);
    if (out) {
        // the result of the whole state (every mode clicks), with the sum of
        // |t| over all subsets and the device time of both steps
        const double sg = ((N - M) & 1) ? -1.0 : 1.0;
        const double r[4] = {sg * full.hi, sg * full.lo, res[2], 0.0};
        fill_result(mats[0], PATH_REAL, r, ms_main + ms_zeta, out);
    }
    return TOR_OK;
}

int tor_debug_zeta(tor_ctx *ctx, int nbits, const double *t, double *g_hi, double *g_lo)
{
    if (!ctx || nbits < 1 || nbits > 26 || !t || !g_hi || !g_lo)
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    const size_t n = (size_t)1 << nbits;
    const size_t oG = align_up(sizeof(double) * n, 256);
    int rc = ensure_ws(ctx, oG + sizeof(ddr) * n);
    if (rc != TOR_OK)
        return rc;
    std::vector<ddr> h(n);
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->ws, t, sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = launch_zeta((const double *)ctx->ws, (ddr *)(ctx->ws + oG), nbits, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h.data(), ctx->ws + oG, sizeof(ddr) * n, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess)
        return hip_status(e);
    for (size_t i = 0; i < n; i++) {
        g_hi[i] = h[i].hi;
        g_lo[i] = h[i].lo;
    }
    return TOR_OK;
}

int tor_eval_plain(tor_ctx *ctx, int n, const double *O, long ld, unsigned long long mask_begin,
                   unsigned long long mask_end, tor_result *out)
{
    if (!ctx || !out || n < 1 || n > 34 || mask_begin > mask_end || mask_end > (1ull << n) || !args_ok(ctx, n, O, ld))
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    // the form the recursive kernel would use (the real quadrature form of a
    // Gaussian-state matrix, else the complex matrix; TOR_FORCE_COMPLEX
    // forces the latter), FP64, unpadded
    std::vector<StageIn> in(1);
    in[0].n = n;
    in[0].O = O;
    in[0].ld = ld;
    std::vector<Mat> mats;
    size_t end = 0;
    const unsigned sfl = stage_flags(ctx->opt.flags) & ~STAGE_DD;
    int rc = stage_sync(ctx, in, (ctx->opt.flags & TOR_INPUT_DEVICE) != 0, sfl, 0, 0, mats, &end);
    if (rc != TOR_OK)
        return rc;
    if (mats[0].status != TOR_OK)
        return mats[0].status;
    const bool real = mats[0].path == PATH_REAL;
    const int chunk = 16;
    // no more waves than chunks of the mask range
    const unsigned long long nchunks = (mask_end - mask_begin + chunk - 1) / chunk;
    const int pgrid = (int)std::max<unsigned long long>(1, std::min<unsigned long long>(ctx->grid[PATH_CPLX], nchunks));
    const size_t bParts = align_up(sizeof(double) * 4 * pgrid, 256);
    rc = ensure_ws_keep(ctx, end + 256 + bParts + 256, end);
    if (rc != TOR_OK)
        return rc;
    const char *dC = mat_ptr(ctx, mats[0]);
    unsigned long long *dCounter = (unsigned long long *)(ctx->ws + end);
    double *dParts = (double *)((char *)dCounter + 256);
    double *dRes = (double *)((char *)dParts + bParts);
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess)
        e = launch_zero(dCounter, 1, ctx->stream);
    PlainParams pp{};
    pp.C = dC;
    pp.n = n;
    pp.N = mats[0].N;
    pp.mask_begin = mask_begin;
    pp.mask_end = mask_end;
    pp.counter = dCounter;
    pp.partials = dParts;
    pp.chunk = chunk;
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev0, ctx->stream);
    if (e == hipSuccess)
        e = launch_plain(pp, real, pgrid, ctx->stream);
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
    fill_result(mats[0], mats[0].path, h, ms, out);
    out->subsets = mask_end - mask_begin;
    return out->status;
}

int tor_eval_removal(tor_ctx *ctx, int n, const double *O, long ld, tor_result *out)
{
    if (!ctx || !out || n < 0 || n > REMOVAL_MAX_N || !args_ok(ctx, n, O, ld))
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    // I - O in the interleaved order a_0, a_0^dag, a_1, ... (the ordering of
    // Sec. 2), the Hermitian completion of its lower triangle, packed by rows
    std::vector<StageIn> in(1);
    in[0].n = n;
    in[0].O = O;
    in[0].ld = ld;
    std::vector<Mat> mats;
    size_t end = 0;
    const unsigned sfl = (stage_flags(ctx->opt.flags) & STAGE_CHECK_HERM) | STAGE_INTERLEAVED;
    int rc = stage_sync(ctx, in, (ctx->opt.flags & TOR_INPUT_DEVICE) != 0, sfl, 0, 0, mats, &end);
    if (rc != TOR_OK)
        return rc;
    if (mats[0].status != TOR_OK)
        return mats[0].status;
    const int grid = ctx->num_cu * MAX_FIT;
    int k = 0;
    while (k < n && (1ll << k) < 4ll * grid)
        ++k;
    const size_t bParts = align_up(sizeof(double) * 4 * grid, 256);
    const long long stride = (long long)align_up(sizeof(c64) * (size_t)(n - k + 1) * (size_t)NSZ(n), 256);
    const size_t bScr = (size_t)stride * grid;
    rc = ensure_ws_keep(ctx, end + 256 + bParts + 256 + bScr, end);
    if (rc != TOR_OK)
        return rc;
    const char *dC = mat_ptr(ctx, mats[0]);
    unsigned long long *dCounter = (unsigned long long *)(ctx->ws + end);
    double *dParts = (double *)((char *)dCounter + 256);
    double *dRes = (double *)((char *)dParts + bParts);
    char *dScr = (char *)dRes + 256;
    hipError_t e = hipSetDevice(ctx->device);
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
    fill_result(mats[0], PATH_CPLX, h, ms, out);
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

int tor_debug_fma_peak(tor_ctx *ctx, int iters, double *tflops, float *ms_out)
{
    if (!ctx || !tflops || iters < 1 || iters > (1 << 20))
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    // 16 workgroups of 256 lanes per CU: every SIMD holds several waves
    const int blocks = 16 * ctx->num_cu;
    const size_t bytes = sizeof(double) * 256 * (size_t)blocks;
    int rc = ensure_ws(ctx, bytes);
    if (rc != TOR_OK)
        return rc;
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess)  // one launch to bring the clocks up, then the timed one
        e = launch_fma_peak((double *)ctx->ws, blocks, iters, ctx->stream);
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev0, ctx->stream);
    if (e == hipSuccess)
        e = launch_fma_peak((double *)ctx->ws, blocks, iters, ctx->stream);
    if (e == hipSuccess)
        e = hipEventRecord(ctx->ev1, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess)
        return hip_status(e);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    const double flop = 2.0 * FMA_PROBE_CHAINS * (double)iters * 256.0 * (double)blocks;
    *tflops = ms > 0.f ? flop / ((double)ms * 1e-3) / 1e12 : 0.0;
    if (ms_out)
        *ms_out = ms;
    return TOR_OK;
}

// ---- serving ---------------------------------------------------------------

int tor_debug_fail_root(tor_ctx *ctx, long long root, int runs)
{
    if (!ctx || runs < 0 || runs > 2)
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->dbg_root = root;
    ctx->dbg_runs = root < 0 ? 0 : runs;
    return TOR_OK;
}

int tor_submit(tor_ctx *ctx, int n, const double *O, long ld, unsigned long long *ticket)
{
    if (!ctx || !ticket || !args_ok(ctx, n, O, ld))
        return TOR_E_INVAL;
    if (request_bytes(n, stage_flags(ctx->opt.flags)) > ctx->pool_bytes)
        return TOR_E_NOMEM;
    Request *r = new (std::nothrow) Request();
    if (!r)
        return TOR_E_NOMEM;
    // a compact copy of the input; it is staged on the device at admission
    const int n2 = 2 * n;
    r->n = n;
    r->raw.resize((size_t)n2 * n2 * 2);
    if (n > 0) {
        if (ctx->opt.flags & TOR_INPUT_DEVICE) {
            hipError_t e = hipSetDevice(ctx->device);
            if (e == hipSuccess)
                e = hipMemcpy2D(r->raw.data(), sizeof(c64) * n2, O, sizeof(c64) * (size_t)ld, sizeof(c64) * n2,
                                       n2, hipMemcpyDeviceToHost);
            if (e != hipSuccess) {
                delete r;
                return hip_status(e);
            }
        } else {
            for (int a = 0; a < n2; a++)
                std::memcpy(r->raw.data() + 2 * (size_t)a * n2, O + 2 * (size_t)a * (size_t)ld, sizeof(c64) * n2);
        }
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

int tor_serve_config(tor_ctx *ctx, long long chunk_subsets, long long express_subsets, double oldest_share,
                     int max_queue)
{
    if (!ctx || chunk_subsets < 1024 || express_subsets < 0 || !(oldest_share >= 0.0 && oldest_share <= 1.0) ||
        max_queue < 1)
        return TOR_E_INVAL;
    std::lock_guard<std::mutex> g(ctx->smu);
    ctx->serve.chunk_subsets = chunk_subsets;
    ctx->serve.express_subsets = express_subsets;
    ctx->serve.oldest_share = oldest_share;
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
