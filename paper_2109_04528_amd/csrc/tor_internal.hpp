// tor_internal.hpp -- structures shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tor {

// complex128 as two doubles (16-byte aligned -> 128-bit loads)
struct __align__(16) c64 {
    double x, y;  // re, im
};

// real double-double: the unevaluated sum hi + lo, |lo| <= ulp(hi) / 2
struct __align__(16) ddr {
    double hi, lo;
};

// Device layout of a node of s modes: the Hermitian (or real symmetric)
// 2s x 2s matrix in mode-interleaved rows, REVERSED (the next mode to decide
// owns the two highest rows), cut into its lower-triangular 2x2 mode blocks
// (a, b), a >= b, numbered a(a+1)/2 + b.  Each block has 4 entries
// e = 0..3: (2a,2b), (2a,2b+1), (2a+1,2b), (2a+1,2b+1) (a diagonal block keeps
// its upper entry as the conjugate of the lower one).  The entries of a block
// form 16-byte granules (two real entries, or one complex entry), and the
// node stores granule g of every block as one array, then granule g+1:
// neighbouring lanes that work on neighbouring blocks touch neighbouring
// 16-byte words.  Dropping the highest mode leaves the first blocks of every
// granule array, so an exclude child is a view of its parent that keeps the
// parent's block count nb as the array stride.
__host__ __device__ constexpr int NB(int s) { return s * (s + 1) / 2; }        // blocks
__host__ __device__ constexpr int NSZ(int s) { return 2 * s * (s + 1); }       // scalars
__host__ __device__ constexpr int bidx(int a, int b) { return a * (a + 1) / 2 + b; }
// entries per 16-byte granule for scalars of sz bytes
__host__ __device__ constexpr int EPG(int sz) { return 16 / sz; }
// scalar index of entry e of block bi in a node whose granule arrays have nb
// blocks
__host__ __device__ constexpr int gpos(int sz, int nb, int bi, int e)
{
    return EPG(sz) * ((e / EPG(sz)) * nb + bi) + e % EPG(sz);
}
// packed lower triangle (registers of the per-lane tail): entry (x, y), y <= x
__host__ __device__ constexpr int E(int s) { return s * (2 * s + 1); }
__host__ __device__ constexpr int pidx(int x, int y) { return x * (x + 1) / 2 + y; }

// One matrix (or a contiguous range of its subtree roots) in a launch.
struct ProblemDesc {
    const void *C;         // device layout of I - O (c64 or double), N modes
    double *slots;         // this matrix's partial slots, 4 doubles per root
    int N;                 // modes after padding (>= R of the kernel)
    int k;                 // split depth: 2^k subtree roots in total
    long long root_begin;  // first root handled by this launch
    long long item_begin;  // queue item of that root in this launch
    long long nroots;      // roots handled by this launch
};

struct MainParams {
    const ProblemDesc *probs;
    int nprob;
    long long total_items;
    unsigned long long *counter;  // queue head, zero before the launch
    char *scratch;                // per-wave stack of the upper include levels
    long long scratch_stride;     // bytes per wave
    long long fail_item1;         // debug: 1 + the queue item whose root reports a
                                  // numeric failure (0: none)
    double *terms;                // every-term launch (one matrix, all roots): the
                                  // signed term of each subset, indexed by subset
                                  // (bit N-1-l = decision at level l); else null
};
// root slot flag (fourth double): a tested pivot failed (I - O is not
// positive definite), or the root's sum is not finite (a numeric failure,
// which the host may re-run); the per-matrix reduction keeps the largest
constexpr double SLOT_NOT_PD = 1.0;
constexpr double SLOT_NUMERIC = 0.5;

struct PlainParams {
    const void *C;                // packed reversed matrix of N modes
    int n;                        // modes of the problem: subsets are masks below 2^n
    int N;                        // modes of the staged form (N >= n; modes n.. are padding)
    unsigned long long mask_begin, mask_end;
    unsigned long long *counter;  // chunk queue head
    double *partials;             // 4 doubles per wave
    int chunk;                    // subsets per queue pop
};

// The removal-order comparison kernel (Algorithm 2): one wave per depth-first
// walk over the removals of the modes k..n-1 below a root (the removal
// decisions on modes 0..k-1).
struct RemovalParams {
    const void *C;                // I - O (c64), interleaved rows, lower triangle packed by pidx
    int n, k;
    unsigned long long *counter;  // root queue head
    char *scratch;                // per wave: levels 0..n-k of NSZ(n) c64 each
    long long scratch_stride;     // bytes per wave
    double *partials;             // 4 doubles per wave
};
constexpr int REMOVAL_MAX_N = 34;

// Device staging (tor_stage.hip): one workgroup per matrix turns the
// caller's O into the layout a kernel reads.
enum : unsigned {
    STAGE_CHECK_HERM = 1u,   // the upper triangle must mirror the lower one
    STAGE_FORCE_CPLX = 2u,   // never the real quadrature form
    STAGE_DD = 4u,           // the real form in double-double (structure required)
    STAGE_INTERLEAVED = 8u,  // the removal-order layout (complex, interleaved rows)
};
constexpr int STAGE_BAD_INPUT = 1;  // a value is not finite, or a required test failed

struct StageInfo {
    int status;   // 0, or STAGE_BAD_INPUT
    int path;     // PATH_* of the staged form
    int N;        // its modes (after padding)
    int unused;
    double cmax;  // max |I - O|
};

struct StageDesc {
    const double *O;   // complex128 row-major (re, im), leading dimension ld
    long ld;           // in complex elements
    const int *sel;    // null, or the n modes (increasing) of an M-mode O
    int n, M;
    unsigned flags;    // STAGE_*
    int min_cplx;      // minimum modes of the complex form
    void *out;         // the staged form (bytes: staged_bytes)
    StageInfo *info;
};

// sum_{i=1..s} 2i(i+1): scalars of all node sizes 1..s
__host__ __device__ constexpr long long Gsum(long long s) { return s <= 0 ? 0 : 2 * s * (s + 1) * (s + 2) / 3; }

// Per-wave stack of a matrix of N modes split at depth k, for a kernel that
// finishes the last R modes in LDS and registers (LA = N - R tier-A levels):
//  * the root node, NSZ(N) scalars: the final root node of N-k modes with
//    its own stride NB(N-k) when the root path ran in LDS, or the node
//    eliminated in place with the matrix's stride NB(N) (an include step
//    only rewrites blocks of the modes that remain, each by the lane that
//    reads it);
//  * tier-A slots l = k+1 .. LA-1, slot l holding a node of N - l modes with
//    its own stride NB(N - l) (the real path keeps level LA-1 in LDS and
//    leaves slot LA-1 unused);
//  * the running determinants of the tier-A levels (LA + 1 real values).
// Scalar offset of tier-A slot l (also of the determinants, at l = LA).
__host__ __device__ constexpr long long tslot_off(int N, int k, int l)
{
    return NSZ(N) + (Gsum(N - k - 1) - Gsum(N - l));
}
// bytes of the stack for scalars of esz bytes and real values of rsz bytes
__host__ __device__ constexpr long long stack_bytes(int N, int k, int R, int esz, int rsz)
{
    const int LA = N - R > 0 ? N - R : 0;
    const long long slots = k < LA ? tslot_off(N, k, LA) : (long long)NSZ(N);
    return esz * slots + (long long)rsz * (LA + 1);
}

// kernel configurations (modes handled per lane, levels expanded in LDS)
// T: modes a lane finishes alone; B: levels between the tier-A leaf and the
// lanes (2^B = 64 lanes); L: the last of those levels taken by each lane in
// registers (the first B - L are expanded in LDS).
constexpr int CPLX_T = 3;
constexpr int CPLX_B = 6;
constexpr int CPLX_L = 2;
constexpr int CPLX_R = CPLX_T + CPLX_B;
constexpr int REAL_T = 5;
constexpr int REAL_B = 6;
constexpr int REAL_L = 2;
constexpr int REAL_R = REAL_T + REAL_B;
// double-double factor (real quadrature form only)
constexpr int QUAD_T = 3;
constexpr int QUAD_B = 6;
constexpr int QUAD_L = 2;
constexpr int QUAD_R = QUAD_T + QUAD_B;

// kernel paths: general Hermitian input, the real quadrature form of a
// Gaussian-state matrix, and that form with a double-double factor
enum { PATH_CPLX = 0, PATH_REAL = 1, PATH_QUAD = 2, NPATH = 3 };
constexpr int MAX_N = 48;
constexpr int MAX_FIT = 8;  // persistent one-wave workgroups per CU, at most

// host-side launchers (defined in tor_kernels.hip unless noted)
hipError_t launch_main(int path, bool dd, const MainParams &p, int grid, hipStream_t s);
// the real-path kernel that stores every term (p.terms) instead of summing
hipError_t launch_main_store(const MainParams &p, int grid, hipStream_t s);
int main_store_occupancy();
// exact double-double subset sums g[S] = sum over Z subset of S of t[Z], for
// the 2^nbits terms t (tor_zeta.hip)
hipError_t launch_zeta(const double *t, ddr *g, int nbits, hipStream_t s);
// per click pattern S of M modes (bit i = API mode i) of a staged form of N
// modes: Tor(O_S) = (-1)^(N-|S|) g[S reversed over N bits], and optionally
// p(S) = Tor(O_S) sqrt(det(I - O)) (tor_zeta.hip)
hipError_t launch_click_out(const ddr *g, int N, int M, const double *sqrt_det, double *probs, double *tor_hi,
                            double *tor_lo, hipStream_t s);
hipError_t launch_reduce(const ProblemDesc *probs, int nprob, double *results, bool dd, hipStream_t s);
hipError_t launch_zero(unsigned long long *p, int count, hipStream_t s);
hipError_t launch_plain(const PlainParams &p, bool real, int grid, hipStream_t s);
hipError_t launch_removal(const RemovalParams &p, int grid, hipStream_t s);
hipError_t launch_plain_reduce(const double *partials, int nwaves, double *result, hipStream_t s);
hipError_t launch_math_probe(const double *x, double *out, int count, hipStream_t s);
// FP64 FMA throughput probe: blocks x 256 lanes, iters x 16 FMAs each
hipError_t launch_fma_peak(double *out, int blocks, int iters, hipStream_t s);
constexpr int FMA_PROBE_CHAINS = 16;
// defined in tor_stage.hip
hipError_t launch_stage(const StageDesc *descs, int count, hipStream_t s);
hipError_t launch_sqrt_det(const double *O, long ld, int M, c64 *scratch, double *out, hipStream_t s);
// resident one-wave workgroups of the main kernel per CU (0 on error)
int main_occupancy(int path);
// the double-double factor's main kernel and its occupancy, used by the two
// above for PATH_QUAD (tor_kernels_quad.hip)
hipError_t launch_main_quad(const MainParams &p, int grid, hipStream_t s);
int main_occupancy_quad();

}  // namespace tor
