// tor_internal.hpp -- structures shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tor {

// complex128 as two doubles (16-byte aligned -> 128-bit loads)
struct __align__(16) c64 {
    double x, y;  // re, im
};

__host__ __device__ constexpr int E(int s) { return s * (2 * s + 1); }  // packed entries, s modes
__host__ __device__ constexpr int pidx(int x, int y) { return x * (x + 1) / 2 + y; }

// One matrix in a launch.
struct ProblemDesc {
    const void *C;         // packed reversed Hermitian (c64) or symmetric (double) matrix, N modes
    int N;                 // modes after padding (>= R of the kernel)
    int k;                 // split depth: 2^k subtree roots
    long long item_begin;  // first queue item (= first partial slot) of this matrix
};

struct MainParams {
    const ProblemDesc *probs;
    int nprob;
    long long total_items;
    unsigned long long *counter;  // queue head, zero before the launch
    double *slots;                // 4 doubles per item: hi, lo, sum|t|, numeric-failure flag
    char *scratch;                // per-wave stack of the upper include levels
    long long scratch_stride;     // bytes per wave
};

struct PlainParams {
    const void *C;                // packed reversed matrix, n modes (no padding)
    int n;
    unsigned long long mask_begin, mask_end;
    unsigned long long *counter;  // chunk queue head
    double *partials;             // 4 doubles per wave
    int chunk;                    // subsets per queue pop
};

// sum_{i=1..s} i(2i+1): packed entries of all node sizes 1..s
__host__ __device__ constexpr long long Fsum(long long s) { return s * (s + 1) * (4 * s + 5) / 6; }
// entry offset of Tier-A stack slot l (covers modes [l, N)), slots 1..N-R
__host__ __device__ constexpr long long slot_off(int N, int l) { return Fsum(N - 1) - Fsum(N - l); }

// kernel configurations (modes handled per lane, levels expanded in LDS)
constexpr int CPLX_T = 3;
constexpr int CPLX_B = 6;
constexpr int CPLX_R = CPLX_T + CPLX_B;
constexpr int REAL_T = 4;
constexpr int REAL_B = 6;
constexpr int REAL_R = REAL_T + REAL_B;
constexpr int MAX_N = 48;

// host-side launchers (defined in tor_kernels.hip)
hipError_t launch_main(bool real_path, bool dd, const MainParams &p, int grid, hipStream_t s);
hipError_t launch_reduce(const ProblemDesc *probs, int nprob, const double *slots, double *results,
                         bool dd, hipStream_t s);
hipError_t launch_zero(unsigned long long *p, int count, hipStream_t s);
hipError_t launch_plain(const PlainParams &p, int grid, hipStream_t s);
hipError_t launch_plain_reduce(const double *partials, int nwaves, double *result, hipStream_t s);
hipError_t launch_math_probe(const double *x, double *out, int count, hipStream_t s);
int main_lds_bytes(bool real_path);

}  // namespace tor
