// Stand-ins for the library's kernel launchers, for the CPU build of its host
// runtime (tests/schedsim).  Each one queues host work on the stream in the
// place of the kernel.  The staging stand-in puts the first real part of the
// input into the staged form and takes an input as a Gaussian state's (real
// quadrature path, N = max(n, REAL_R)) unless the imaginary part of its first
// entry is positive (then general Hermitian input: the complex path, N =
// max(n, min_cplx)); the recursive stand-in gives
// root r of a matrix of N modes split at depth k the slot (c 2^(N-k), 0,
// 2^(N-k), 0), c that staged value, so a matrix's sum is c 2^N whatever its
// split, and every root counts once: a root run twice or not at all, or a
// slot of another request, changes it.  A launch sleeps for its subsets at
// SCHEDSIM_RATE subsets per second (default 2e10), so that launches overlap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <thread>

#include "../../paper_2109_04528_amd/csrc/tor_internal.hpp"

namespace tor {

namespace {
double rate()
{
    static const double r = [] {
        const char *e = std::getenv("SCHEDSIM_RATE");
        const double v = e ? std::atof(e) : 2e10;
        return v > 0 ? v : 2e10;
    }();
    return r;
}
void pause_for(double subsets)
{
    const double us = 1e6 * subsets / rate();
    if (us >= 1.0)
        std::this_thread::sleep_for(std::chrono::microseconds((long long)us));
}
}  // namespace

int main_occupancy(int path) { return path == PATH_REAL ? 8 : 7; }
int main_store_occupancy() { return 8; }

hipError_t launch_stage(const StageDesc *descs, int count, hipStream_t s)
{
    fake_enqueue(s, [=] {
        for (int i = 0; i < count; i++) {
            const StageDesc &D = descs[i];
            double c = 0.0;
            bool general = false;
            if (D.O && D.n > 0) {
                c = D.O[0];
                general = D.O[1] > 0.0;
            }
            const bool cplx = (D.flags & STAGE_FORCE_CPLX) != 0 || (general && !(D.flags & STAGE_DD));
            if (D.out)
                std::memcpy(D.out, &c, sizeof c);
            D.info->status = (std::isfinite(c) ? 0 : STAGE_BAD_INPUT);
            D.info->path = cplx ? PATH_CPLX : ((D.flags & STAGE_DD) ? PATH_QUAD : PATH_REAL);
            const int R = cplx ? std::max(D.min_cplx, 0) : ((D.flags & STAGE_DD) ? QUAD_R : REAL_R);
            D.info->N = std::max(D.n, R);
            D.info->cmax = 1.0;
        }
    });
    return hipSuccess;
}

hipError_t launch_main(int, bool, const MainParams &p, int grid, hipStream_t s)
{
    if (grid <= 0)
        return hipErrorInvalidValue;
    const MainParams mp = p;
    fake_enqueue(s, [mp] {
        double work = 0.0;
        for (int i = 0; i < mp.nprob; i++) {
            const ProblemDesc &d = mp.probs[i];
            double c;
            std::memcpy(&c, d.C, sizeof c);
            const double per = std::ldexp(1.0, d.N - d.k);
            for (long long r = d.root_begin; r < d.root_begin + d.nroots; r++) {
                double *sl = d.slots + 4 * r;
                sl[0] = c * per;
                sl[1] = 0.0;
                sl[2] = per;
                sl[3] = 0.0;
            }
            work += per * (double)d.nroots;
        }
        pause_for(work);
    });
    return hipSuccess;
}

hipError_t launch_main_store(const MainParams &p, int grid, hipStream_t s) { return launch_main(PATH_REAL, false, p, grid, s); }

hipError_t launch_reduce(const ProblemDesc *probs, int nprob, double *results, bool, hipStream_t s)
{
    fake_enqueue(s, [=] {
        for (int j = 0; j < nprob; j++) {
            const ProblemDesc &d = probs[j];
            double h = 0.0, ab = 0.0, bad = 0.0;
            for (long long r = 0; r < (1ll << d.k); r++) {
                h += d.slots[4 * r];
                ab += d.slots[4 * r + 2];
                bad = std::max(bad, d.slots[4 * r + 3]);
            }
            results[4 * j] = h;
            results[4 * j + 1] = 0.0;
            results[4 * j + 2] = ab;
            results[4 * j + 3] = bad;
        }
    });
    return hipSuccess;
}

hipError_t launch_zero(unsigned long long *p, int count, hipStream_t s)
{
    fake_enqueue(s, [=] { std::memset(p, 0, sizeof(unsigned long long) * (size_t)count); });
    return hipSuccess;
}

// not used by serving: no work
hipError_t launch_zeta(const double *, ddr *, int, hipStream_t) { return hipSuccess; }
hipError_t launch_click_out(const ddr *, int, int, const double *, double *, double *, double *, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_plain(const PlainParams &, bool, int, hipStream_t) { return hipSuccess; }
hipError_t launch_removal(const RemovalParams &, int, hipStream_t) { return hipSuccess; }
hipError_t launch_plain_reduce(const double *, int, double *, hipStream_t) { return hipSuccess; }
hipError_t launch_math_probe(const double *, double *, int, hipStream_t) { return hipSuccess; }
hipError_t launch_fma_peak(double *, int, int, hipStream_t) { return hipSuccess; }
hipError_t launch_sqrt_det(const double *, long, int, c64 *, double *, hipStream_t) { return hipSuccess; }

}  // namespace tor
