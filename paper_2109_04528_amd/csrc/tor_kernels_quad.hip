// tor_kernels_quad.hip -- the double-double factor's main kernel
// (Algorithm 2 and Eq. 2 with every step in double-double arithmetic, the
// extended-precision evaluation of Sec. 5), instantiated in a translation
// unit of its own.
//
// The kernel template is the one in tor_kernels.hip, included here without
// that file's launchers and plain kernels, so that this unit can be compiled
// with its own code-generation options: the library builds it with the
// AMDGPU scheduler's register-pressure trackers (-mllvm
// -amdgpu-use-amdgpu-trackers), which schedule this kernel about 4 % faster
// (n = 30: 22.6 against 23.6 ms, the same results bit for bit) but the FP64
// kernels no faster.
#define TOR_KERNELS_TEMPLATES_ONLY
#include "tor_kernels.hip"

namespace tor {

hipError_t launch_main_quad(const MainParams &p, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((tor_main<ddr, QUAD_T, QUAD_B, QUAD_L, AccQ>), dim3(grid), dim3(64), 0, s, p);
    return hipGetLastError();
}

int main_occupancy_quad()
{
    int n = 0;
    const hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, tor_main<ddr, QUAD_T, QUAD_B, QUAD_L, AccQ>, 64, 0);
    return e == hipSuccess ? n : 0;
}

}  // namespace tor
