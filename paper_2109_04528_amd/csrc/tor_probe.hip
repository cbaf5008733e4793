// tor_probe.hip -- measurement aids: the accuracy of the device reciprocal
// and reciprocal square root as the kernels form them, and the device's FP64
// FMA throughput (the peak the roofline is quoted against).
#include "tor_device.hpp"
#include "tor_internal.hpp"

namespace tor {

// FP64 FMA throughput: FMA_PROBE_CHAINS independent FMA chains per lane, so
// that the vector unit, not the latency of one chain, sets the rate.  Each
// lane's sum is stored so that no chain is removed.
__global__ void __launch_bounds__(256) tor_fma_peak(double *out, int iters)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    double a[FMA_PROBE_CHAINS];
#pragma unroll
    for (int j = 0; j < FMA_PROBE_CHAINS; ++j)
        a[j] = 1.0 + 1e-3 * (double)((g + j) & 255);
    const double m = 1.0 + 1e-9, c = 1e-12;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < FMA_PROBE_CHAINS; ++j)
            a[j] = fma(a[j], m, c);
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < FMA_PROBE_CHAINS; ++j)
        s += a[j];
    out[g] = s;
}

// accuracy probe of the device reciprocal / reciprocal square root
__global__ void tor_math_probe(const double *x, double *out, int count)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        out[4 * i] = rsqrt_nr(x[i]);
        out[4 * i + 1] = rcp_nr(x[i]);
        out[4 * i + 2] = __builtin_amdgcn_rsq(x[i]);
        out[4 * i + 3] = __builtin_amdgcn_rcp(x[i]);
    }
}

hipError_t launch_fma_peak(double *out, int blocks, int iters, hipStream_t s)
{
    hipLaunchKernelGGL(tor_fma_peak, dim3(blocks), dim3(256), 0, s, out, iters);
    return hipGetLastError();
}

hipError_t launch_math_probe(const double *x, double *out, int count, hipStream_t s)
{
    hipLaunchKernelGGL(tor_math_probe, dim3((count + 63) / 64), dim3(64), 0, s, x, out, count);
    return hipGetLastError();
}

}  // namespace tor
