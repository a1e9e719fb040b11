// pj_probe.hip -- known-work microbenchmarks that calibrate the roofline
// peaks used to report the refinement kernel's efficiency: scalar
// (non-packed) FP32 FMA issue rate and FP64 FMA rate.
#include "pj_internal.h"

namespace pj {

template <class T>
__global__ __launch_bounds__(256) void k_fma_probe(T *out, T x, T y, int iters)
{
    T a0 = (T)threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;
    for (int i = 0; i < iters; ++i) {
        a0 = a0 * x + y;
        a1 = a1 * x + y;
        a2 = a2 * x + y;
        a3 = a3 * x + y;
        a4 = a4 * x + y;
        a5 = a5 * x + y;
        a6 = a6 * x + y;
        a7 = a7 * x + y;
    }
    out[blockIdx.x * 256 + threadIdx.x] = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
}

hipError_t launch_fma_probe(int fp64, void *out, int blocks, int iters, hipStream_t st)
{
    if (fp64)
        hipLaunchKernelGGL(k_fma_probe<double>, dim3(blocks), dim3(256), 0, st, (double *)out, 0.999999, 1e-7, iters);
    else
        hipLaunchKernelGGL(k_fma_probe<float>, dim3(blocks), dim3(256), 0, st, (float *)out, 0.999999f, 1e-7f, iters);
    return hipGetLastError();
}

// plain streaming copy (16-byte vectors): calibrates the HBM byte counters
__global__ __launch_bounds__(256) void k_copy_probe(const float4 *__restrict__ src, float4 *__restrict__ dst, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
}

hipError_t launch_copy_probe(const void *src, void *dst, int64_t nbytes, int blocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy_probe, dim3(blocks), dim3(256), 0, st, (const float4 *)src, (float4 *)dst, nbytes / 16);
    return hipGetLastError();
}

}  // namespace pj
