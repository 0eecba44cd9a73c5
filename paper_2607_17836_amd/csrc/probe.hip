// Achievable-bandwidth probe: a plain streaming copy and a STREAM-style
// triad over device buffers, timed with HIP events.  Used to state how far
// the step kernel is from what the memory system delivers in practice, and
// as the known-size reference that calibrates hardware byte counters.
#include "lpt_kernels.h"

namespace lpt {

__global__ __launch_bounds__(256) void copy_kernel(const float4 *__restrict__ a,
                                                   float4 *__restrict__ b, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        b[i] = a[i];
}

__global__ __launch_bounds__(256) void triad_kernel(const float4 *__restrict__ b,
                                                    const float4 *__restrict__ c,
                                                    float4 *__restrict__ a, float s, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float4 x = b[i], y = c[i];
        a[i] = make_float4(x.x + s * y.x, x.y + s * y.y, x.z + s * y.z, x.w + s * y.w);
    }
}

hipError_t launch_copy(const void *src, void *dst, int64_t bytes, hipStream_t st)
{
    const int64_t n = bytes / 16;
    const int b = 256;
    const int64_t g = (n + b - 1) / b;
    const unsigned grid = (unsigned)(g < 65536 * 8 ? g : 65536 * 8);
    hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(b), 0, st, (const float4 *)src,
                       (float4 *)dst, n);
    return hipGetLastError();
}

hipError_t launch_triad(const void *b_, const void *c_, void *a_, int64_t bytes, hipStream_t st)
{
    const int64_t n = bytes / 16;
    const int b = 256;
    const int64_t g = (n + b - 1) / b;
    const unsigned grid = (unsigned)(g < 65536 * 8 ? g : 65536 * 8);
    hipLaunchKernelGGL(triad_kernel, dim3(grid), dim3(b), 0, st, (const float4 *)b_,
                       (const float4 *)c_, (float4 *)a_, 1.5f, n);
    return hipGetLastError();
}

}  // namespace lpt
