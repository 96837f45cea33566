// Copy kernel of the mapped host call (grid_fd_grad_mapped): moves the packed outputs from
// device memory into pinned host memory through its device mapping, so that the transfer is
// a kernel's stores over the host link rather than a copy-engine job (whose start-up latency
// dominates transfers of the few hundred kilobytes a batch of knots produces).
//
// Each thread moves 16 bytes per step (dwordx4 load and store) over a grid-stride loop; the
// tail of n mod 4 floats is moved one float per thread by the first threads.
#include <hip/hip_runtime.h>

#include "grid_internal.h"

extern "C" __global__ void __launch_bounds__(256)
grid_copy_out_kernel(const float4* __restrict__ src, float4* __restrict__ dst, long n4,
                     const float* __restrict__ src_tail, float* __restrict__ dst_tail, int tail)
{
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        dst[i] = src[i];
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t < tail)
        dst_tail[t] = src_tail[t];
}

namespace grid_impl {

hipError_t launch_copy_out(const float* src, float* dst, size_t n, hipStream_t stream)
{
    // both buffers start 16-byte aligned (device allocation, pinned host allocation)
    const long n4 = (long)(n / 4);
    const int tail = (int)(n % 4);
    long blocks = (n4 + 255) / 256;
    if (blocks < 1)
        blocks = 1;
    if (blocks > 1024)
        blocks = 1024;
    hipLaunchKernelGGL(grid_copy_out_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                       reinterpret_cast<const float4*>(src), reinterpret_cast<float4*>(dst), n4,
                       src + 4 * n4, dst + 4 * n4, tail);
    return hipGetLastError();
}

}  // namespace grid_impl
