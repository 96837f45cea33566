// Vector-Jacobian product of forward dynamics from the dFD outputs (Sec. IV-B:
// dqdd/du = -M^-1 dRNEA/du, dqdd/dtau = M^-1):
//   qbar = (dqdd/dq)^T g,  qdbar = (dqdd/dqd)^T g,  taubar = M^-1 g  (M^-1 symmetric).
// One thread per (knot, joint j); for a fixed row i the threads of a knot read the
// contiguous row i of each matrix.
#include <hip/hip_runtime.h>

extern "C" __global__ void __launch_bounds__(256)
grid_vjp_kernel(int nknots, int n, const float* __restrict__ dq, const float* __restrict__ dqd,
                const float* __restrict__ Minv, const float* __restrict__ g,
                float* __restrict__ qbar, float* __restrict__ qdbar, float* __restrict__ taubar)
{
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nknots * n)
        return;
    const long k = idx / n;
    const int j = (int)(idx % n);
    const long m0 = k * n * n;
    const float* gk = g + k * n;
    float sq = 0.0f, sqd = 0.0f, st = 0.0f;
    for (int i = 0; i < n; ++i) {
        const float gi = gk[i];
        const long o = m0 + (long)i * n + j;
        sq += dq[o] * gi;
        sqd += dqd[o] * gi;
        st += Minv[o] * gi;
    }
    qbar[idx] = sq;
    qdbar[idx] = sqd;
    taubar[idx] = st;
}

namespace grid_impl {

hipError_t launch_vjp(int nknots, int n, const float* dq, const float* dqd, const float* Minv,
                      const float* g, float* qbar, float* qdbar, float* taubar, hipStream_t stream)
{
    const long total = (long)nknots * n;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(grid_vjp_kernel, dim3(blocks), dim3(256), 0, stream, nknots, n, dq, dqd,
                       Minv, g, qbar, qdbar, taubar);
    return hipGetLastError();
}

}  // namespace grid_impl
