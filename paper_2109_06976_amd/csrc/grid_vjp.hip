// Kernels that consume the dFD outputs (robot independent, built into the library).
//
// Vector-Jacobian product of forward dynamics (Sec. IV-B: dqdd/du = -M^-1 dRNEA/du,
// dqdd/dtau = M^-1):
//   qbar = (dqdd/dq)^T g,  qdbar = (dqdd/dqd)^T g,  taubar = M^-1 g  (M^-1 symmetric).
// One thread per (knot, joint j); for a fixed row i the threads of a knot read the
// contiguous row i of each matrix.
//
// Jacobians of one semi-implicit Euler step, the discrete-time dynamics of trajectory
// optimisation: qd' = qd + dt qdd(q, qd, tau), q' = q + dt qd', x = (q, qd):
//   A = dx'/dx   = [[1 + dt^2 Dq, dt 1 + dt^2 Dqd], [dt Dq, 1 + dt Dqd]]   [2n][2n]
//   B = dx'/dtau = [[dt^2 M^-1], [dt M^-1]]                               [2n][n]
// with Dq = dqdd/dq, Dqd = dqdd/dqd. One thread per entry of A and B (6 n^2 per knot),
// consecutive threads writing consecutive entries.
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

extern "C" __global__ void __launch_bounds__(256)
grid_dt_kernel(int nknots, int n, float dt, const float* __restrict__ dq,
               const float* __restrict__ dqd, const float* __restrict__ Minv,
               float* __restrict__ A, float* __restrict__ B)
{
    const long per = 6L * n * n;                 // 4 n^2 entries of A, then 2 n^2 of B
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nknots * per)
        return;
    const long k = idx / per;
    const long e = idx % per;
    const long m0 = k * n * n;
    const float dt2 = dt * dt;
    if (e < 4L * n * n) {
        const int r = (int)(e / (2 * n)), c = (int)(e % (2 * n));
        const int i = r % n, j = c % n;
        const bool top = r < n, left = c < n;
        const float d = left ? dq[m0 + (long)i * n + j] : dqd[m0 + (long)i * n + j];
        const float eye = (i == j) ? 1.0f : 0.0f;
        float v;
        if (top)
            v = left ? eye + dt2 * d : dt * eye + dt2 * d;
        else
            v = left ? dt * d : eye + dt * d;
        A[k * 4L * n * n + e] = v;
    } else {
        const long f = e - 4L * n * n;
        const int r = (int)(f / n), j = (int)(f % n);
        const int i = r % n;
        const float mi = Minv[m0 + (long)i * n + j];
        B[k * 2L * n * n + f] = (r < n ? dt2 : dt) * mi;
    }
}

namespace grid_impl {

hipError_t launch_dt(int nknots, int n, float dt, const float* dq, const float* dqd,
                     const float* Minv, float* A, float* B, hipStream_t stream)
{
    const long total = (long)nknots * 6L * n * n;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(grid_dt_kernel, dim3(blocks), dim3(256), 0, stream, nknots, n, dt, dq,
                       dqd, Minv, A, B);
    return hipGetLastError();
}

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
