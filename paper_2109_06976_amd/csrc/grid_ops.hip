// The paper's other algorithms as kernels of their own (Sec. IV-B), quad layout (gfx950):
//   grid_op_id      tau = ID(q, qd, qdd) = RNEA                      one quad per problem
//   grid_op_fd      qdd = FD(q, qd, tau) = M^-1 (tau - c)            one quad per column of M
//   grid_op_minv    M^-1                                             one quad per column of M
//   grid_op_idgrad  dtau/dq, dtau/dqd at the given qdd (Algorithm 1  one quad per derivative
//                   forward pass and the backward pass)              column
// A (knot, branch) problem uses the building blocks of the fused kernels; M comes from
// unit-acceleration columns and its sparse L^T L factor, as there.

namespace gridq {

enum Op : int { kOpId = 0, kOpFd = 1, kOpMinv = 2, kOpIdGrad = 3 };

struct OpArgs {
    int nknots;
    const float* q;
    const float* qd;      // unused by grid_op_minv
    const float* u;       // qdd (ID, dID), tau (FD), unused (M^-1)
    float* out0;          // tau (ID), qdd (FD), M^-1 (M^-1), dtau/dq (dID)
    float* out1;          // dtau/dqd (dID)
};

// problems (knot, branch) per workgroup
template <class S, int OP>
__device__ __forceinline__ constexpr int op_problems()
{
    return OP == kOpId ? 16
           : OP == kOpIdGrad ? (GRID_WAVES / S::W) * (16 / S::Q)
                             : PipeShape<S::B>::P;
}

template <class I, int OP>
__device__ __forceinline__ void run_op(const OpArgs& A, int block)
{
    using S = typename I::S;
    constexpr int B = S::B;
    constexpr int N = GRID_N;
    constexpr int P = op_problems<S, OP>();
    constexpr int Q = OP == kOpId ? 1
                      : OP == kOpIdGrad ? S::Q
                                        : PipeShape<B>::QB;   // quads per problem per wavefront
    constexpr int W = OP == kOpIdGrad ? S::W : 1;             // wavefronts per problem
    __shared__ float s_M[OP == kOpFd || OP == kOpMinv ? P : 1][B][B];

    const int tid = (int)threadIdx.x;
    const int wave = tid / 64;
    const int lane = tid % 64;
    const int c = lane & 3;
    const Lane ln = lane_of(c == 3 ? 0 : c);
    const int quad = (lane / 4) % Q;
    const int pslot = (wave / W) * (16 / Q) + (lane / 4) / Q;
    const int s = quad + Q * (wave % W);
    const int kraw = block * P + pslot;
    const bool valid = kraw < A.nknots;
    const int knot = valid ? kraw : A.nknots - 1;           // tail slots recompute the last knot
    const long vbase = (long)knot * N;
    const long mbase = (long)knot * N * N;

    float qd[B];
    Rot E[B];
    LaneK K[B];
    load_bodies<I, OP != kOpMinv>(A.q, A.qd, vbase, ln, qd, E, K);

    if constexpr (OP == kOpId || OP == kOpIdGrad) {
        float qdd[B];
#pragma unroll
        for (int i = 0; i < B; ++i)
            qdd[i] = A.u[vbase + I::body[i]];
        V v[B], gam[B], F[B], xa[B];
        rnea_at<I>(ln, qd, qdd, E, K, v, gam, F, xa);
        if constexpr (OP == kOpId) {
            if (valid) {
#pragma unroll
                for (int i = 0; i < B; ++i) {
                    const float tau = qperm<kZ>(F[i].a);
                    if ((i & 3) == c)
                        A.out0[vbase + I::body[i]] = tau;
                }
            }
        } else {
            // column (u, j) of the quad: u = 0 -> d/dq_j, u = 1 -> d/dqd_j
            const bool owns_col = s < 2 * B;
            const int u = owns_col ? s / B : 1;
            const int j = s % B;
            Rot Ej;
            LaneK Kj;
            pick_joint<I>(E, K, j, Ej, Kj);
            const V vxs = cross_s(ln, pick<B>(v, j));
            const V src_v = u == 0 ? vxs : V{ln.sz, 0.0f};
            const V src_a = u == 0 ? cross_s(ln, pick<B>(xa, j)) : vxs;
            const V zeta = back_source(ln, Ej, Kj, pick<B>(F, j));
            const V src_f = u == 0 ? zeta : V{0.0f, 0.0f};
            float dx[B];
            drnea_column<I, true>(ln, qd, E, K, v, gam, j, src_v, src_a, src_f, dx);
            if (!valid)
                return;
            if (owns_col) {
                float* out = u == 0 ? A.out0 : A.out1;
                const int gj = I::body_of(j);
#pragma unroll
                for (int i = 0; i < B; ++i)
                    if ((i & 3) == c)
                        out[mbase + (long)I::body[i] * N + gj] = dx[i];
            }
            zero_fill<I>(A.out0, A.out1, mbase, lane % (4 * Q) + 64 * (wave % W), 4 * Q * W);
        }
    } else {
        // FD and M^-1: the columns of M, exchanged inside the wavefront, and the factor
        constexpr int CB = PipeShape<B>::CB;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const bool owns = s + 16 * cb < B;
            const int jm = owns ? s + 16 * cb : 0;
            V fm[B];
            m_column<I>(ln, E, K, jm, fm);
            if (owns && c == 2) {
#pragma unroll
                for (int i = 0; i < B; ++i)
                    s_M[pslot][i][jm] = fm[i].a;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float Lf[B][B], dinv[B];
#pragma unroll
        for (int i = 0; i < B; ++i)
#pragma unroll
            for (int b = 0; b <= i; ++b)
                if (b == i || is_anc<S>(b, i))
                    Lf[i][b] = s_M[pslot][i][b];
        ltl_factor<S>(Lf, dinv);
        if constexpr (OP == kOpMinv) {
            minv_columns<I, CB, P, false>(A.out0, Lf, dinv, pslot, s, c, valid, mbase,
                                          lane % (4 * Q), 4 * Q, s_M);
        } else {
            V v[B], gam[B], F[B], xa0[B];
            rnea0<I>(ln, qd, E, K, v, gam, F, xa0);
            float x[B];
#pragma unroll
            for (int i = 0; i < B; ++i)
                x[i] = A.u[vbase + I::body[i]] - qperm<kZ>(F[i].a);
            ltl_solve<S>(Lf, dinv, x);
            if (valid && s == 0) {
#pragma unroll
                for (int i = 0; i < B; ++i)
                    if ((i & 3) == c)
                        A.out0[vbase + I::body[i]] = x[i];
            }
        }
    }
}

}  // namespace gridq

// defined by the generated epilogue: workgroup -> (branch, problem group)
template <int OP>
__device__ void grid_dispatch_op(const gridq::OpArgs& args, int block);

extern "C" __global__ void __launch_bounds__(64) grid_op_id(gridq::OpArgs args)
{
    grid_dispatch_op<gridq::kOpId>(args, (int)blockIdx.x);
}

extern "C" __global__ void __launch_bounds__(64) grid_op_fd(gridq::OpArgs args)
{
    grid_dispatch_op<gridq::kOpFd>(args, (int)blockIdx.x);
}

extern "C" __global__ void __launch_bounds__(64) grid_op_minv(gridq::OpArgs args)
{
    grid_dispatch_op<gridq::kOpMinv>(args, (int)blockIdx.x);
}

extern "C" __global__ void __launch_bounds__(64 * GRID_WAVES) grid_op_idgrad(gridq::OpArgs args)
{
    grid_dispatch_op<gridq::kOpIdGrad>(args, (int)blockIdx.x);
}
