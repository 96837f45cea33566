// The paper's other algorithms as kernels of their own (Sec. IV-B), quad layout (gfx950):
//   grid_op_id      tau = ID(q, qd, qdd) = RNEA                      one quad per problem
//   grid_op_fd      qdd = FD(q, qd, tau) = M^-1 (tau - c)            one quad per column of M
//   grid_op_minv    M^-1                                             one quad per column of M
//   grid_op_idgrad  dtau/dq, dtau/dqd at the given qdd (Algorithm 1  one quad per derivative
//                   forward pass and the backward pass)              column
//   grid_op_vjp     the vector-Jacobian product of FD without its     one quad per column of M
//                   Jacobians: taubar = M^-1 g, qbar = -(dtau/dq)^T taubar,
//                   qdbar = -(dtau/dqd)^T taubar, by one reverse sweep over RNEA
// A (knot, branch) problem uses the building blocks of the fused kernels; M comes from
// unit-acceleration columns and its sparse L^T L factor, as there.

namespace gridq {

enum Op : int { kOpId = 0, kOpFd = 1, kOpMinv = 2, kOpIdGrad = 3, kOpVjp = 4 };

struct OpArgs {
    int nknots;
    const float* q;
    const float* qd;      // unused by grid_op_minv
    const float* u;       // qdd (ID, dID, VJP), tau (FD), unused (M^-1)
    const float* u2;      // g (VJP)
    float* out0;          // tau (ID), qdd (FD), M^-1 (M^-1), dtau/dq (dID), qbar (VJP)
    float* out1;          // dtau/dqd (dID), qdbar (VJP)
    float* out2;          // taubar (VJP)
};

// v x m = [w x w'; w x v' + v x w'] (motion cross product)
__device__ __forceinline__ V crm(Nb v, Nb m)
{
    V y;
    y.a = v.a1 * m.a2 - v.a2 * m.a1;
    y.l = v.a1 * m.l2 - v.a2 * m.l1 + v.l1 * m.a2 - v.l2 * m.a1;
    return y;
}

// f . m over the six components: the quad's lanes 0..2 hold one pair each
__device__ __forceinline__ float dot6(V f, V m)
{
    const float p = f.a * m.a + f.l * m.l;
    return p + qperm<kNb1>(p) + qperm<kNb2>(p);
}

// Reverse sweep for w^T dtau/dq and w^T dtau/dqd at (q, qd, qdd), w given per joint. With
// the virtual displacement u_i = X_i u_lambda + S w_i, w^T tau = sum_i u_i . f_i (f_i the
// body's own force I_i a_i + v_i x* I_i v_i), and dX_i/dq_i = -(S x) X_i. Adjoints, leaves
// to root: ub_i = f_i + sum_c X_c^T ub_c (the accumulated force), ab_i = I_i u_i +
// sum_c X_c^T ab_c, vb_i = I_i (u_i x v_i) - u_i x* (I_i v_i) + (S x* ab_i) qd_i +
// sum_c X_c^T vb_c; then
//   w^T dtau/dq_i  = -(ub_i . (S x X_i u_lambda) + vb_i . (S x X_i v_lambda)
//                      + ab_i . (S x X_i a_lambda))
//   w^T dtau/dqd_i = vb_i . S + ab_i . (v_i x S)
template <class I>
__device__ __forceinline__ void drnea_adjoint(const Lane& ln, const float (&qd)[I::S::B],
                                              const float (&qdd)[I::S::B], const float (&w)[I::S::B],
                                              const Rot (&E)[I::S::B], const LaneK (&K)[I::S::B],
                                              float (&gq)[I::S::B], float (&gqd)[I::S::B])
{
    using S = typename I::S;
    constexpr int B = S::B;
    V v[B], u[B], xv[B], xa[B], xu[B], ub[B], ab[B], vb[B];
    {
        V a[B];
        Nb nv[B], na[B], nu[B];
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const int p = S::parent[i];
            if (p >= 0) {
                xv[i] = xmv(E[i], K[i], v[p < 0 ? 0 : p], nv[p < 0 ? 0 : p]);
                xa[i] = xmv(E[i], K[i], a[p < 0 ? 0 : p], na[p < 0 ? 0 : p]);
                xu[i] = xmv(E[i], K[i], u[p < 0 ? 0 : p], nu[p < 0 ? 0 : p]);
            } else {
                const V g{0.0f, ln.g};
                xv[i] = V{0.0f, 0.0f};
                xa[i] = xmv(E[i], K[i], g, gather(g));
                xu[i] = V{0.0f, 0.0f};
            }
            const bool pr = prismatic<I>(i);
            v[i] = add_s(ln, pr, xv[i], qd[i]);
            nv[i] = gather(v[i]);
            const V vxs = cross_s(ln, pr, v[i]);
            const V xs = add_s(ln, pr, xa[i], qdd[i]);
            a[i] = V{xs.a + vxs.a * qd[i], xs.l + vxs.l * qd[i]};
            na[i] = gather(a[i]);
            u[i] = add_s(ln, pr, xu[i], w[i]);
            nu[i] = gather(u[i]);
            const float m = mass<I>(i);
            const V Iv = imv(K[i], m, v[i], nv[i]);
            ub[i] = add(imv(K[i], m, a[i], na[i]), crf(nv[i], gather(Iv)));
            ab[i] = imv(K[i], m, u[i], nu[i]);
            const V uxv = crm(nu[i], nv[i]);
            vb[i] = add(imv(K[i], m, uxv, gather(uxv)), neg(crf(nu[i], gather(Iv))));
        }
    }
#pragma unroll
    for (int i = B - 1; i >= 0; --i) {
        const bool pr = prismatic<I>(i);
        const V sxab = s_crf(ln, pr, ab[i]);                // S x* ab_i
        vb[i] = V{vb[i].a + sxab.a * qd[i], vb[i].l + sxab.l * qd[i]};
        // S x y = -(y x S)
        gq[i] = -(dot6(ub[i], neg(cross_s(ln, pr, xu[i]))) +
                  dot6(vb[i], neg(cross_s(ln, pr, xv[i]))) +
                  dot6(ab[i], neg(cross_s(ln, pr, xa[i]))));
        gqd[i] = qperm<kZ>(s_half(pr, vb[i])) + dot6(ab[i], cross_s(ln, pr, v[i]));
        const int p = S::parent[i];
        if (p >= 0) {
            ub[p < 0 ? 0 : p] = add(ub[p < 0 ? 0 : p], xtfv(E[i], K[i], ub[i], gather(ub[i])));
            ab[p < 0 ? 0 : p] = add(ab[p < 0 ? 0 : p], xtfv(E[i], K[i], ab[i], gather(ab[i])));
            vb[p < 0 ? 0 : p] = add(vb[p < 0 ? 0 : p], xtfv(E[i], K[i], vb[i], gather(vb[i])));
        }
    }
}

// problems (knot, branch) per workgroup
template <class S, int OP>
__device__ __forceinline__ constexpr int op_problems()
{
    return OP == kOpId ? 16
           : OP == kOpIdGrad ? (GRID_WAVES / S::W) * (16 / S::Q)
                             : PipeShape<S::B>::P;   // FD, M^-1, VJP
}

template <class I, int OP>
__device__ __forceinline__ void run_op(const OpArgs& A, int block)
{
    using S = typename I::S;
    constexpr int B = S::B;
    constexpr int N = I::N;
    constexpr int P = op_problems<S, OP>();
    constexpr int Q = OP == kOpId ? 1
                      : OP == kOpIdGrad ? S::Q
                                        : PipeShape<B>::QB;   // quads per problem per wavefront
    constexpr int W = OP == kOpIdGrad ? S::W : 1;             // wavefronts per problem
    __shared__ float s_M[OP == kOpFd || OP == kOpMinv || OP == kOpVjp ? P : 1][B][B];
    __shared__ float4 s_tab[3 * B * 4];

    const int tid = (int)threadIdx.x;
    const int wave = tid / 64;
    const int lane = tid % 64;
    const int c = lane & 3;
    const Lane ln = lane_of(c == 3 ? 0 : c, I::a0());
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
    const float* tab = lane_table<I, OP == kOpIdGrad ? 64 * GRID_WAVES : 64>(s_tab, tid, c);
    load_bodies<I, OP != kOpMinv>(A.q, A.qd, vbase, ln, tab, qd, E, K);

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
                    const float tau = qperm<kZ>(s_half(prismatic<I>(i), F[i]));
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
            const bool pj = prismatic<I>(j);
            const V vxs = cross_s(ln, pj, pick<B>(v, j));
            const V src_v = u == 0 ? vxs : s_vec(ln, pj, 1.0f);
            const V src_a = u == 0 ? cross_s(ln, pj, pick<B>(xa, j)) : vxs;
            const V zeta = back_source(ln, pj, Ej, Kj, pick<B>(F, j));
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
                    s_M[pslot][i][jm] = s_half(prismatic<I>(i), fm[i]);
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
        } else if constexpr (OP == kOpVjp) {
            float lam[B], qdd[B], gq[B], gqd[B];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                lam[i] = A.u2[vbase + I::body[i]];
                qdd[i] = A.u[vbase + I::body[i]];
            }
            ltl_solve<S>(Lf, dinv, lam);      // taubar = M^-1 g (this branch's block)
            drnea_adjoint<I>(ln, qd, qdd, lam, E, K, gq, gqd);
            if (valid && s == 0) {
#pragma unroll
                for (int i = 0; i < B; ++i)
                    if ((i & 3) == c) {
                        const long o = vbase + I::body[i];
                        A.out0[o] = -gq[i];
                        A.out1[o] = -gqd[i];
                        A.out2[o] = lam[i];
                    }
            }
        } else {
            V v[B], gam[B], F[B], xa0[B];
            rnea0<I>(ln, qd, E, K, v, gam, F, xa0);
            float x[B];
#pragma unroll
            for (int i = 0; i < B; ++i)
                x[i] = A.u[vbase + I::body[i]] - qperm<kZ>(s_half(prismatic<I>(i), F[i]));
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

// kernels of a one-robot module (a module of several robots defines GRID_PIPE_ONLY and its
// own entry point, grid_fdgrad_pipe_mixed)
#ifndef GRID_PIPE_ONLY

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

extern "C" __global__ void __launch_bounds__(64) grid_op_vjp(gridq::OpArgs args)
{
    grid_dispatch_op<gridq::kOpVjp>(args, (int)blockIdx.x);
}

#endif  // GRID_PIPE_ONLY
