// Batched gradient of forward dynamics, CDNA4 (gfx950) device code.
//
// Compiled at model-creation time (hiprtc) behind a generated prelude that writes one
// robot's topology out as compile-time structures (grid_codegen.cpp):
//   GRID_WS_*                   staged-pipeline workspace offsets
//   Shape<s>  { B, L, parent[B], anc[B] }   a base branch shape: B bodies in local
//                               numbering, lanes per knot L, parents, strict-ancestor masks
//   Inst<k>   { using S; N; body[B]; consts(); a0() } one base branch of a robot: its shape,
//                               the robot's joint count N, the robot index of each local body,
//                               its constants as float literals (folded into the
//                               instructions) and -g, the base acceleration carrying gravity
//   grid_dispatch(args, block)  maps a workgroup to (branch, knot group) and runs it
//
// Branches hanging off the fixed base are dynamically independent: M is block diagonal
// over them, so M^-1, qdd and dqdd/du are computed branch by branch, each by its own lane
// group, and rows of other branches are zero.
//
// One workgroup is one wavefront. A branch of B bodies occupies L lanes (a power of two
// >= 2B), so a wavefront holds K = 64 / L (knot, branch) problems. Every lane keeps the
// branch's body quantities in registers and runs the shared recursions itself, so the
// tree sweeps need no cross-lane traffic; lanes differ only in the derivative column
// they own. The single exchange is the mass matrix, passed through LDS once.
//
// Per (knot, branch), all float32 (Sec. IV-B):
//   1. X_i = (E_i, r_i): E_i = E_z(q_i) E_T,i for a revolute joint; E_i = E_T,i and
//      r_i = r_T,i + q_i E_T,i^T e_z for a prismatic joint
//   2. RNEA(q, qd, 0): v_i, a_i, f_i outward, accumulated f inward; c_i = S^T f_i
//   3. column t of M as ID(q, 0, e_t) without gravity (one column per lane), LDS exchange
//   4. M = L^T L, sparse factorization along ancestor paths (no fill-in on a tree)
//   5. qdd = M^-1 (tau - c) by the two triangular solves
//   6. RNEA at qdd as the increment over step 2 (RNEA is affine in qdd); the lane keeps
//      the source terms of its own column j: (X_j v_lambda) x S = v_j x S,
//      (X_j a_lambda) x S and X_j^T (S x* f_j)
//   7. dRNEA forward (Algorithm 1) and backward pass for the lane's column (u, j)
//   8. dqdd/du_j = -M^-1 dtau/du_j and column t of M^-1 by the same solves; stores
//
// Spatial vectors are [angular; linear]; S = e_3 for a joint revolute about its z axis and
// S = e_6 for one prismatic along it (Inst::prism marks the prismatic bodies).

namespace grid {

constexpr int kConstStride = 24;   // floats of model constants per body
// body constants: [0..8] E_T (row-major), [9..11] r, [12..17] Ibar (xx yy zz xy xz yz about
// the body origin), [18..20] h = m c, [21] m

struct Args {
    int nknots;
    float* work;          // staged pipeline workspace, GRID_WS_STRIDE floats per knot
    const float* q;
    const float* qd;
    const float* tau;
    float* qdd;
    float* Minv;
    float* dqdd_dq;
    float* dqdd_dqd;
};

__device__ __forceinline__ void wave_sync()
{
    // a workgroup is exactly one wavefront: this only orders its LDS traffic
    __syncthreads();
}

// X m = [E w; E (v - r x w)]
__device__ __forceinline__ void x_mv(const float* E, const float* r, const float* m, float* y)
{
    const float t0 = m[3] - (r[1] * m[2] - r[2] * m[1]);
    const float t1 = m[4] - (r[2] * m[0] - r[0] * m[2]);
    const float t2 = m[5] - (r[0] * m[1] - r[1] * m[0]);
    y[0] = E[0] * m[0] + E[1] * m[1] + E[2] * m[2];
    y[1] = E[3] * m[0] + E[4] * m[1] + E[5] * m[2];
    y[2] = E[6] * m[0] + E[7] * m[1] + E[8] * m[2];
    y[3] = E[0] * t0 + E[1] * t1 + E[2] * t2;
    y[4] = E[3] * t0 + E[4] * t1 + E[5] * t2;
    y[5] = E[6] * t0 + E[7] * t1 + E[8] * t2;
}

// X^T f = [E^T n + r x (E^T f_l); E^T f_l]
__device__ __forceinline__ void xt_fv(const float* E, const float* r, const float* f, float* y)
{
    const float l0 = E[0] * f[3] + E[3] * f[4] + E[6] * f[5];
    const float l1 = E[1] * f[3] + E[4] * f[4] + E[7] * f[5];
    const float l2 = E[2] * f[3] + E[5] * f[4] + E[8] * f[5];
    y[0] = E[0] * f[0] + E[3] * f[1] + E[6] * f[2] + (r[1] * l2 - r[2] * l1);
    y[1] = E[1] * f[0] + E[4] * f[1] + E[7] * f[2] + (r[2] * l0 - r[0] * l2);
    y[2] = E[2] * f[0] + E[5] * f[1] + E[8] * f[2] + (r[0] * l1 - r[1] * l0);
    y[3] = l0;
    y[4] = l1;
    y[5] = l2;
}

// rigid-body inertia about the body origin: I x = [Ibar w + h x v; m v - h x w]
__device__ __forceinline__ void inertia_mv(const float* c, const float* x, float* y)
{
    const float* Ib = c + 12;
    const float* h = c + 18;
    const float m = c[21];
    y[0] = Ib[0] * x[0] + Ib[3] * x[1] + Ib[4] * x[2] + (h[1] * x[5] - h[2] * x[4]);
    y[1] = Ib[3] * x[0] + Ib[1] * x[1] + Ib[5] * x[2] + (h[2] * x[3] - h[0] * x[5]);
    y[2] = Ib[4] * x[0] + Ib[5] * x[1] + Ib[2] * x[2] + (h[0] * x[4] - h[1] * x[3]);
    y[3] = m * x[3] - (h[1] * x[2] - h[2] * x[1]);
    y[4] = m * x[4] - (h[2] * x[0] - h[0] * x[2]);
    y[5] = m * x[5] - (h[0] * x[1] - h[1] * x[0]);
}

// v x* f = [w x n + v_l x f_l; w x f_l]
__device__ __forceinline__ void crf_mv(const float* v, const float* f, float* y)
{
    y[0] = v[1] * f[2] - v[2] * f[1] + v[4] * f[5] - v[5] * f[4];
    y[1] = v[2] * f[0] - v[0] * f[2] + v[5] * f[3] - v[3] * f[5];
    y[2] = v[0] * f[1] - v[1] * f[0] + v[3] * f[4] - v[4] * f[3];
    y[3] = v[1] * f[5] - v[2] * f[4];
    y[4] = v[2] * f[3] - v[0] * f[5];
    y[5] = v[0] * f[4] - v[1] * f[3];
}

// joint i of branch I is prismatic (S = e_6) rather than revolute (S = e_3)
template <class I>
__device__ __forceinline__ constexpr bool prismatic(int i)
{
    return (I::prism >> i) & 1ull;
}

// the component S selects: angular z (revolute) or linear z (prismatic)
__device__ __forceinline__ constexpr int s_index(bool pr)
{
    return pr ? 5 : 2;
}

// (m x) S: (m_1, -m_0, 0, m_4, -m_3, 0) for S = e_3, (0, 0, 0, m_1, -m_0, 0) for S = e_6
__device__ __forceinline__ void cross_S(bool pr, const float* m, float* y)
{
    y[0] = pr ? 0.0f : m[1];
    y[1] = pr ? 0.0f : -m[0];
    y[2] = 0.0f;
    y[3] = pr ? m[1] : m[4];
    y[4] = pr ? -m[0] : -m[3];
    y[5] = 0.0f;
}

// S x* f: (-f_1, f_0, 0, -f_4, f_3, 0) for S = e_3, (-f_4, f_3, 0, 0, 0, 0) for S = e_6
__device__ __forceinline__ void s_crf(bool pr, const float* f, float* y)
{
    y[0] = pr ? -f[4] : -f[1];
    y[1] = pr ? f[3] : f[0];
    y[2] = 0.0f;
    y[3] = pr ? 0.0f : -f[4];
    y[4] = pr ? 0.0f : f[3];
    y[5] = 0.0f;
}

template <class S>
__device__ __forceinline__ constexpr bool is_anc(int a, int i)   // a strict ancestor of i
{
    return (S::anc[i] >> a) & 1ull;
}

// In place x <- (L^T L)^-1 x for the factor produced by ltl_factor (L lower triangular,
// nonzero only on ancestor paths; dinv[k] = 1 / L_kk).
template <class S>
__device__ __forceinline__ void ltl_solve(const float (&Lf)[S::B][S::B], const float (&dinv)[S::B],
                                          float (&x)[S::B])
{
    constexpr int B = S::B;
#pragma unroll
    for (int k = B - 1; k >= 0; --k) {       // x <- L^-T x
        x[k] *= dinv[k];
#pragma unroll
        for (int a = 0; a < B; ++a)
            if (is_anc<S>(a, k))
                x[a] -= Lf[k][a] * x[k];
    }
#pragma unroll
    for (int k = 0; k < B; ++k) {            // x <- L^-1 x
#pragma unroll
        for (int a = 0; a < B; ++a)
            if (is_anc<S>(a, k))
                x[k] -= Lf[k][a] * x[a];
        x[k] *= dinv[k];
    }
}

// Stages: the fused kernel runs everything; the staged pipeline splits the same steps
// over five launches with their intermediates in a device workspace (HBM).
enum Stage : int {
    kFused = 0,
    kStageRnea = 1,     // transforms, RNEA(q, qd, 0)             -> c
    kStageMinv = 2,     // transforms, M, M = L^T L               -> L, 1/L_kk, M^-1
    kStageQdd = 3,      // L, c, tau                              -> qdd
    kStageDrnea = 4,    // transforms, RNEA, RNEA at qdd, dRNEA   -> dtau/dq, dtau/dqd
    kStageFdgrad = 5,   // L, dtau                                -> dqdd/dq, dqdd/dqd
};

template <class I, int ST>
__device__ __forceinline__ void run_branch(const Args& A, int kg)
{
    using S = typename I::S;
    constexpr int B = S::B;
    constexpr int L = S::L;
    constexpr int K = 64 / L;
    constexpr int N = I::N;
    constexpr bool kFullSweeps = ST == kFused || ST == kStageRnea || ST == kStageDrnea;
    constexpr bool kNeedsX = kFullSweeps || ST == kStageMinv;
    __shared__ float s_M[K][B][B];

    const int lane = threadIdx.x;
    const int g = lane / L;                 // problem slot in the wavefront
    const int t = lane % L;                 // lane within the problem
    const int kraw = kg * K + g;
    const bool valid = kraw < A.nknots;
    const int knot = valid ? kraw : A.nknots - 1;   // tail slots recompute the last knot
    const float* C = I::consts();           // generated literals: folded into the code
    float* W = A.work + (long)knot * GRID_WS_STRIDE;   // staged pipeline only

    // lane roles: M column jm; derivative column (u, j): u = 0 -> d/dq, u = 1 -> d/dqd
    const int jm = t % B;
    const int col = t % (2 * B);
    const int u = col / B;
    const int j = col % B;
    const bool owns_col = t < 2 * B;
    const long vbase = (long)knot * N;
    const long mbase = (long)knot * N * N;

    // ------------------------------------------------------------ 1. transforms
    float qd[B], tau[B], E[B][9], R[B][3];
    if constexpr (kNeedsX) {
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const long o = vbase + I::body[i];
            const float* c = C + i * kConstStride;
            const float qi = A.q[o];
            qd[i] = A.qd[o];
            tau[i] = A.tau[o];
            if (prismatic<I>(i)) {
                // translation along the joint z axis: E = E_T, r = r_T + q E_T^T e_z
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    E[i][k] = c[k];
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    R[i][k] = c[9 + k] + qi * c[6 + k];
                continue;
            }
            // sin and cos by the hardware units (angle in revolutions, reduced to [0, 1))
            const float rev = __builtin_amdgcn_fractf(qi * 0.159154943091895336f);
            const float s = __builtin_amdgcn_sinf(rev);
            const float co = __builtin_amdgcn_cosf(rev);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                E[i][k] = co * c[k] + s * c[3 + k];
                E[i][3 + k] = co * c[3 + k] - s * c[k];
                E[i][6 + k] = c[6 + k];
                R[i][k] = c[9 + k];
            }
        }
    }
    const float a0[6] = {0.0f, 0.0f, 0.0f, I::a0()[0], I::a0()[1], I::a0()[2]};   // -g
    const float zero6[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};

    // ------------------------------------------------------------ 2. RNEA(q, qd, 0)
    // v_i, a_i, f_i outward (f accumulated inward below); gamma_i = I_i v_i is kept for
    // the derivative sweep, and the lane keeps v_j and X_j a_lambda(j) of its own column
    float v[B][6], F[B][6], gam[B][6];
    float av[6], ab[6];
    float x[B];                                   // tau - c, then qdd
    if constexpr (kFullSweeps) {
        float a[B][6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            av[k] = 0.0f;
            ab[k] = 0.0f;
        }
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const int p = S::parent[i];
            const float* c = C + i * kConstStride;
            float xv[6], xa[6], vxs[6], Ia[6], w[6];
            x_mv(E[i], R[i], p < 0 ? zero6 : v[p < 0 ? 0 : p], xv);
            x_mv(E[i], R[i], p < 0 ? a0 : a[p < 0 ? 0 : p], xa);
            xv[s_index(prismatic<I>(i))] += qd[i];
            cross_S(prismatic<I>(i), xv, vxs);
            const bool mine = i == j;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                v[i][k] = xv[k];
                a[i][k] = xa[k] + vxs[k] * qd[i];
                av[k] = mine ? xv[k] : av[k];
                ab[k] = mine ? xa[k] : ab[k];
            }
            inertia_mv(c, v[i], gam[i]);
            inertia_mv(c, a[i], Ia);
            crf_mv(v[i], gam[i], w);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                F[i][k] = Ia[k] + w[k];
        }
#pragma unroll
        for (int i = B - 1; i >= 0; --i) {
            const int p = S::parent[i];
            if (p >= 0) {
                float y[6];
                xt_fv(E[i], R[i], F[i], y);
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    F[p][k] += y[k];
            }
        }
#pragma unroll
        for (int i = 0; i < B; ++i)
            x[i] = tau[i] - F[i][s_index(prismatic<I>(i))];   // tau - c
        if constexpr (ST == kStageRnea) {
            if (valid && t < B) {
#pragma unroll
                for (int i = 0; i < B; ++i)
                    if (t == i)
                        W[GRID_WS_C + I::body[i]] = F[i][s_index(prismatic<I>(i))];
            }
            return;
        }
    }

    // ------------------------------------------------------------ 3-4. M = L^T L
    float Lf[B][B], dinv[B];
    if constexpr (ST == kFused || ST == kStageMinv) {
        // column jm of M as ID(q, 0, e_jm) without gravity, exchanged through LDS
        {
            float am[B][6], fm[B][6];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const int p = S::parent[i];
                const float* c = C + i * kConstStride;
                if (p >= 0)
                    x_mv(E[i], R[i], am[p < 0 ? 0 : p], am[i]);
                else
#pragma unroll
                    for (int k = 0; k < 6; ++k)
                        am[i][k] = 0.0f;
                am[i][s_index(prismatic<I>(i))] += (i == jm) ? 1.0f : 0.0f;
                inertia_mv(c, am[i], fm[i]);
            }
#pragma unroll
            for (int i = B - 1; i >= 0; --i) {
                const int p = S::parent[i];
                if (p >= 0) {
                    float y[6];
                    xt_fv(E[i], R[i], fm[i], y);
#pragma unroll
                    for (int k = 0; k < 6; ++k)
                        fm[p][k] += y[k];
                }
            }
            if (t < B) {
#pragma unroll
                for (int i = 0; i < B; ++i)
                    s_M[g][i][t] = fm[i][s_index(prismatic<I>(i))];
            }
        }
        wave_sync();
#pragma unroll
        for (int i = 0; i < B; ++i)
#pragma unroll
            for (int b = 0; b <= i; ++b)
                if (b == i || is_anc<S>(b, i))
                    Lf[i][b] = s_M[g][i][b];
        // sparse factorisation along ancestor paths: for k from the leaves,
        // L_kk = sqrt(M_kk), L_ka = M_ka / L_kk, M_ab -= L_ka L_kb (a, b ancestors of k)
#pragma unroll
        for (int k = B - 1; k >= 0; --k) {
            const float di = __builtin_amdgcn_rsqf(Lf[k][k]);   // 1 / L_kk
            dinv[k] = di;
#pragma unroll
            for (int b = 0; b < B; ++b)
                if (is_anc<S>(b, k))
                    Lf[k][b] *= di;
#pragma unroll
            for (int a2 = 0; a2 < B; ++a2)
                if (is_anc<S>(a2, k))
#pragma unroll
                    for (int b = 0; b < B; ++b)
                        if (b == a2 || is_anc<S>(b, a2))
                            Lf[a2][b] -= Lf[k][a2] * Lf[k][b];
        }
    } else if constexpr (ST == kStageQdd || ST == kStageFdgrad) {
        const float* Wl = W + GRID_WS_L + I::loff;
#pragma unroll
        for (int i = 0; i < B; ++i) {
            dinv[i] = W[GRID_WS_DINV + I::body[i]];
#pragma unroll
            for (int b = 0; b < B; ++b)
                if (is_anc<S>(b, i))
                    Lf[i][b] = Wl[i * B + b];
        }
    }

    // ------------------------------------------------------------ M^-1 and the factor
    if constexpr (ST == kFused || ST == kStageMinv) {
        float mc[B];                              // column jm of M^-1
#pragma unroll
        for (int i = 0; i < B; ++i)
            mc[i] = (i == jm) ? 1.0f : 0.0f;
        ltl_solve<S>(Lf, dinv, mc);
        if (valid) {
#pragma unroll
            for (int i = 0; i < B; ++i) {
                // entry (i, jm) with i <= jm is written to both mirrored positions by the
                // lane owning column jm, so M^-1 comes out exactly symmetric
                if (t < B && i <= jm) {
                    const int gi = I::body[i];
                    const int gj = I::body_of(jm);
                    A.Minv[mbase + (long)gi * N + gj] = mc[i];
                    A.Minv[mbase + (long)gj * N + gi] = mc[i];
                }
            }
            if (N > B) {
                for (int e = t; e < B * N; e += L) {
                    const int i = e / N, c2 = e % N;
                    if (!I::contains(c2))
                        A.Minv[mbase + (long)I::body_of(i) * N + c2] = 0.0f;
                }
            }
        }
        if constexpr (ST == kStageMinv) {
            if (valid && t == 0) {
                float* Wl = W + GRID_WS_L + I::loff;
#pragma unroll
                for (int i = 0; i < B; ++i) {
                    W[GRID_WS_DINV + I::body[i]] = dinv[i];
#pragma unroll
                    for (int b = 0; b < B; ++b)
                        if (is_anc<S>(b, i))
                            Wl[i * B + b] = Lf[i][b];
                }
            }
            return;
        }
    }

    // ------------------------------------------------------------ 5. qdd
    if constexpr (ST == kFused || ST == kStageQdd) {
        if constexpr (ST == kStageQdd) {
#pragma unroll
            for (int i = 0; i < B; ++i)
                x[i] = A.tau[vbase + I::body[i]] - W[GRID_WS_C + I::body[i]];
        }
        ltl_solve<S>(Lf, dinv, x);
        if (valid) {
#pragma unroll
            for (int i = 0; i < B; ++i)
                if (t == i)
                    A.qdd[vbase + I::body[i]] = x[i];
        }
        if constexpr (ST == kStageQdd)
            return;
    }
    if constexpr (ST == kStageDrnea) {
#pragma unroll
        for (int i = 0; i < B; ++i)
            x[i] = A.qdd[vbase + I::body[i]];
    }

    float dx[B];                                  // dtau/du_j, then dqdd/du_j
    if constexpr (kFullSweeps) {
        // -------------------------------------------------------- 6. RNEA at qdd
        // RNEA is affine in qdd: a_i(qdd) = a_i(0) + Da_i and f_i(qdd) = f_i(0) + Df_i,
        // Da_i = X_i Da_lambda + S qdd_i (Da_0 = 0), Df_i = I_i Da_i accumulated inward
        float Fj[6], Ej[9], rj[3];
        {
            float Da[B][6], Df[B][6];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const int p = S::parent[i];
                const float* c = C + i * kConstStride;
                float xd[6];
                if (p >= 0)
                    x_mv(E[i], R[i], Da[p < 0 ? 0 : p], xd);
                else
#pragma unroll
                    for (int k = 0; k < 6; ++k)
                        xd[k] = 0.0f;
                const bool mine = i == j;
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    Da[i][k] = xd[k];
                    ab[k] = mine ? ab[k] + xd[k] : ab[k];      // X_j a_lambda(j) at qdd
                }
                Da[i][s_index(prismatic<I>(i))] += x[i];
                inertia_mv(c, Da[i], Df[i]);
            }
#pragma unroll
            for (int i = B - 1; i >= 0; --i) {
                const int p = S::parent[i];
                if (p >= 0) {
                    float y[6];
                    xt_fv(E[i], R[i], Df[i], y);
#pragma unroll
                    for (int k = 0; k < 6; ++k)
                        Df[p][k] += y[k];
                }
            }
#pragma unroll
            for (int k = 0; k < 6; ++k)
                Fj[k] = 0.0f;
#pragma unroll
            for (int k = 0; k < 9; ++k)
                Ej[k] = 0.0f;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                rj[k] = 0.0f;
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const bool mine = i == j;
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    Fj[k] = mine ? F[i][k] + Df[i][k] : Fj[k];
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    Ej[k] = mine ? E[i][k] : Ej[k];
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    rj[k] = mine ? R[i][k] : rj[k];
            }
        }
        // source terms of column (u, j):
        //   u = q : dv += (X_j v_lambda) x S = v_j x S,  da += (X_j a_lambda) x S,
        //           backward += X_j^T (S x* f_j)
        //   u = qd: dv += S,                             da += v_j x S
        float src_v[6], src_a[6], src_f[6];
        {
            const bool pj = (I::prism >> j) & 1ull;        // joint j is prismatic
            float vxs[6], axs[6], sf[6];
            cross_S(pj, av, vxs);
            cross_S(pj, ab, axs);
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                src_v[k] = u == 0 ? vxs[k] : (k == s_index(pj) ? 1.0f : 0.0f);
                src_a[k] = u == 0 ? axs[k] : vxs[k];
            }
            s_crf(pj, Fj, sf);                                   // S x* f
            xt_fv(Ej, rj, sf, src_f);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                src_f[k] = u == 0 ? src_f[k] : 0.0f;
        }

        // -------------------------------------------------------- 7. dRNEA column (u, j)
        float df[B][6];
        {
            float dv[B][6], da[B][6];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const int p = S::parent[i];
                const float* c = C + i * kConstStride;
                const float sel = (i == j) ? 1.0f : 0.0f;
                float xdv[6], xda[6];
                if (p >= 0) {
                    x_mv(E[i], R[i], dv[p < 0 ? 0 : p], xdv);
                    x_mv(E[i], R[i], da[p < 0 ? 0 : p], xda);
                } else {
#pragma unroll
                    for (int k = 0; k < 6; ++k) {
                        xdv[k] = 0.0f;
                        xda[k] = 0.0f;
                    }
                }
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    dv[i][k] = xdv[k] + sel * src_v[k];
                float dvxs[6];
                cross_S(prismatic<I>(i), dv[i], dvxs);
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    da[i][k] = xda[k] + dvxs[k] * qd[i] + sel * src_a[k];
                // df_i = I_i da_i + dv_i x* gamma_i + v_i x* (I_i dv_i)
                float t1[6], t2[6], t3[6], Idv[6];
                inertia_mv(c, da[i], t1);
                crf_mv(dv[i], gam[i], t2);
                inertia_mv(c, dv[i], Idv);
                crf_mv(v[i], Idv, t3);
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    df[i][k] = t1[k] + t2[k] + t3[k];
            }
        }
#pragma unroll
        for (int i = B - 1; i >= 0; --i) {
            dx[i] = df[i][s_index(prismatic<I>(i))];
            const int p = S::parent[i];
            if (p >= 0) {
                const float sel = (i == j) ? 1.0f : 0.0f;
                float y[6];
                xt_fv(E[i], R[i], df[i], y);
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    df[p][k] += y[k] + sel * src_f[k];
            }
        }
        if constexpr (ST == kStageDrnea) {
            if (valid && owns_col) {
                float* Wd = W + GRID_WS_DTAU + u * N * N;
                const int gj = I::body_of(j);
#pragma unroll
                for (int i = 0; i < B; ++i)
                    Wd[I::body[i] * N + gj] = dx[i];
            }
            return;
        }
    }
    if constexpr (ST == kStageFdgrad) {
        const float* Wd = W + GRID_WS_DTAU + u * N * N;
        const int gj = I::body_of(j);
#pragma unroll
        for (int i = 0; i < B; ++i)
            dx[i] = Wd[I::body[i] * N + gj];
    }

    // ------------------------------------------------------------ 8. -M^-1 dtau/du_j
    if constexpr (ST == kFused || ST == kStageFdgrad) {
        ltl_solve<S>(Lf, dinv, dx);
        if (!valid)
            return;
        if (owns_col) {
            float* out = u == 0 ? A.dqdd_dq : A.dqdd_dqd;
            const int gj = I::body_of(j);
#pragma unroll
            for (int i = 0; i < B; ++i)
                out[mbase + (long)I::body[i] * N + gj] = -dx[i];
        }
        if (N > B) {
            // this branch's rows hold zeros in the other branches' columns
            for (int e = t; e < B * N; e += L) {
                const int i = e / N, c2 = e % N;
                if (!I::contains(c2)) {
                    const long o = mbase + (long)I::body_of(i) * N + c2;
                    A.dqdd_dq[o] = 0.0f;
                    A.dqdd_dqd[o] = 0.0f;
                }
            }
        }
    }
}

}  // namespace grid

using namespace grid;

// kernels of a one-robot module (a module of several robots defines GRID_PIPE_ONLY and its
// own entry point, grid_fdgrad_pipe_mixed)
#ifndef GRID_PIPE_ONLY

// defined by the generated epilogue: workgroup -> (branch, knot group)
template <int ST>
__device__ void grid_dispatch(const Args& args, int block);

// Three builds of the fused kernel differ only in the register budget the compiler may
// use: 1, 2 or 4 resident wavefronts per SIMD (more registers and no spills, or more
// wavefronts to hide latency at large N). The autotuner picks one per batch size.
extern "C" __global__ void __launch_bounds__(64) grid_fdgrad_fused(Args args)
{
    grid_dispatch<kFused>(args, (int)blockIdx.x);
}

extern "C" __global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2)))
grid_fdgrad_fused_w2(Args args)
{
    grid_dispatch<kFused>(args, (int)blockIdx.x);
}

extern "C" __global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4)))
grid_fdgrad_fused_w4(Args args)
{
    grid_dispatch<kFused>(args, (int)blockIdx.x);
}

extern "C" __global__ void __launch_bounds__(64) grid_stage_rnea(Args args)
{
    grid_dispatch<kStageRnea>(args, (int)blockIdx.x);
}

extern "C" __global__ void __launch_bounds__(64) grid_stage_minv(Args args)
{
    grid_dispatch<kStageMinv>(args, (int)blockIdx.x);
}

extern "C" __global__ void __launch_bounds__(64) grid_stage_qdd(Args args)
{
    grid_dispatch<kStageQdd>(args, (int)blockIdx.x);
}

extern "C" __global__ void __launch_bounds__(64) grid_stage_drnea(Args args)
{
    grid_dispatch<kStageDrnea>(args, (int)blockIdx.x);
}

extern "C" __global__ void __launch_bounds__(64) grid_stage_fdgrad(Args args)
{
    grid_dispatch<kStageFdgrad>(args, (int)blockIdx.x);
}

#endif  // GRID_PIPE_ONLY
