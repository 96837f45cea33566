// Batched gradient of forward dynamics, CDNA4 (gfx950) device code.
//
// This file is compiled at model-creation time (hiprtc) behind a generated prelude that
// fixes one robot's topology as compile-time tables (see grid_codegen.cpp):
//   GRID_N, GRID_L, GRID_NLEV, GRID_NROUND, GRID_MAXANC, GRID_DYN_DOUBLE,
//   kParent[n], kBranch[n], kLevelMask[NLEV], kRoundMask[NROUND].
// Every loop over bodies is unrolled against those tables, so a kernel is one robot's
// kinematic tree written out (the paper's code generation, Sec. IV-C).
//
// One workgroup is one wavefront (64 lanes) and holds K = 64 / GRID_L knots; each knot
// owns GRID_L lanes and a private LDS slice. Because a workgroup is a single wavefront,
// the level-by-level sweeps synchronise with a wave barrier only.
//
// Per knot (paper Sec. IV-B):
//   1. X_i(q_i) = (E_i, r_i) with E_i = E_z(q_i) E_T,i                  [lanes = bodies]
//   2. RNEA(q, qd, 0) outward by tree level, f_i, inward by rounds -> c  [lanes = bodies]
//      composite inertias (CRBA) ride along the same inward rounds
//   3. M from the composite inertias, each lane walking its ancestors    [lanes = columns]
//   4. M^-1 by in-place Gauss-Jordan (M is SPD: no pivoting)             [lanes = entries]
//   5. qdd = M^-1 (tau - c)                                              [lanes = rows]
//   6. RNEA at qdd: a_i, f_i and the column-independent temporaries of Algorithm 2
//      (alpha_i = v_i x S, beta_i = (X_i a_lambda) x S, gamma_i = I_i v_i, and the
//      backward source zeta_i = X_i^T (S x* f_i))                        [lanes = bodies]
//   7. dRNEA forward and backward pass, one derivative column per lane   [lanes = 2n columns]
//   8. dqdd/du = -M^-1 dtau/du for the lane's column; stores             [lanes = columns]
// Steps 1-6 run in DT (double when GRID_DYN_DOUBLE: M can be ill-conditioned); the
// derivative sweeps 7-8, the bulk of the arithmetic, run in float.
//
// Spatial vectors are [angular; linear]; S = e_3 (revolute about the joint z axis).

#ifndef GRID_N
#error "GRID_N must be defined by the generated prelude"
#endif

namespace grid {

constexpr int N = GRID_N;
constexpr int L = GRID_L;              // lanes per knot
constexpr int K = 64 / GRID_L;         // knots per wavefront
constexpr int NN = N * N;
constexpr int kBodyStride = 24;        // doubles of model constants per body
// body constant layout: [0..8] E_T (row-major), [9..11] r, [12..17] Ibar (xx yy zz xy xz yz
// about the body origin), [18..20] h = m c, [21] m

#if GRID_DYN_DOUBLE
typedef double DT;
#else
typedef float DT;
#endif

struct Args {
    const double* model;   // N * kBodyStride
    double a0[3];          // linear part of the base acceleration, -g
    int nknots;
    const float* q;
    const float* qd;
    const float* tau;
    float* qdd;
    float* Minv;
    float* dqdd_dq;
    float* dqdd_dqd;
};

struct KnotLds {
    DT E[N][9];
    DT r[N][3];
    DT v[N][6];
    DT a[N][6];
    DT F[N][6];
    DT IC[N][10];          // composite inertia: m, h[3], Ibar[6]
    DT M[N][N];            // M, then M^-1 in place
    DT qd[N];
    DT tmc[N];             // tau - c
    DT qdd[N];
    float Ef[N][12];       // E (9) and r (3) in float
    float vf[N][6];
    float gam[N][6];       // gamma_i = I_i v_i
    float alpha[N][6];     // alpha_i = v_i x S
    float beta[N][6];      // beta_i = (X_i a_lambda) x S
    float zeta[N][6];      // X_i^T (S x* f_i)
    float qdf[N];
    float minvf[N][N];
};

__device__ __forceinline__ void wave_sync()
{
    // the workgroup is exactly one wavefront: this orders LDS traffic within it
    __syncthreads();
}

template <class T>
__device__ __forceinline__ void x_mv(const T* E, const T* r, const T* m, T* y)
{
    // X m = [E w; E (v - r x w)]
    const T t0 = m[3] - (r[1] * m[2] - r[2] * m[1]);
    const T t1 = m[4] - (r[2] * m[0] - r[0] * m[2]);
    const T t2 = m[5] - (r[0] * m[1] - r[1] * m[0]);
    y[0] = E[0] * m[0] + E[1] * m[1] + E[2] * m[2];
    y[1] = E[3] * m[0] + E[4] * m[1] + E[5] * m[2];
    y[2] = E[6] * m[0] + E[7] * m[1] + E[8] * m[2];
    y[3] = E[0] * t0 + E[1] * t1 + E[2] * t2;
    y[4] = E[3] * t0 + E[4] * t1 + E[5] * t2;
    y[5] = E[6] * t0 + E[7] * t1 + E[8] * t2;
}

template <class T>
__device__ __forceinline__ void xt_fv(const T* E, const T* r, const T* f, T* y)
{
    // X^T f = [E^T n + r x (E^T f_l); E^T f_l]
    const T l0 = E[0] * f[3] + E[3] * f[4] + E[6] * f[5];
    const T l1 = E[1] * f[3] + E[4] * f[4] + E[7] * f[5];
    const T l2 = E[2] * f[3] + E[5] * f[4] + E[8] * f[5];
    const T n0 = E[0] * f[0] + E[3] * f[1] + E[6] * f[2];
    const T n1 = E[1] * f[0] + E[4] * f[1] + E[7] * f[2];
    const T n2 = E[2] * f[0] + E[5] * f[1] + E[8] * f[2];
    y[0] = n0 + (r[1] * l2 - r[2] * l1);
    y[1] = n1 + (r[2] * l0 - r[0] * l2);
    y[2] = n2 + (r[0] * l1 - r[1] * l0);
    y[3] = l0;
    y[4] = l1;
    y[5] = l2;
}

template <class T>
__device__ __forceinline__ void inertia_mv(const T* Ib, const T* h, T m, const T* x, T* y)
{
    // I x = [Ibar w + h x v; m v - h x w]
    y[0] = Ib[0] * x[0] + Ib[3] * x[1] + Ib[4] * x[2] + (h[1] * x[5] - h[2] * x[4]);
    y[1] = Ib[3] * x[0] + Ib[1] * x[1] + Ib[5] * x[2] + (h[2] * x[3] - h[0] * x[5]);
    y[2] = Ib[4] * x[0] + Ib[5] * x[1] + Ib[2] * x[2] + (h[0] * x[4] - h[1] * x[3]);
    y[3] = m * x[3] - (h[1] * x[2] - h[2] * x[1]);
    y[4] = m * x[4] - (h[2] * x[0] - h[0] * x[2]);
    y[5] = m * x[5] - (h[0] * x[1] - h[1] * x[0]);
}

template <class T>
__device__ __forceinline__ void crf_mv(const T* v, const T* f, T* y)
{
    // v x* f = [w x n + v_l x f_l; w x f_l]
    y[0] = v[1] * f[2] - v[2] * f[1] + v[4] * f[5] - v[5] * f[4];
    y[1] = v[2] * f[0] - v[0] * f[2] + v[5] * f[3] - v[3] * f[5];
    y[2] = v[0] * f[1] - v[1] * f[0] + v[3] * f[4] - v[4] * f[3];
    y[3] = v[1] * f[5] - v[2] * f[4];
    y[4] = v[2] * f[3] - v[0] * f[5];
    y[5] = v[0] * f[4] - v[1] * f[3];
}

// (m x) S for S = e_3
template <class T>
__device__ __forceinline__ void cross_S(const T* m, T* y)
{
    y[0] = m[1];
    y[1] = -m[0];
    y[2] = 0;
    y[3] = m[4];
    y[4] = -m[3];
    y[5] = 0;
}

// Composite inertia update IC_p += X^T IC_i X for rigid-body inertias kept as
// (m, h, Ibar): h' = E^T h + m r,
// Ibar' = E^T Ibar E + (m|r|^2 + 2 r.y) 1 - m r r^T - y r^T - r y^T, y = E^T h.
__device__ __forceinline__ void inertia_to_parent(const DT* E, const DT* r, const DT* ic, DT* out)
{
    const DT m = ic[0];
    const DT* h = ic + 1;
    const DT* I = ic + 4;   // xx yy zz xy xz yz
    const DT Ib[9] = {I[0], I[3], I[4], I[3], I[1], I[5], I[4], I[5], I[2]};
    DT y[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        y[a] = E[0 * 3 + a] * h[0] + E[1 * 3 + a] * h[1] + E[2 * 3 + a] * h[2];
    DT B[9];   // Ibar E
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            B[a * 3 + b] = Ib[a * 3 + 0] * E[0 * 3 + b] + Ib[a * 3 + 1] * E[1 * 3 + b] +
                           Ib[a * 3 + 2] * E[2 * 3 + b];
    DT C[9];   // E^T B (symmetric)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b)
            C[a * 3 + b] = E[0 * 3 + a] * B[0 * 3 + b] + E[1 * 3 + a] * B[1 * 3 + b] +
                           E[2 * 3 + a] * B[2 * 3 + b];
    const DT ry = r[0] * y[0] + r[1] * y[1] + r[2] * y[2];
    const DT rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const DT d = m * rr + 2 * ry;
    out[0] += m;
    out[1] += y[0] + m * r[0];
    out[2] += y[1] + m * r[1];
    out[3] += y[2] + m * r[2];
    out[4] += C[0] + d - m * r[0] * r[0] - 2 * y[0] * r[0];
    out[5] += C[4] + d - m * r[1] * r[1] - 2 * y[1] * r[1];
    out[6] += C[8] + d - m * r[2] * r[2] - 2 * y[2] * r[2];
    out[7] += C[1] - m * r[0] * r[1] - y[0] * r[1] - r[0] * y[1];
    out[8] += C[2] - m * r[0] * r[2] - y[0] * r[2] - r[0] * y[2];
    out[9] += C[5] - m * r[1] * r[2] - y[1] * r[2] - r[1] * y[2];
}

__device__ __forceinline__ void sincos_dt(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ void sincos_dt(float x, float* s, float* c) { sincosf(x, s, c); }

__device__ __forceinline__ bool in_mask(unsigned long long mask, int t)
{
    return t < 64 && ((mask >> t) & 1ull);
}

}  // namespace grid

using namespace grid;

extern "C" __global__ void __launch_bounds__(64) grid_fdgrad_fused(Args args)
{
    __shared__ double s_model[N * kBodyStride];
    __shared__ KnotLds s_knot[K];

    const int lane = threadIdx.x;
    const int g = lane / L;            // knot slot in this wavefront
    const int t = lane % L;            // lane within the knot
    const int knot_raw = blockIdx.x * K + g;
    const bool valid = knot_raw < args.nknots;
    const int knot = valid ? knot_raw : args.nknots - 1;   // tail slots recompute the last knot
    KnotLds& S = s_knot[g];

    for (int e = lane; e < N * kBodyStride; e += 64)
        s_model[e] = args.model[e];

    // ---------------------------------------------------------------- 1. transforms
    DT my_tau = 0;
    if (t < N) {
        const DT qi = (DT)args.q[(long)knot * N + t];
        const DT qdi = (DT)args.qd[(long)knot * N + t];
        my_tau = (DT)args.tau[(long)knot * N + t];
        DT s, c;
        sincos_dt(qi, &s, &c);
        const double* b = args.model + t * kBodyStride;   // read once from global
        DT ET[9], rT[3];
#pragma unroll
        for (int k = 0; k < 9; ++k)
            ET[k] = (DT)b[k];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            rT[k] = (DT)b[9 + k];
        // E = E_z(q) E_T, E_z = [[c, s, 0], [-s, c, 0], [0, 0, 1]]
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            S.E[t][k] = c * ET[k] + s * ET[3 + k];
            S.E[t][3 + k] = -s * ET[k] + c * ET[3 + k];
            S.E[t][6 + k] = ET[6 + k];
            S.r[t][k] = rT[k];
        }
        S.qd[t] = qdi;
        S.qdf[t] = (float)qdi;
        S.IC[t][0] = (DT)b[21];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            S.IC[t][1 + k] = (DT)b[18 + k];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            S.IC[t][4 + k] = (DT)b[12 + k];
    }
    wave_sync();

    // ---------------------------------------------------------------- 2. RNEA(q, qd, 0)
    // outward by tree level: v_i = X_i v_p + S qd_i, a_i = X_i a_p + (v_i x S) qd_i
#pragma unroll
    for (int l = 0; l < GRID_NLEV; ++l) {
        if (in_mask(kLevelMask[l], t)) {
            const int p = kParent[t];
            DT vp[6], ap[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                vp[k] = p < 0 ? (DT)0 : S.v[p][k];
                ap[k] = p < 0 ? (k < 3 ? (DT)0 : (DT)args.a0[k - 3]) : S.a[p][k];
            }
            DT v[6], xa[6], vxs[6];
            x_mv(S.E[t], S.r[t], vp, v);
            v[2] += S.qd[t];
            x_mv(S.E[t], S.r[t], ap, xa);
            cross_S(v, vxs);
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                S.v[t][k] = v[k];
                S.a[t][k] = xa[k] + vxs[k] * S.qd[t];
            }
        }
        wave_sync();
    }
    // f_i = I_i a_i + v_i x* (I_i v_i)
    if (t < N) {
        const double* b = s_model + t * kBodyStride;
        DT Ib[6], h[3];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            Ib[k] = (DT)b[12 + k];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            h[k] = (DT)b[18 + k];
        const DT m = (DT)b[21];
        DT v[6], a[6], Iv[6], Ia[6], w[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            v[k] = S.v[t][k];
            a[k] = S.a[t][k];
        }
        inertia_mv(Ib, h, m, v, Iv);
        inertia_mv(Ib, h, m, a, Ia);
        crf_mv(v, Iv, w);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            S.F[t][k] = Ia[k] + w[k];
            S.vf[t][k] = (float)v[k];
            S.gam[t][k] = (float)Iv[k];
        }
#pragma unroll
        for (int k = 0; k < 9; ++k)
            S.Ef[t][k] = (float)S.E[t][k];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            S.Ef[t][9 + k] = (float)S.r[t][k];
    }
    wave_sync();
    // inward: f_p += X_i^T f_i and IC_p += X_i^T IC_i X_i, in rounds whose bodies have
    // distinct parents, deepest level first
#pragma unroll
    for (int rd = 0; rd < GRID_NROUND; ++rd) {
        if (in_mask(kRoundMask[rd], t)) {
            const int p = kParent[t];
            DT y[6];
            xt_fv(S.E[t], S.r[t], S.F[t], y);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                S.F[p][k] += y[k];
            inertia_to_parent(S.E[t], S.r[t], S.IC[t], S.IC[p]);
        }
        wave_sync();
    }
    if (t < N)
        S.tmc[t] = my_tau - S.F[t][2];   // c_i = S^T f_i

    // ---------------------------------------------------------------- 3. M from IC
    // lane t owns column t: F = IC_t S, M_tt = S^T F; walk up j -> parent(j):
    // F = X_j^T F, M_{parent(j), t} = S^T F
    if (t < N) {
        DT f[6];
        f[0] = S.IC[t][8];     // Ibar_xz
        f[1] = S.IC[t][9];     // Ibar_yz
        f[2] = S.IC[t][6];     // Ibar_zz
        f[3] = -S.IC[t][2];    // -h_y
        f[4] = S.IC[t][1];     //  h_x
        f[5] = 0;
        S.M[t][t] = f[2];
        int j = t;
#pragma unroll
        for (int step = 0; step < GRID_MAXANC; ++step) {
            const int p = j < 0 ? -1 : kParent[j];
            if (p >= 0) {
                DT y[6];
                xt_fv(S.E[j], S.r[j], f, y);
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    f[k] = y[k];
                S.M[p][t] = f[2];
                S.M[t][p] = f[2];
            }
            j = p;
        }
    }
    wave_sync();
    // zero the entries no walk touched: (i, k) with neither an ancestor of the other
    for (int e = t; e < NN; e += L) {
        const int i = e / N, k = e % N;
        if (!(kRelated[i] >> k & 1ull))
            S.M[i][k] = 0;
    }
    wave_sync();

    // ---------------------------------------------------------------- 4. Gauss-Jordan
    constexpr int EPL = (NN + L - 1) / L;   // entries per lane
#pragma unroll 1
    for (int p = 0; p < N; ++p) {
        DT nv[EPL];
        const DT piv = (DT)1 / S.M[p][p];
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
            const int e = t + s * L;
            if (e < NN) {
                const int i = e / N, k = e % N;
                const DT aik = S.M[i][k], aip = S.M[i][p], apk = S.M[p][k];
                DT r;
                if (i == p && k == p)
                    r = piv;
                else if (i == p)
                    r = apk * piv;
                else if (k == p)
                    r = -aip * piv;
                else
                    r = aik - aip * apk * piv;
                nv[s] = r;
            }
        }
        wave_sync();
#pragma unroll
        for (int s = 0; s < EPL; ++s) {
            const int e = t + s * L;
            if (e < NN)
                S.M[e / N][e % N] = nv[s];
        }
        wave_sync();
    }
    // mirror the upper triangle: M^-1 is returned exactly symmetric
    for (int e = t; e < NN; e += L) {
        const int i = e / N, k = e % N;
        const DT val = i <= k ? S.M[i][k] : S.M[k][i];
        S.minvf[i][k] = (float)val;
    }

    // ---------------------------------------------------------------- 5. qdd
    if (t < N) {
        DT acc = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const DT mik = t <= k ? S.M[t][k] : S.M[k][t];
            acc += mik * S.tmc[k];
        }
        S.qdd[t] = acc;
        if (valid)
            args.qdd[(long)knot * N + t] = (float)acc;
    }
    wave_sync();

    // ---------------------------------------------------------------- 6. RNEA at qdd
#pragma unroll
    for (int l = 0; l < GRID_NLEV; ++l) {
        if (in_mask(kLevelMask[l], t)) {
            const int p = kParent[t];
            DT ap[6];
#pragma unroll
            for (int k = 0; k < 6; ++k)
                ap[k] = p < 0 ? (k < 3 ? (DT)0 : (DT)args.a0[k - 3]) : S.a[p][k];
            DT xa[6], vxs[6], v[6], bxs[6];
#pragma unroll
            for (int k = 0; k < 6; ++k)
                v[k] = S.v[t][k];
            x_mv(S.E[t], S.r[t], ap, xa);
            cross_S(v, vxs);
            cross_S(xa, bxs);
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                S.a[t][k] = xa[k] + vxs[k] * S.qd[t];
                S.beta[t][k] = (float)bxs[k];
                S.alpha[t][k] = (float)vxs[k];
            }
            S.a[t][2] += S.qdd[t];
        }
        wave_sync();
    }
    if (t < N) {
        const double* b = s_model + t * kBodyStride;
        DT Ib[6], h[3];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            Ib[k] = (DT)b[12 + k];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            h[k] = (DT)b[18 + k];
        const DT m = (DT)b[21];
        DT a[6], v[6], Ia[6], w[6], Iv[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            a[k] = S.a[t][k];
            v[k] = S.v[t][k];
        }
        inertia_mv(Ib, h, m, a, Ia);
        inertia_mv(Ib, h, m, v, Iv);
        crf_mv(v, Iv, w);
#pragma unroll
        for (int k = 0; k < 6; ++k)
            S.F[t][k] = Ia[k] + w[k];
    }
    wave_sync();
#pragma unroll
    for (int rd = 0; rd < GRID_NROUND; ++rd) {
        if (in_mask(kRoundMask[rd], t)) {
            const int p = kParent[t];
            DT y[6];
            xt_fv(S.E[t], S.r[t], S.F[t], y);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                S.F[p][k] += y[k];
        }
        wave_sync();
    }
    if (t < N) {
        // zeta_i = X_i^T (S x* f_i), S x* f = [-f1, f0, 0, -f4, f3, 0]
        DT sf[6], y[6];
        sf[0] = -S.F[t][1];
        sf[1] = S.F[t][0];
        sf[2] = 0;
        sf[3] = -S.F[t][4];
        sf[4] = S.F[t][3];
        sf[5] = 0;
        xt_fv(S.E[t], S.r[t], sf, y);
#pragma unroll
        for (int k = 0; k < 6; ++k)
            S.zeta[t][k] = (float)y[k];
    }
    wave_sync();

    // ---------------------------------------------------------------- 7. dRNEA columns
    // lane t < 2N: u = t / N (0: d/dq, 1: d/dqd), column j = t % N
    const bool col_lane = t < 2 * N;
    const int u = t < N ? 0 : 1;
    const int j = col_lane ? (t % N) : 0;
    float src_v[6], src_a[6], src_f[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        // u = q : dv += (X_j v_p) x S = alpha_j,  da += beta_j,  backward += zeta_j
        // u = qd: dv += S,                         da += alpha_j (= v_j x S)
        src_v[k] = u == 0 ? S.alpha[j][k] : (k == 2 ? 1.0f : 0.0f);
        src_a[k] = u == 0 ? S.beta[j][k] : S.alpha[j][k];
        src_f[k] = u == 0 ? S.zeta[j][k] : 0.0f;
    }
    float dv[N][6], da[N][6], df[N][6];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int p = kParent[i];
        const float* E = S.Ef[i];
        const float* r = S.Ef[i] + 9;
        const float sel = (i == j) ? 1.0f : 0.0f;
        float xdv[6], xda[6];
        if (p >= 0) {
            x_mv(E, r, dv[p], xdv);
            x_mv(E, r, da[p], xda);
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
        cross_S(dv[i], dvxs);
        const float qdi = S.qdf[i];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            da[i][k] = xda[k] + dvxs[k] * qdi + sel * src_a[k];
        // df_i = I_i da_i + dv_i x* gamma_i + v_i x* (I_i dv_i)
        const double* b = s_model + i * kBodyStride;
        float Ib[6], h[3];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            Ib[k] = (float)b[12 + k];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            h[k] = (float)b[18 + k];
        const float m = (float)b[21];
        float t1[6], t2[6], t3[6], Idv[6];
        inertia_mv(Ib, h, m, da[i], t1);
        crf_mv(dv[i], S.gam[i], t2);
        inertia_mv(Ib, h, m, dv[i], Idv);
        crf_mv(S.vf[i], Idv, t3);
#pragma unroll
        for (int k = 0; k < 6; ++k)
            df[i][k] = t1[k] + t2[k] + t3[k];
    }
    float dtau[N];
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        dtau[i] = df[i][2];
        const int p = kParent[i];
        if (p >= 0) {
            const float* E = S.Ef[i];
            const float* r = S.Ef[i] + 9;
            const float sel = (i == j) ? 1.0f : 0.0f;
            float y[6];
            xt_fv(E, r, df[i], y);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                df[p][k] += y[k] + sel * src_f[k];
        }
    }

    // ---------------------------------------------------------------- 8. -M^-1 dtau
    if (col_lane && valid) {
        float* out = (u == 0 ? args.dqdd_dq : args.dqdd_dqd) + (long)knot * NN;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            float acc = 0.0f;
#pragma unroll
            for (int k = 0; k < N; ++k) {
                if (kBranch[i] == kBranch[k])      // M^-1 couples bodies of one base branch only
                    acc += S.minvf[i][k] * dtau[k];
            }
            out[i * N + j] = -acc;
        }
    }
    if (valid) {
        float* out = args.Minv + (long)knot * NN;
        for (int e = t; e < NN; e += L)
            out[e] = S.minvf[e / N][e % N];
    }
}
