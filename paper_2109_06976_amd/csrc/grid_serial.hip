// Fused kernel with one lane per (knot, branch) problem (gfx950): grid_fdgrad_serial.
//
// Every lane of a wavefront works on the same branch of the same robot for a different knot,
// so all model constants are instruction literals, nothing crosses lanes, and no work is
// repeated: the fewest instructions per knot of all the builds (the throughput form; its
// latency is one lane's whole chain). Per problem, float32 (Sec. IV-B):
//   1. X_i = (E_i, r_i), E_i = E_z(q_i) E_T,i (revolute), or E_i = E_T,i and
//      r_i = r_T,i + q_i E_T,i^T e_z (prismatic)
//   2. RNEA(q, qd, 0): v_i, a_i, gamma_i = I_i v_i, f_i, accumulated inward; c_i = S^T f_i
//   3. M by composite rigid bodies: I^c_i = I_i + sum over children of X^T I^c X, kept as
//      (mass, first moment, rotational inertia about the origin); M_ii = S^T I^c_i S and
//      M_ki = S^T (X^T ... X^T I^c_i S) for the ancestors k of i
//   4. M = L^T L along ancestor paths, M^-1 by B solves, qdd = M^-1 (tau - c)
//   5. RNEA at qdd as the increment over step 2 (Da_i, Df_i)
//   6. for each joint j the columns d/dq_j and d/dqd_j together: Algorithm 1 forward over
//      the subtree of j, the backward pass over the subtree and the ancestors of j, and
//      dqdd/du_j = -M^-1 dtau/du_j by the two triangular solves
//
// Transform of a rigid-body inertia (m, h, Ibar) of frame i into its parent frame, X = (E, r):
//   m' = m, h' = E^T h + m r,
//   Ibar' = E^T Ibar E + 2 (r . h~) 1 - r h~^T - h~ r^T + m (|r|^2 1 - r r^T),  h~ = E^T h
// (from X^T I X written out with a x b x = b a^T - (a . b) 1).

namespace grids {

using grid::crf_mv;
using grid::cross_S;
using grid::inertia_mv;
using grid::kConstStride;
using grid::prismatic;
using grid::s_crf;
using grid::s_index;
using grid::x_mv;
using grid::xt_fv;

template <class S>
__device__ __forceinline__ bool in_subtree(int i, int j)   // i == j or j a strict ancestor of i
{
    return i == j || ((S::anc[i] >> j) & 1ull);
}

struct RB {         // rigid-body inertia about the frame origin
    float m, h[3], I[6];   // I: xx yy zz xy xz yz
};

__device__ __forceinline__ RB rb_to_parent(const float* E, const float* r, const RB& c)
{
    const float Ib[3][3] = {{c.I[0], c.I[3], c.I[4]}, {c.I[3], c.I[1], c.I[5]},
                            {c.I[4], c.I[5], c.I[2]}};
    float T[3][3];    // Ibar E
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            T[a][b] = Ib[a][0] * E[b] + Ib[a][1] * E[3 + b] + Ib[a][2] * E[6 + b];
    float ht[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        ht[a] = E[a] * c.h[0] + E[3 + a] * c.h[1] + E[6 + a] * c.h[2];
    const float rh = r[0] * ht[0] + r[1] * ht[1] + r[2] * ht[2];
    const float rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    RB o;
    o.m = c.m;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        o.h[a] = ht[a] + c.m * r[a];
    const int ia[6] = {0, 1, 2, 0, 0, 1};
    const int ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const int a = ia[e], b = ib[e];
        const float etib = E[a] * T[0][b] + E[3 + a] * T[1][b] + E[6 + a] * T[2][b];
        const float diag = (a == b) ? 2.0f * rh + c.m * rr : 0.0f;
        o.I[e] = etib + diag - r[a] * ht[b] - ht[a] * r[b] - c.m * r[a] * r[b];
    }
    return o;
}

__device__ __forceinline__ void rb_add(RB& x, const RB& y)
{
    x.m += y.m;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        x.h[a] += y.h[a];
#pragma unroll
    for (int e = 0; e < 6; ++e)
        x.I[e] += y.I[e];
}

// X_i = (E_i, r_i) of one body at joint position qi: E = E_z(q) E_T (hardware sin and cos,
// argument in revolutions reduced to [0, 1)), r = r_T; prismatic: E = E_T, r = r_T + q E_T^T e_z
template <class I>
__device__ __forceinline__ void serial_transform(int i, float qi, float (&E)[9], float (&R)[3])
{
    const float* c = I::consts() + i * kConstStride;
    if (prismatic<I>(i)) {
#pragma unroll
        for (int k = 0; k < 9; ++k)
            E[k] = c[k];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            R[k] = c[9 + k] + qi * c[6 + k];
        return;
    }
    const float rev = __builtin_amdgcn_fractf(qi * 0.159154943091895336f);
    const float s = __builtin_amdgcn_sinf(rev);
    const float co = __builtin_amdgcn_cosf(rev);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        E[k] = co * c[k] + s * c[3 + k];
        E[3 + k] = co * c[3 + k] - s * c[k];
        E[6 + k] = c[6 + k];
        R[k] = c[9 + k];
    }
}

// M by composite rigid bodies, factored: I^c_i = I_i + sum over children of X^T I^c X as
// (mass, first moment, rotational inertia); M_ii = S^T I^c_i S and M_ki = S^T (X^T ... I^c_i S)
// up the ancestor path of i; then M = L^T L in place (Lf, dinv = 1 / L_kk)
template <class I>
__device__ __forceinline__ void serial_mass_factor(const float (&E)[I::S::B][9],
                                                   const float (&R)[I::S::B][3],
                                                   float (&Lf)[I::S::B][I::S::B],
                                                   float (&dinv)[I::S::B])
{
    using S = typename I::S;
    constexpr int B = S::B;
    const float* C = I::consts();
    RB Ic[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
        const float* c = C + i * kConstStride;
        Ic[i].m = c[21];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            Ic[i].h[k] = c[18 + k];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            Ic[i].I[k] = c[12 + k];
    }
#pragma unroll
    for (int i = B - 1; i >= 0; --i) {
        // I^c_i S: [Ibar e_z; -(h x e_z)] for S = (e_z, 0), [h x e_z; m e_z] for (0, e_z)
        float f[6] = {Ic[i].I[4], Ic[i].I[5], Ic[i].I[2], -Ic[i].h[1], Ic[i].h[0], 0.0f};
        if (prismatic<I>(i)) {
            f[0] = Ic[i].h[1];
            f[1] = -Ic[i].h[0];
            f[2] = 0.0f;
            f[3] = 0.0f;
            f[4] = 0.0f;
            f[5] = Ic[i].m;
        }
        Lf[i][i] = f[s_index(prismatic<I>(i))];
        // up the ancestor path (ancestors have smaller indices): f into the parent
        // frame of k, M_{lambda(k), i} = S^T f
#pragma unroll
        for (int k = B - 1; k >= 0; --k) {
            if (k <= i && (k == i || gridq::is_anc<S>(k, i)) && S::parent[k] >= 0) {
                float y[6];
                xt_fv(E[k], R[k], f, y);
#pragma unroll
                for (int e = 0; e < 6; ++e)
                    f[e] = y[e];
                const int pk = S::parent[k] < 0 ? 0 : S::parent[k];
                Lf[i][pk] = f[s_index(prismatic<I>(pk))];
            }
        }
        const int p = S::parent[i];
        if (p >= 0)
            rb_add(Ic[p], rb_to_parent(E[i], R[i], Ic[i]));
    }
    gridq::ltl_factor<S>(Lf, dinv);
}

template <int B>
__device__ __forceinline__ void pick6(const float (&arr)[B][6], int j, float (&out)[6])
{
#pragma unroll
    for (int k = 0; k < 6; ++k)
        out[k] = arr[0][k];
#pragma unroll
    for (int i = 1; i < B; ++i)
#pragma unroll
        for (int k = 0; k < 6; ++k)
            out[k] = (i == j) ? arr[i][k] : out[k];
}

// The K knots of a wavefront own one contiguous block of each output array when their branch
// is the whole robot (N == B). Lane-per-knot stores of one element each hit 64 addresses
// N^2 floats apart, so for small robots the outputs are staged in LDS (two [K][N][N] arrays)
// and written out by the wavefront as contiguous 16-byte stores.
template <int B, int N, int K>
struct SerialStage {
    static constexpr bool on = N == B && 2 * K * N * N * 4 <= 32 * 1024;
    static constexpr int floats = on ? K * N * N : 4;
};

// A branch that is not the whole robot (N > B) owns B rows of each knot's blocks, scattered
// over the robot's numbering: lane-per-knot stores of one element each would again hit 64
// addresses N^2 floats apart. Its rows are staged instead ([K][B][N], local row i, robot
// column) while two such tiles fit 32 KB, and the wavefront writes each row's N floats with
// consecutive lanes on consecutive elements, zeros in the other branches' columns included.
// With four lanes per knot (whose stores already put four columns side by side) the dispatch
// stages only when every branch of the robot fits: on a robot whose long branch does not,
// staging its short ones made the launch slower.
template <int B, int N, int K, bool kAllowed = true>
struct SerialRows {
    static constexpr bool fits = N > B && 2 * K * B * N * 4 <= 32 * 1024;
    static constexpr bool on = kAllowed && fits;
    static constexpr int floats = on ? K * B * N : 4;
};

template <class I, int L>
constexpr bool serial_rows_fit()
{
    return SerialRows<I::S::B, I::N, 64 / L>::fits;
}

// floats of LDS one branch's staging takes (its two tiles); the dispatch of a robot allocates
// the largest over its branches once, so that the branches of one kernel share it
template <class I, int L, bool kRows>
constexpr int serial_stage_floats()
{
    using ST = SerialStage<I::S::B, I::N, 64 / L>;
    using SR = SerialRows<I::S::B, I::N, 64 / L, kRows>;
    return 2 * (ST::on ? ST::floats : SR::floats);
}

constexpr int cmax(int a) { return a; }
template <class... T>
constexpr int cmax(int a, int b, T... rest) { return cmax(a > b ? a : b, rest...); }

// write the staged rows of the wavefront's nv valid knots: element (knot, local row i, column c)
// goes to row body(i) of that knot's block; `dst` is the block of the wavefront's first knot
template <class I>
__device__ __forceinline__ void flush_rows(float* dst, const float* tile, int nv, int lane)
{
    constexpr int B = I::S::B;
    constexpr int N = I::N;
    for (int e = lane; e < nv * B * N; e += 64) {
        const int kl = e / (B * N), rem = e - kl * (B * N);
        const int i = rem / N, c2 = rem - i * N;
        const float v = I::contains(c2) ? tile[e] : 0.0f;
        dst[(long)kl * N * N + (long)I::body_of(i) * N + c2] = v;
    }
}

// the workgroup is one wavefront: ordering its own LDS traffic needs no workgroup barrier
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// copy `cnt` floats from LDS to global memory: 16 bytes per lane and step when the destination
// is 16-byte aligned (the staging array is; a wavefront's block starts at a multiple of 64 N
// floats, so only the caller's base address decides), else one float per lane and step
__device__ __forceinline__ void flush_stage(float* dst, const float* src, int cnt, int lane)
{
    int done = 0;
    if ((reinterpret_cast<unsigned long>(dst) & 15ul) == 0) {
        const int n4 = cnt / 4;
        for (int e = lane; e < n4; e += 64)
            reinterpret_cast<float4*>(dst)[e] = reinterpret_cast<const float4*>(src)[e];
        done = 4 * n4;
    }
    for (int e = done + lane; e < cnt; e += 64)
        dst[e] = src[e];
}

// L lanes per knot (1: build 5; 4: build 6; 2: build 7). Every lane of a knot runs steps 1-5; the columns
// of M^-1 and the joints j of step 6 are dealt out among them (lane h takes h, h + L, ...), so
// a wavefront holds 64 / L knots: L times the wavefronts of build 5 for the same batch, at the
// cost of repeating steps 1-5 L times. The lanes of a knot are adjacent.
// `pool` is the dispatch's LDS array of at least serial_stage_floats<I, L, kRows>() floats;
// kRows allows the row staging of a branch smaller than the robot.
template <class I, int L, bool kRows>
__device__ __forceinline__ void run_serial(const grid::Args& A, int block, float* pool)
{
    using S = typename I::S;
    constexpr int B = S::B;
    constexpr int N = I::N;
    constexpr int K = 64 / L;                        // knots per wavefront
    using ST = SerialStage<B, N, K>;
    using SR = SerialRows<B, N, K, kRows>;
    float* const s_stage[2] = {pool, pool + serial_stage_floats<I, L, kRows>() / 2};
    const int lane = (int)threadIdx.x;
    const int h = lane % L;                          // this lane's share of the columns
    const int kl = lane / L;                         // the knot within the wavefront
    const int kraw = block * K + kl;
    const bool valid = kraw < A.nknots;
    const int knot = valid ? kraw : A.nknots - 1;   // tail lanes recompute the last knot
    const float* C = I::consts();                   // literals: folded into the code
    const long vbase = (long)knot * N;
    const long mbase = (long)knot * N * N;

    // ------------------------------------------------------------ 1. transforms
    float qd[B], E[B][9], R[B][3];
#pragma unroll
    for (int i = 0; i < B; ++i) {
        const long o = vbase + I::body[i];
        qd[i] = A.qd[o];
        serial_transform<I>(i, A.q[o], E[i], R[i]);
    }
    const float a0[6] = {0.0f, 0.0f, 0.0f, I::a0()[0], I::a0()[1], I::a0()[2]};   // -g
    const float zero6[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};

    // ------------------------------------------------------------ 2. RNEA(q, qd, 0)
    float v[B][6], gam[B][6], F[B][6], xa[B][6];   // xa_i = X_i a_lambda(i)
    {
        float a[B][6];
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const int p = S::parent[i];
            const float* c = C + i * kConstStride;
            x_mv(E[i], R[i], p < 0 ? zero6 : v[p < 0 ? 0 : p], v[i]);
            x_mv(E[i], R[i], p < 0 ? a0 : a[p < 0 ? 0 : p], xa[i]);
            v[i][s_index(prismatic<I>(i))] += qd[i];
            float vxs[6], Ia[6], w[6];
            cross_S(prismatic<I>(i), v[i], vxs);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                a[i][k] = xa[i][k] + vxs[k] * qd[i];
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
    }

    // ------------------------------------------------------------ 3. M by composite bodies
    float Lf[B][B], dinv[B];
    serial_mass_factor<I>(E, R, Lf, dinv);

    // ------------------------------------------------------------ 4. M^-1 and qdd
    if (valid && L == 1) {
#pragma unroll
        for (int jm = 0; jm < B; ++jm) {
            float mc[B];
#pragma unroll
            for (int i = 0; i < B; ++i)
                mc[i] = (i == jm) ? 1.0f : 0.0f;
            gridq::ltl_solve<S>(Lf, dinv, mc);
            // entries (i, jm), i <= jm, written to both mirrored positions: exactly symmetric
#pragma unroll
            for (int i = 0; i <= jm; ++i) {
                if constexpr (ST::on) {
                    s_stage[0][kl * N * N + I::body[i] * N + I::body[jm]] = mc[i];
                    s_stage[0][kl * N * N + I::body[jm] * N + I::body[i]] = mc[i];
                } else if constexpr (SR::on) {
                    s_stage[0][kl * B * N + i * N + I::body[jm]] = mc[i];
                    s_stage[0][kl * B * N + jm * N + I::body[i]] = mc[i];
                } else {
                    A.Minv[mbase + (long)I::body[i] * N + I::body[jm]] = mc[i];
                    A.Minv[mbase + (long)I::body[jm] * N + I::body[i]] = mc[i];
                }
            }
        }
    } else if (valid) {
        // the knot's lanes share the columns of M^-1
#pragma unroll 1
        for (int jm = h; jm < B; jm += L) {
            float mc[B];
#pragma unroll
            for (int i = 0; i < B; ++i)
                mc[i] = (i == jm) ? 1.0f : 0.0f;
            gridq::ltl_solve<S>(Lf, dinv, mc);
            const int gm = I::body_of(jm);
#pragma unroll
            for (int i = 0; i < B; ++i) {
                if (i > jm)
                    continue;
                if constexpr (ST::on) {
                    s_stage[0][kl * N * N + I::body[i] * N + gm] = mc[i];
                    s_stage[0][kl * N * N + gm * N + I::body[i]] = mc[i];
                } else if constexpr (SR::on) {
                    s_stage[0][kl * B * N + i * N + gm] = mc[i];
                    s_stage[0][kl * B * N + jm * N + I::body[i]] = mc[i];
                } else {
                    A.Minv[mbase + (long)I::body[i] * N + gm] = mc[i];
                    A.Minv[mbase + (long)gm * N + I::body[i]] = mc[i];
                }
            }
        }
    }
    float x[B];
#pragma unroll
    for (int i = 0; i < B; ++i)
        x[i] = A.tau[vbase + I::body[i]] - F[i][s_index(prismatic<I>(i))];
    gridq::ltl_solve<S>(Lf, dinv, x);
    // the wavefront's valid knots (its first knot is block * K) and their output blocks
    const int nv = min(K, A.nknots - block * K);
    const long kb = (long)block * K;
    if constexpr (ST::on) {
        if (valid && h == 0) {
#pragma unroll
            for (int i = 0; i < B; ++i)
                s_stage[1][kl * N + I::body[i]] = x[i];
        }
        wave_lds_sync();                      // M^-1 and qdd staged
        flush_stage(A.Minv + kb * N * N, s_stage[0], nv * N * N, lane);
        flush_stage(A.qdd + kb * N, s_stage[1], nv * N, lane);
        wave_lds_sync();                      // staging free for the derivative columns
    } else {
        if (valid && h == 0) {
#pragma unroll
            for (int i = 0; i < B; ++i)
                A.qdd[vbase + I::body[i]] = x[i];
        }
        if constexpr (SR::on) {
            wave_lds_sync();                  // the rows of M^-1 staged
            flush_rows<I>(A.Minv + kb * N * N, s_stage[0], nv, lane);
            wave_lds_sync();                  // staging free for the derivative columns
        }
    }

    // ------------------------------------------------------------ 5. RNEA at qdd
    {
        float Da[B][6], Df[B][6];
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const int p = S::parent[i];
            const float* c = C + i * kConstStride;
            if (p >= 0) {
                x_mv(E[i], R[i], Da[p < 0 ? 0 : p], Da[i]);
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    xa[i][k] += Da[i][k];
            } else {
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    Da[i][k] = 0.0f;
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
#pragma unroll
            for (int k = 0; k < 6; ++k)
                F[i][k] += Df[i][k];
        }
    }

    // ------------------------------------------------------------ 6. dRNEA and dFD columns
    // One lane per knot and a branch of up to 8 bodies: the loop is unrolled, so that j is a
    // constant in each copy (no selects of the joint's quantities, the subtree tests folded;
    // chain7 at 65536 knots 44.6 -> 37.1 us); otherwise one copy of the body, j at run time.
    constexpr int kUnrollJ = (L == 1 && B <= 8) ? B : 1;
#pragma unroll kUnrollJ
    for (int j = h; j < B; j += L) {
        // sources of joint j: u = q: dv += v_j x S, da += (X_j a_lambda(j)) x S,
        // backward += X_j^T (S x* f_j); u = qd: dv += S, da += v_j x S
        float vj[6], xaj[6], Fj[6], Ej[9], rj[3];
        pick6<B>(v, j, vj);
        pick6<B>(xa, j, xaj);
        pick6<B>(F, j, Fj);
#pragma unroll
        for (int k = 0; k < 9; ++k)
            Ej[k] = E[0][k];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            rj[k] = R[0][k];
#pragma unroll
        for (int i = 1; i < B; ++i) {
#pragma unroll
            for (int k = 0; k < 9; ++k)
                Ej[k] = (i == j) ? E[i][k] : Ej[k];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                rj[k] = (i == j) ? R[i][k] : rj[k];
        }
        const bool pj = (I::prism >> j) & 1ull;            // joint j is prismatic
        float vxs[6], axs[6], srcf[6];
        cross_S(pj, vj, vxs);
        cross_S(pj, xaj, axs);
        {
            float sf[6];
            s_crf(pj, Fj, sf);                               // S x* f_j
            xt_fv(Ej, rj, sf, srcf);
        }
        // columns d/dq_j (index 0) and d/dqd_j (index 1), side by side
        float df[2][B][6];
        {
            float dv[2][B][6], da[2][B][6];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const int p = S::parent[i];
                const float* c = C + i * kConstStride;
                if (in_subtree<S>(i, j)) {
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        float xdv[6], xda[6];
                        if (i == j || p < 0) {
#pragma unroll
                            for (int k = 0; k < 6; ++k) {
                                xdv[k] = 0.0f;
                                xda[k] = 0.0f;
                            }
                        } else {
                            x_mv(E[i], R[i], dv[u][p < 0 ? 0 : p], xdv);
                            x_mv(E[i], R[i], da[u][p < 0 ? 0 : p], xda);
                        }
                        if (i == j) {
#pragma unroll
                            for (int k = 0; k < 6; ++k) {
                                xdv[k] = u == 0 ? vxs[k] : (k == s_index(pj) ? 1.0f : 0.0f);
                                xda[k] = u == 0 ? axs[k] : vxs[k];
                            }
                        }
                        float dvxs[6];
                        cross_S(prismatic<I>(i), xdv, dvxs);
#pragma unroll
                        for (int k = 0; k < 6; ++k) {
                            dv[u][i][k] = xdv[k];
                            da[u][i][k] = xda[k] + dvxs[k] * qd[i];
                        }
                        // df_i = I_i da_i + dv_i x* gamma_i + v_i x* (I_i dv_i)
                        float t1[6], t2[6], t3[6], Idv[6];
                        inertia_mv(c, da[u][i], t1);
                        crf_mv(dv[u][i], gam[i], t2);
                        inertia_mv(c, dv[u][i], Idv);
                        crf_mv(v[i], Idv, t3);
#pragma unroll
                        for (int k = 0; k < 6; ++k)
                            df[u][i][k] = t1[k] + t2[k] + t3[k];
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int k = 0; k < 6; ++k)
                            df[u][i][k] = 0.0f;
                }
            }
        }
        float dx[2][B];
#pragma unroll
        for (int i = B - 1; i >= 0; --i) {
            const int p = S::parent[i];
            const bool live = in_subtree<S>(i, j) || ((S::anc[j < 0 ? 0 : j] >> i) & 1ull);
#pragma unroll
            for (int u = 0; u < 2; ++u)
                dx[u][i] = df[u][i][s_index(prismatic<I>(i))];
            if (p >= 0 && live) {
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    float y[6];
                    xt_fv(E[i], R[i], df[u][i], y);
                    const float sel = (u == 0 && i == j) ? 1.0f : 0.0f;
#pragma unroll
                    for (int k = 0; k < 6; ++k)
                        df[u][p < 0 ? 0 : p][k] += y[k] + sel * srcf[k];
                }
            }
        }
        gridq::ltl_solve<S>(Lf, dinv, dx[0]);
        gridq::ltl_solve<S>(Lf, dinv, dx[1]);
        if (valid) {
            const int gj = I::body_of(j);
#pragma unroll
            for (int i = 0; i < B; ++i) {
                if constexpr (ST::on) {
                    s_stage[0][kl * N * N + I::body[i] * N + gj] = -dx[0][i];
                    s_stage[1][kl * N * N + I::body[i] * N + gj] = -dx[1][i];
                } else if constexpr (SR::on) {
                    s_stage[0][kl * B * N + i * N + gj] = -dx[0][i];
                    s_stage[1][kl * B * N + i * N + gj] = -dx[1][i];
                } else {
                    A.dqdd_dq[mbase + (long)I::body[i] * N + gj] = -dx[0][i];
                    A.dqdd_dqd[mbase + (long)I::body[i] * N + gj] = -dx[1][i];
                }
            }
        }
    }
    if constexpr (ST::on) {
        wave_lds_sync();                      // every column staged
        flush_stage(A.dqdd_dq + kb * N * N, s_stage[0], nv * N * N, lane);
        flush_stage(A.dqdd_dqd + kb * N * N, s_stage[1], nv * N * N, lane);
    }
    if constexpr (SR::on) {
        wave_lds_sync();                      // every column staged
        flush_rows<I>(A.dqdd_dq + kb * N * N, s_stage[0], nv, lane);
        flush_rows<I>(A.dqdd_dqd + kb * N * N, s_stage[1], nv, lane);
    }
    if (valid && N > B && !SR::on) {
        // this branch's rows hold zeros in the other branches' columns
        for (int e = h; e < B * N; e += L) {
            const int i = e / N, c2 = e % N;
            if (!I::contains(c2)) {
                const long o = mbase + (long)I::body_of(i) * N + c2;
                A.Minv[o] = 0.0f;
                A.dqdd_dq[o] = 0.0f;
                A.dqdd_dqd[o] = 0.0f;
            }
        }
    }
}

// ------------------------------------------------------------------ M^-1 alone, two routes
//
// One lane per (knot, branch) problem, as build 5, computing only M^-1, by either route:
//   kDirect = false: M by composite rigid bodies, M = L^T L along ancestor paths, and the B
//     columns of M^-1 by two triangular solves each (the route every fused build takes);
//   kDirect = true: the paper's direct inverse (Sec. IV-B): the articulated-body recursion
//     with zero velocity and gravity and the identity as its B right-hand sides. Inward,
//     U_i = IA_i S_i, D_i = S_i^T U_i, row_i = (e_i^T - S_i^T F_i) / D_i over the columns
//     of the subtree of i, IA_lambda += X^T (IA_i - U_i U_i^T / D_i) X and
//     F_lambda += X^T (F_i + U_i row_i); outward, per column c, A = X_i P_lambda,
//     row_i -= U_i^T A / D_i and P_i = A + S_i row_i; M^-1 = [row_i]. The articulated
//     inertias do not depend on the right-hand sides, so they come first, and then each
//     column runs its inward and outward steps (the same arithmetic, fewer live values).
// Both write the upper triangle of the branch's block to both mirrored positions (exactly
// symmetric) and zeros in the other branches' columns, one float per store.

// articulated-body inertia [[A, B], [B^T, C]] in a body frame: A, C symmetric (xx yy zz xy xz
// yz), B row-major
struct AB {
    float A[6], B[9], C[6];
};

__device__ __forceinline__ constexpr int sym3(int a, int b)
{
    return a == b ? a : (a + b == 1 ? 3 : (a + b == 2 ? 4 : 5));
}

// X^T Ia X for X = [E 0; -E r~ E]: with A' = E^T A E, B' = E^T B E, C' = E^T C E,
//   C'' = C', B'' = B' + r~ C', A'' = A' + G + G^T - r~ C' r~, G = r~ B'^T
// (X = diag(E, E) [1 0; -r~ 1]; for a rigid body this is the transform rb_to_parent writes out)
__device__ __forceinline__ AB ab_to_parent(const float* E, const float* r, const AB& x)
{
    float A1[6], C1[6], B1[3][3];
    {
        float Ta[3][3], Tb[3][3], Tc[3][3];    // A E, B E, C E
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                Ta[a][b] = x.A[sym3(a, 0)] * E[b] + x.A[sym3(a, 1)] * E[3 + b] +
                           x.A[sym3(a, 2)] * E[6 + b];
                Tb[a][b] = x.B[3 * a] * E[b] + x.B[3 * a + 1] * E[3 + b] + x.B[3 * a + 2] * E[6 + b];
                Tc[a][b] = x.C[sym3(a, 0)] * E[b] + x.C[sym3(a, 1)] * E[3 + b] +
                           x.C[sym3(a, 2)] * E[6 + b];
            }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                B1[a][b] = E[a] * Tb[0][b] + E[3 + a] * Tb[1][b] + E[6 + a] * Tb[2][b];
                if (a <= b) {
                    A1[sym3(a, b)] = E[a] * Ta[0][b] + E[3 + a] * Ta[1][b] + E[6 + a] * Ta[2][b];
                    C1[sym3(a, b)] = E[a] * Tc[0][b] + E[3 + a] * Tc[1][b] + E[6 + a] * Tc[2][b];
                }
            }
    }
    const float rt[3][3] = {{0.0f, -r[2], r[1]}, {r[2], 0.0f, -r[0]}, {-r[1], r[0], 0.0f}};
    float W[3][3], G[3][3];                    // r~ C', r~ B'^T
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            W[a][b] = rt[a][0] * C1[sym3(0, b)] + rt[a][1] * C1[sym3(1, b)] +
                      rt[a][2] * C1[sym3(2, b)];
            G[a][b] = rt[a][0] * B1[b][0] + rt[a][1] * B1[b][1] + rt[a][2] * B1[b][2];
        }
    AB o;
#pragma unroll
    for (int e = 0; e < 6; ++e)
        o.C[e] = C1[e];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            o.B[3 * a + b] = B1[a][b] + W[a][b];
            if (a <= b) {
                const float wr = W[a][0] * rt[0][b] + W[a][1] * rt[1][b] + W[a][2] * rt[2][b];
                o.A[sym3(a, b)] = A1[sym3(a, b)] + G[a][b] + G[b][a] - wr;
            }
        }
    return o;
}

template <class I, bool kDirect>
__device__ __forceinline__ void run_minv(const grid::Args& A, int block)
{
    using S = typename I::S;
    constexpr int B = S::B;
    constexpr int N = I::N;
    const int lane = (int)threadIdx.x;
    const int kraw = block * 64 + lane;
    const bool valid = kraw < A.nknots;
    const int knot = valid ? kraw : A.nknots - 1;
    const long mbase = (long)knot * N * N;
    float E[B][9], R[B][3];
#pragma unroll
    for (int i = 0; i < B; ++i)
        serial_transform<I>(i, A.q[(long)knot * N + I::body[i]], E[i], R[i]);
    const auto put = [&](int i, int c, float x) {   // entry (i, c), i <= c, and its mirror
        if (valid) {
            A.Minv[mbase + (long)I::body[i] * N + I::body[c]] = x;
            A.Minv[mbase + (long)I::body[c] * N + I::body[i]] = x;
        }
    };
    if constexpr (!kDirect) {
        float Lf[B][B], dinv[B];
        serial_mass_factor<I>(E, R, Lf, dinv);
#pragma unroll
        for (int c = 0; c < B; ++c) {
            float mc[B];
#pragma unroll
            for (int i = 0; i < B; ++i)
                mc[i] = (i == c) ? 1.0f : 0.0f;
            gridq::ltl_solve<S>(Lf, dinv, mc);
#pragma unroll
            for (int i = 0; i <= c; ++i)
                put(i, c, mc[i]);
        }
    } else {
        const float* C = I::consts();
        float U[B][6], dv[B];
        {
            // inward: the articulated inertias, U_i = IA_i S_i and 1 / D_i (no right-hand side
            // enters them)
            AB Ia[B];
#pragma unroll
            for (int i = 0; i < B; ++i) {   // I_i = [[Ibar, h~], [-h~, m 1]]
                const float* c = C + i * kConstStride;
                const float h0 = c[18], h1 = c[19], h2 = c[20], m = c[21];
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    Ia[i].A[k] = c[12 + k];
                const float hb[9] = {0.0f, -h2, h1, h2, 0.0f, -h0, -h1, h0, 0.0f};
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    Ia[i].B[k] = hb[k];
                const float cm[6] = {m, m, m, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    Ia[i].C[k] = cm[k];
            }
#pragma unroll
            for (int i = B - 1; i >= 0; --i) {
                const AB& x = Ia[i];
                if (prismatic<I>(i)) {        // IA_i e_6 = [B[:, 2]; C[:, 2]]
                    const float u[6] = {x.B[2], x.B[5], x.B[8], x.C[4], x.C[5], x.C[2]};
#pragma unroll
                    for (int k = 0; k < 6; ++k)
                        U[i][k] = u[k];
                } else {                      // IA_i e_3 = [A[:, 2]; B[2, :]]
                    const float u[6] = {x.A[4], x.A[5], x.A[2], x.B[6], x.B[7], x.B[8]};
#pragma unroll
                    for (int k = 0; k < 6; ++k)
                        U[i][k] = u[k];
                }
                dv[i] = 1.0f / U[i][s_index(prismatic<I>(i))];
                const int p = S::parent[i];
                if (p < 0)
                    continue;
                AB y = x;                     // IA_i - U_i U_i^T / D_i
                const float* Ua = U[i];
                const float* Ul = U[i] + 3;
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        y.B[3 * a + b] -= Ua[a] * Ul[b] * dv[i];
                        if (a <= b) {
                            y.A[sym3(a, b)] -= Ua[a] * Ua[b] * dv[i];
                            y.C[sym3(a, b)] -= Ul[a] * Ul[b] * dv[i];
                        }
                    }
                const AB z = ab_to_parent(E[i], R[i], y);
                const int pp = p < 0 ? 0 : p;
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    Ia[pp].A[k] += z.A[k];
                    Ia[pp].C[k] += z.C[k];
                }
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    Ia[pp].B[k] += z.B[k];
            }
        }
        // the right-hand sides one column c at a time (the recursion is linear in them): F_i
        // of column c is nonzero only on the ancestor path of c, so inward it is one 6-vector
        // carried from c to the root; outward every body takes its row entry
#pragma unroll
        for (int c = 0; c < B; ++c) {
            float row[B];
            {
                float f[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int i = B - 1; i >= 0; --i) {
                    if (!in_subtree<S>(c, i)) {
                        row[i] = 0.0f;
                        continue;
                    }
                    row[i] = ((c == i ? 1.0f : 0.0f) - f[s_index(prismatic<I>(i))]) * dv[i];
                    if (S::parent[i] >= 0) {
                        float col[6];
#pragma unroll
                        for (int k = 0; k < 6; ++k)
                            col[k] = f[k] + U[i][k] * row[i];
                        xt_fv(E[i], R[i], col, f);
                    }
                }
            }
            float P[B][6];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const int p = S::parent[i];
                float Av[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                float x = row[i];
                if (p >= 0) {
                    x_mv(E[i], R[i], P[p < 0 ? 0 : p], Av);
                    float ua = 0.0f;
#pragma unroll
                    for (int k = 0; k < 6; ++k)
                        ua += U[i][k] * Av[k];
                    x -= ua * dv[i];
                }
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    P[i][k] = Av[k];
                P[i][s_index(prismatic<I>(i))] += x;
                if (i <= c)
                    put(i, c, x);
            }
        }
    }
    if (valid && N > B) {
        // this branch's rows hold zeros in the other branches' columns
#pragma unroll
        for (int i = 0; i < B; ++i)
#pragma unroll
            for (int c2 = 0; c2 < N; ++c2)
                if (!I::contains(c2))
                    A.Minv[mbase + (long)I::body[i] * N + c2] = 0.0f;
    }
}

}  // namespace grids

// kernels of a one-robot module (a module of several robots defines GRID_PIPE_ONLY and its
// own entry point, grid_fdgrad_pipe_mixed)
#ifndef GRID_PIPE_ONLY

// defined by the generated epilogue: workgroup -> (branch, 64 knots)
__device__ void grid_dispatch_s(const grid::Args& args, int block);

extern "C" __global__ void __launch_bounds__(64) grid_fdgrad_serial(grid::Args args)
{
    grid_dispatch_s(args, (int)blockIdx.x);
}

// defined by the generated epilogue: workgroup -> (branch, 16 knots), four lanes per knot
__device__ void grid_dispatch_s4(const grid::Args& args, int block);

extern "C" __global__ void __launch_bounds__(64) grid_fdgrad_serial4(grid::Args args)
{
    grid_dispatch_s4(args, (int)blockIdx.x);
}

// defined by the generated epilogue: workgroup -> (branch, 32 knots), two lanes per knot
__device__ void grid_dispatch_s2(const grid::Args& args, int block);

extern "C" __global__ void __launch_bounds__(64) grid_fdgrad_serial2(grid::Args args)
{
    grid_dispatch_s2(args, (int)blockIdx.x);
}

// defined by the generated epilogue: workgroup -> (branch, 64 knots), M^-1 by either route
template <bool kDirect>
__device__ void grid_dispatch_minv(const grid::Args& args, int block);

// M^-1 alone, one lane per knot: composite bodies and the L^T L factor
extern "C" __global__ void __launch_bounds__(64) grid_minv_serial(grid::Args args)
{
    grid_dispatch_minv<false>(args, (int)blockIdx.x);
}

// M^-1 alone, one lane per knot: the direct articulated-body inverse (Sec. IV-B)
extern "C" __global__ void __launch_bounds__(64) grid_minv_direct(grid::Args args)
{
    grid_dispatch_minv<true>(args, (int)blockIdx.x);
}

#endif  // GRID_PIPE_ONLY
