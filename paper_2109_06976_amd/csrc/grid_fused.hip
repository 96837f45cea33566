// Fused kernels in quad layout (gfx950).
//
// A spatial 6-vector is spread over the four lanes of a quad: lane c (c = 0, 1, 2) holds
// angular component c and linear component c; lane 3 repeats lane 0. The other two
// components a lane needs for a cross product or a 3x3 row come from its quad neighbours
// through DPP quad permutations, so a transform, an inertia product or a cross product
// costs a few DPP moves and about three FMAs per lane instead of a whole 6-vector per lane.
// A quad owns one derivative column (u, j) of a (knot, branch) problem, and all quads of a
// problem run the shared sweeps in lockstep. The per-lane model constants come from a lane
// table generated with the model and copied to LDS by each workgroup.
//
// Steps per (knot, branch), float32 (Sec. IV-B): transforms; RNEA(q, qd, 0); column s of M
// as ID(q, 0, e_s) without gravity; M = L^T L along ancestor paths; qdd; RNEA at qdd as the
// increment over RNEA(q, qd, 0); the dRNEA forward (Algorithm 1) and backward pass of each
// column; dqdd/du = -M^-1 dtau/du.
//
// grid_fdgrad_quad runs all steps in every quad. A problem with 2B columns uses Q quads
// (power of two >= 2B, at most 16) in each of W wavefronts (W * Q >= 2B).
//
// grid_fdgrad_pipe splits the steps over three roles that run at the same time on different
// wavefronts of a workgroup, shortening the dependency chain:
//   role A (2B columns, one per quad, 2..4 wavefronts): RNEA(q, qd, 0); the dRNEA columns
//                        with the sources taken at qdd = 0
//   role B (B columns, one or two per quad, one wavefront): M and its factor; qdd once
//                        role A has published the bias forces; RNEA increments at qdd; the
//                        part of each q-column that depends on qdd
//   role C (B columns, one wavefront; branches of up to 16 bodies): once role B has
//                        published M, its factor and M^-1. Beyond 16 bodies role B publishes
//                        its factor instead (after the first barrier, behind an LDS flag):
//                        role A's qd-columns solve for the columns of M^-1 before the second
//                        barrier, every column ends with two triangular solves, and the
//                        outputs are staged in LDS and written as whole rows
// dtau/dqd does not depend on qdd, and dtau/dq is affine in the two source terms that do:
// the parent acceleration (X_j a_lambda(j)) x S enters the forward sweep and the term
// X_j^T (S x* f_j) the backward sweep, each linearly, so the qdd part of a q-column is the
// same sweep with the increments X_j Da_lambda(j) and Df_j as sources and dv = 0
// (da_i = X_i da_lambda + source, df_i = I_i da_i). Role A adds role B's parts and
// multiplies by role C's M^-1, both read from LDS. Two workgroup barriers: after RNEA and
// the columns of M, and before the final products (beyond 16 bodies a third before the staged
// rows go out).

namespace gridq {

using grid::kConstStride;
using grid::prismatic;

// quad permutations: lane (0,1,2,3) reads lane (..); lane 3 shadows component 0
constexpr int kNb1 = 1 | (2 << 2) | (0 << 4) | (1 << 6);   // component c+1
constexpr int kNb2 = 2 | (0 << 2) | (1 << 4) | (2 << 6);   // component c+2
constexpr int kZ = 2 | (2 << 2) | (2 << 4) | (2 << 6);     // component 2 (the joint axis)
constexpr int kXS = 1 | (0 << 2) | (2 << 4) | (1 << 6);    // (x x e_z): lane 0 <- 1, 1 <- 0

template <int CTRL>
__device__ __forceinline__ float qperm(float x)
{
    return __builtin_bit_cast(
        float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xf, 0xf, true));
}

struct V {          // this lane's components of a 6-vector
    float a, l;
};

struct Nb {         // the quad neighbours' components: a1 = angular c+1, a2 = angular c+2, ...
    float a1, a2, l1, l2;
};

__device__ __forceinline__ Nb gather(V x)
{
    return Nb{qperm<kNb1>(x.a), qperm<kNb2>(x.a), qperm<kNb1>(x.l), qperm<kNb2>(x.l)};
}

struct Rot {        // this lane's entries of E: row c (e0, e1, e2) and column c (e0, f1, f2)
    float e0, e1, e2, f1, f2;
};

struct LaneK {      // per-lane body constants
    float rr1, rr2, I0, I1, I2, h1, h2;
};

struct Lane {       // per-lane selectors
    float sxs;      // (x x S)_c = sxs * x_{c+1 or c-1}: +1 for c = 0, -1 for c = 1, 0 for c = 2
    float sz;       // S_c: 1 for c = 2
    float g;        // component c of -g, the base acceleration that carries gravity
    float oh0, oh1, oh2;   // one-hot of the lane's component c
};

// a0: -g, the robot's base acceleration
__device__ __forceinline__ Lane lane_of(int c3, const float* a0)
{
    return Lane{c3 == 0 ? 1.0f : (c3 == 1 ? -1.0f : 0.0f), c3 == 2 ? 1.0f : 0.0f,
                c3 == 0 ? a0[0] : (c3 == 1 ? a0[1] : a0[2]),
                c3 == 0 ? 1.0f : 0.0f, c3 == 1 ? 1.0f : 0.0f, c3 == 2 ? 1.0f : 0.0f};
}

// X m = [E w; E (v - r x w)]
__device__ __forceinline__ V xmv(const Rot& e, const LaneK& k, V m, Nb n)
{
    V y;
    y.a = e.e0 * m.a + e.e1 * n.a1 + e.e2 * n.a2;
    const float t = m.l - k.rr1 * n.a2 + k.rr2 * n.a1;
    y.l = e.e0 * t + e.e1 * qperm<kNb1>(t) + e.e2 * qperm<kNb2>(t);
    return y;
}

// X^T f = [E^T n + r x (E^T f_l); E^T f_l]
__device__ __forceinline__ V xtfv(const Rot& e, const LaneK& k, V f, Nb n)
{
    const float l = e.e0 * f.l + e.f1 * n.l1 + e.f2 * n.l2;
    const float nn = e.e0 * f.a + e.f1 * n.a1 + e.f2 * n.a2;
    V y;
    y.a = nn + k.rr1 * qperm<kNb2>(l) - k.rr2 * qperm<kNb1>(l);
    y.l = l;
    return y;
}

// I x = [Ibar w + h x v; m v - h x w]
__device__ __forceinline__ V imv(const LaneK& k, float m, V x, Nb n)
{
    V y;
    y.a = k.I0 * x.a + k.I1 * n.a1 + k.I2 * n.a2 + (k.h1 * n.l2 - k.h2 * n.l1);
    y.l = m * x.l - (k.h1 * n.a2 - k.h2 * n.a1);
    return y;
}

// v x* f = [w x n + v_l x f_l; w x f_l]
__device__ __forceinline__ V crf(Nb v, Nb f)
{
    V y;
    y.a = v.a1 * f.a2 - v.a2 * f.a1 + v.l1 * f.l2 - v.l2 * f.l1;
    y.l = v.a1 * f.l2 - v.a2 * f.l1;
    return y;
}

// The joint axis is e_z of the joint frame: S = (e_z, 0) for a revolute joint (pr = false),
// (0, e_z) for a prismatic one (pr = true).

// S s: s in component 2 of the angular (revolute) or linear (prismatic) half
__device__ __forceinline__ V s_vec(const Lane& ln, bool pr, float s)
{
    return pr ? V{0.0f, ln.sz * s} : V{ln.sz * s, 0.0f};
}

// x + S s (the other half untouched)
__device__ __forceinline__ V add_s(const Lane& ln, bool pr, V x, float s)
{
    return pr ? V{x.a, x.l + ln.sz * s} : V{x.a + ln.sz * s, x.l};
}

// x x S: (x_1, -x_0, 0) in both halves (revolute); (0; w_1, -w_0, 0) (prismatic)
__device__ __forceinline__ V cross_s(const Lane& ln, bool pr, V x)
{
    const float pa = ln.sxs * qperm<kXS>(x.a);
    return pr ? V{0.0f, pa} : V{pa, ln.sxs * qperm<kXS>(x.l)};
}

// S x* f: (e_z x n; e_z x f_l) (revolute); (e_z x f_l; 0) (prismatic)
__device__ __forceinline__ V s_crf(const Lane& ln, bool pr, V f)
{
    const float pl = -ln.sxs * qperm<kXS>(f.l);
    return pr ? V{pl, 0.0f} : V{-ln.sxs * qperm<kXS>(f.a), pl};
}

// the half whose component 2 is S^T x (read on lane 2 of the quad)
__device__ __forceinline__ float s_half(bool pr, V x)
{
    return pr ? x.l : x.a;
}

__device__ __forceinline__ V add(V x, V y) { return V{x.a + y.a, x.l + y.l}; }

__device__ __forceinline__ V neg(V x) { return V{-x.a, -x.l}; }

template <int B, class T>
__device__ __forceinline__ T pick(const T (&arr)[B], int j)
{
    T r = arr[0];
#pragma unroll
    for (int i = 1; i < B; ++i)
        r = (i == j) ? arr[i] : r;
    return r;
}

__device__ __forceinline__ Rot pick_rot(const Rot& x, bool take, const Rot& keep)
{
    return Rot{take ? x.e0 : keep.e0, take ? x.e1 : keep.e1, take ? x.e2 : keep.e2,
               take ? x.f1 : keep.f1, take ? x.f2 : keep.f2};
}

template <class S>
__device__ __forceinline__ constexpr bool is_anc(int a, int i)
{
    return (S::anc[i] >> a) & 1ull;
}

// Columns j >= JMIN only: body i carries a nonzero forward derivative only in the subtree of
// j (local indices >= j), and a nonzero backward one only there or on j's ancestor path.
// Known at compile time once the body loops are unrolled, so the dead bodies cost nothing.
template <class S, int JMIN>
__device__ __forceinline__ constexpr bool live_back(int i)
{
    if (i >= JMIN)
        return true;
    for (int k = JMIN; k < S::B; ++k)
        if (is_anc<S>(i, k))
            return true;
    return false;
}

template <class I>
__device__ __forceinline__ float mass(int i)
{
    return I::consts()[i * kConstStride + 21];
}

// ------------------------------------------------------------------ building blocks

// The workgroup copies the model's lane table of branch I to LDS (16 floats per lane
// component c and body: r_c+1, r_c+2, Ibar_cc, Ibar_c,c+1, Ibar_c+2,c, h_c+1, h_c+2 and
// E_T[row][(c + col) % 3]); returns this lane's part. Every thread of the workgroup calls it.
template <class I, int THREADS>
__device__ __forceinline__ const float* lane_table(float4 (&s_tab)[3 * I::S::B * 4], int tid,
                                                   int c)
{
    for (int e = tid; e < 3 * I::S::B * 4; e += THREADS)
        s_tab[e] = reinterpret_cast<const float4*>(I::lanek())[e];
    __syncthreads();                          // lane table in LDS
    return reinterpret_cast<const float*>(s_tab) + (c == 3 ? 0 : c) * I::S::B * 16;
}

// The lane's share of every body: E_i = E_z(q_i) E_T,i from the hardware sin and cos (angle
// in revolutions, reduced to [0, 1)), or E_i = E_T,i and r_i = r_T,i + q_i E_T,i^T e_z for a
// prismatic joint, and the per-lane constants from the lane table (`tab`, this lane's part):
// four 16-byte LDS reads per body. Row c of E is alpha E_T,0 + beta E_T,1 + gamma E_T,2 with
// (alpha, beta, gamma) = (cos, sin, 0), (-sin, cos, 0), (0, 0, 1) for c = 0, 1, 2 (rows of
// E_z); the lane keeps its row in the order (E_cc, E_c,c+1, E_c,c+2), and the column entries
// E_c+1,c and E_c+2,c are the neighbours' third and second row entries.
template <class I>
__device__ __forceinline__ void make_body(int i, float qi, const Lane& ln, const float* tab,
                                          Rot& E, LaneK& K)
{
    const float4* t = reinterpret_cast<const float4*>(tab + i * 16);
    const float4 t0 = t[0], t1 = t[1], t2 = t[2], t3 = t[3];
    // t1.w, t2, t3: E_T[row][(c + col) % 3] at 3 row + col
    const float pT[3][3] = {{t1.w, t2.x, t2.y}, {t2.z, t2.w, t3.x}, {t3.y, t3.z, t3.w}};
    K = LaneK{t0.x, t0.y, t0.z, t0.w, t1.x, t1.y, t1.z};
    float sn = 0.0f, co = 1.0f;                      // prismatic: E = E_T
    if (prismatic<I>(i)) {
        // r = r_T + q E_T^T e_z: components c+1 and c+2 of the third row of E_T
        K.rr1 += qi * pT[2][1];
        K.rr2 += qi * pT[2][2];
    } else {
        const float rev = __builtin_amdgcn_fractf(qi * 0.159154943091895336f);
        sn = __builtin_amdgcn_sinf(rev);
        co = __builtin_amdgcn_cosf(rev);
    }
    const float al = ln.oh0 * co - ln.oh1 * sn;
    const float be = ln.oh0 * sn + ln.oh1 * co;
    E.e0 = al * pT[0][0] + be * pT[1][0] + ln.oh2 * pT[2][0];
    E.e1 = al * pT[0][1] + be * pT[1][1] + ln.oh2 * pT[2][1];
    E.e2 = al * pT[0][2] + be * pT[1][2] + ln.oh2 * pT[2][2];
    E.f1 = qperm<kNb1>(E.e2);
    E.f2 = qperm<kNb2>(E.e1);
}

template <class I, bool kQd = true>
__device__ __forceinline__ void load_bodies(const float* q_in, const float* qd_in, long vbase,
                                                const Lane& ln, const float* tab,
                                                float (&qd)[I::S::B], Rot (&E)[I::S::B],
                                                LaneK (&K)[I::S::B])
{
#pragma unroll
    for (int i = 0; i < I::S::B; ++i) {
        const long o = vbase + I::body[i];
        const float qi = q_in[o];
        qd[i] = kQd ? qd_in[o] : 0.0f;
        make_body<I>(i, qi, ln, tab, E[i], K[i]);
    }
}

// RNEA(q, qd, 0): v_i, gamma_i = I_i v_i, f_i accumulated inward, and xa0_i = X_i a_lambda(i)
template <class I>
__device__ __forceinline__ void rnea0(const Lane& ln, const float (&qd)[I::S::B],
                                      const Rot (&E)[I::S::B], const LaneK (&K)[I::S::B],
                                      V (&v)[I::S::B], V (&gam)[I::S::B], V (&F)[I::S::B],
                                      V (&xa0)[I::S::B])
{
    using S = typename I::S;
    constexpr int B = S::B;
    V a[B];
    Nb na[B], nv[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
        const int p = S::parent[i];
        V xv;
        if (p >= 0) {
            xv = xmv(E[i], K[i], v[p < 0 ? 0 : p], nv[p < 0 ? 0 : p]);
            xa0[i] = xmv(E[i], K[i], a[p < 0 ? 0 : p], na[p < 0 ? 0 : p]);
        } else {
            xv = V{0.0f, 0.0f};
            const V g{0.0f, ln.g};
            xa0[i] = xmv(E[i], K[i], g, gather(g));
        }
        const bool pr = prismatic<I>(i);
        v[i] = add_s(ln, pr, xv, qd[i]);
        nv[i] = gather(v[i]);
        const V vxs = cross_s(ln, pr, v[i]);       // a_i = X a_lambda + (v_i x S) qd_i
        a[i] = V{xa0[i].a + vxs.a * qd[i], xa0[i].l + vxs.l * qd[i]};
        na[i] = gather(a[i]);
        gam[i] = imv(K[i], mass<I>(i), v[i], nv[i]);
        F[i] = add(imv(K[i], mass<I>(i), a[i], na[i]), crf(nv[i], gather(gam[i])));
    }
#pragma unroll
    for (int i = B - 1; i >= 0; --i) {
        const int p = S::parent[i];
        if (p >= 0)
            F[p < 0 ? 0 : p] = add(F[p < 0 ? 0 : p], xtfv(E[i], K[i], F[i], gather(F[i])));
    }
}

// RNEA(q, qd, qdd): v_i, gamma_i = I_i v_i, f_i accumulated inward, and xa_i = X_i a_lambda(i)
// (a_lambda at this qdd)
template <class I>
__device__ __forceinline__ void rnea_at(const Lane& ln, const float (&qd)[I::S::B],
                                        const float (&qdd)[I::S::B], const Rot (&E)[I::S::B],
                                        const LaneK (&K)[I::S::B], V (&v)[I::S::B],
                                        V (&gam)[I::S::B], V (&F)[I::S::B], V (&xa)[I::S::B])
{
    using S = typename I::S;
    constexpr int B = S::B;
    V a[B];
    Nb na[B], nv[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
        const int p = S::parent[i];
        V xv;
        if (p >= 0) {
            xv = xmv(E[i], K[i], v[p < 0 ? 0 : p], nv[p < 0 ? 0 : p]);
            xa[i] = xmv(E[i], K[i], a[p < 0 ? 0 : p], na[p < 0 ? 0 : p]);
        } else {
            xv = V{0.0f, 0.0f};
            const V g{0.0f, ln.g};
            xa[i] = xmv(E[i], K[i], g, gather(g));
        }
        const bool pr = prismatic<I>(i);
        v[i] = add_s(ln, pr, xv, qd[i]);
        nv[i] = gather(v[i]);
        const V vxs = cross_s(ln, pr, v[i]);   // a_i = X a_lambda + S qdd_i + (v_i x S) qd_i
        const V xs = add_s(ln, pr, xa[i], qdd[i]);
        a[i] = V{xs.a + vxs.a * qd[i], xs.l + vxs.l * qd[i]};
        na[i] = gather(a[i]);
        gam[i] = imv(K[i], mass<I>(i), v[i], nv[i]);
        F[i] = add(imv(K[i], mass<I>(i), a[i], na[i]), crf(nv[i], gather(gam[i])));
    }
#pragma unroll
    for (int i = B - 1; i >= 0; --i) {
        const int p = S::parent[i];
        if (p >= 0)
            F[p < 0 ? 0 : p] = add(F[p < 0 ? 0 : p], xtfv(E[i], K[i], F[i], gather(F[i])));
    }
}

// column jm of M as ID(q, 0, e_jm) without gravity; M_i,jm = S^T f_i is s_half(f_i) on
// lane 2 of the quad. JMIN: jm >= JMIN is known (rows outside jm's subtree and ancestor path
// come out zero)
template <class I, int JMIN = 0>
__device__ __forceinline__ void m_column(const Lane& ln, const Rot (&E)[I::S::B],
                                         const LaneK (&K)[I::S::B], int jm, V (&fm)[I::S::B],
                                         V (&am)[I::S::B])
{
    using S = typename I::S;
    constexpr int B = S::B;
    Nb nam[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
        const int p = S::parent[i];
        if (i < JMIN) {                       // not in the subtree of jm
            fm[i] = V{0.0f, 0.0f};
            am[i] = V{0.0f, 0.0f};
            continue;
        }
        if (p >= JMIN)
            am[i] = xmv(E[i], K[i], am[p < 0 ? 0 : p], nam[p < 0 ? 0 : p]);
        else
            am[i] = V{0.0f, 0.0f};
        const float e = (i == jm) ? ln.sz : 0.0f;
        am[i] = prismatic<I>(i) ? V{am[i].a, am[i].l + e} : V{am[i].a + e, am[i].l};
        nam[i] = gather(am[i]);
        fm[i] = imv(K[i], mass<I>(i), am[i], nam[i]);
    }
#pragma unroll
    for (int i = B - 1; i >= 0; --i) {
        const int p = S::parent[i];
        if (p >= 0 && live_back<S, JMIN>(i))
            fm[p < 0 ? 0 : p] = add(fm[p < 0 ? 0 : p], xtfv(E[i], K[i], fm[i], gather(fm[i])));
    }
}

template <class I, int JMIN = 0>
__device__ __forceinline__ void m_column(const Lane& ln, const Rot (&E)[I::S::B],
                                         const LaneK (&K)[I::S::B], int jm, V (&fm)[I::S::B])
{
    V am[I::S::B];
    m_column<I, JMIN>(ln, E, K, jm, fm, am);
}

// M = L^T L in place (L lower triangular, nonzero on ancestor paths only): for k from the
// leaves, L_kk = sqrt(M_kk), L_ka = M_ka / L_kk, M_ab -= L_ka L_kb (a, b ancestors of k)
template <class S>
__device__ __forceinline__ void ltl_factor(float (&Lf)[S::B][S::B], float (&dinv)[S::B])
{
    constexpr int B = S::B;
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
}

// x <- (L^T L)^-1 x
template <class S>
__device__ __forceinline__ void ltl_solve(const float (&Lf)[S::B][S::B], const float (&dinv)[S::B],
                                          float (&x)[S::B])
{
    constexpr int B = S::B;
#pragma unroll
    for (int k = B - 1; k >= 0; --k) {
        x[k] *= dinv[k];
#pragma unroll
        for (int a = 0; a < B; ++a)
            if (is_anc<S>(a, k))
                x[a] -= Lf[k][a] * x[k];
    }
#pragma unroll
    for (int k = 0; k < B; ++k) {
#pragma unroll
        for (int a = 0; a < B; ++a)
            if (is_anc<S>(a, k))
                x[k] -= Lf[k][a] * x[a];
        x[k] *= dinv[k];
    }
}

// RNEA increments at qdd (RNEA is affine in qdd): Da_i = X_i Da_lambda + S qdd_i,
// Df_i = I_i Da_i accumulated inward. Returns xd_i = X_i Da_lambda(i) and Df_i.
template <class I>
__device__ __forceinline__ void delta_rnea(const Lane& ln, const Rot (&E)[I::S::B],
                                           const LaneK (&K)[I::S::B], const float (&qdd)[I::S::B],
                                           V (&xd)[I::S::B], V (&Df)[I::S::B])
{
    using S = typename I::S;
    constexpr int B = S::B;
    V Da[B];
    Nb nDa[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
        const int p = S::parent[i];
        xd[i] = V{0.0f, 0.0f};
        if (p >= 0)
            xd[i] = xmv(E[i], K[i], Da[p < 0 ? 0 : p], nDa[p < 0 ? 0 : p]);
        Da[i] = add_s(ln, prismatic<I>(i), xd[i], qdd[i]);
        nDa[i] = gather(Da[i]);
        Df[i] = imv(K[i], mass<I>(i), Da[i], nDa[i]);
    }
#pragma unroll
    for (int i = B - 1; i >= 0; --i) {
        const int p = S::parent[i];
        if (p >= 0)
            Df[p < 0 ? 0 : p] = add(Df[p < 0 ? 0 : p], xtfv(E[i], K[i], Df[i], gather(Df[i])));
    }
}

// One dRNEA column (Algorithm 1 forward, then the backward pass) with sources src_v, src_a
// entering at body j and src_f entering j's parent. kVel = false is the sweep with dv = 0
// (da_i = X_i da_lambda + source, df_i = I_i da_i). Returns dtau (every lane of the quad).
template <class I, bool kVel, int JMIN = 0>
__device__ __forceinline__ void drnea_column(const Lane& ln, const float (&qd)[I::S::B],
                                             const Rot (&E)[I::S::B], const LaneK (&K)[I::S::B],
                                             const V (&v)[I::S::B], const V (&gam)[I::S::B],
                                             int j, V src_v, V src_a, V src_f,
                                             float (&dx)[I::S::B])
{
    using S = typename I::S;
    constexpr int B = S::B;
    V df[B];
    {
        V dv[B], da[B];
        Nb ndv[B], nda[B];
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const int p = S::parent[i];
            if (i < JMIN) {                   // j >= JMIN: not in the subtree of j
                df[i] = V{0.0f, 0.0f};
                continue;
            }
            const float sel = (i == j) ? 1.0f : 0.0f;
            V xdv{0.0f, 0.0f}, xda{0.0f, 0.0f};
            if (p >= JMIN) {
                if constexpr (kVel)
                    xdv = xmv(E[i], K[i], dv[p < 0 ? 0 : p], ndv[p < 0 ? 0 : p]);
                xda = xmv(E[i], K[i], da[p < 0 ? 0 : p], nda[p < 0 ? 0 : p]);
            }
            if constexpr (kVel) {
                dv[i] = V{xdv.a + sel * src_v.a, xdv.l + sel * src_v.l};
                ndv[i] = gather(dv[i]);
                const V dvxs = cross_s(ln, prismatic<I>(i), dv[i]);
                da[i] = V{xda.a + dvxs.a * qd[i] + sel * src_a.a,
                          xda.l + dvxs.l * qd[i] + sel * src_a.l};
            } else {
                da[i] = V{xda.a + sel * src_a.a, xda.l + sel * src_a.l};
            }
            nda[i] = gather(da[i]);
            df[i] = imv(K[i], mass<I>(i), da[i], nda[i]);
            if constexpr (kVel) {
                // df_i = I_i da_i + dv_i x* gamma_i + v_i x* (I_i dv_i)
                const V Idv = imv(K[i], mass<I>(i), dv[i], ndv[i]);
                df[i] = add(add(df[i], crf(ndv[i], gather(gam[i]))), crf(gather(v[i]), gather(Idv)));
            }
        }
    }
#pragma unroll
    for (int i = B - 1; i >= 0; --i) {
        if (!live_back<S, JMIN>(i)) {         // off j's subtree and ancestor path
            dx[i] = 0.0f;
            continue;
        }
        dx[i] = qperm<kZ>(s_half(prismatic<I>(i), df[i]));
        const int p = S::parent[i];
        if (p >= 0) {
            const float sel = (i == j) ? 1.0f : 0.0f;
            const V y = xtfv(E[i], K[i], df[i], gather(df[i]));
            df[p < 0 ? 0 : p] = V{df[p < 0 ? 0 : p].a + y.a + sel * src_f.a,
                                  df[p < 0 ? 0 : p].l + y.l + sel * src_f.l};
        }
    }
}

// X_j^T (S x* f): the backward source of a q-column (pj: joint j is prismatic)
__device__ __forceinline__ V back_source(const Lane& ln, bool pj, const Rot& Ej, const LaneK& Kj,
                                         V f)
{
    const V sxf = s_crf(ln, pj, f);
    return xtfv(Ej, Kj, sxf, gather(sxf));
}

template <class I>
__device__ __forceinline__ void pick_joint(const Rot (&E)[I::S::B], const LaneK (&K)[I::S::B],
                                           int j, Rot& Ej, LaneK& Kj)
{
    Ej = E[0];
    Kj = K[0];
#pragma unroll
    for (int i = 1; i < I::S::B; ++i) {
        Ej = pick_rot(E[i], i == j, Ej);
        Kj.rr1 = (i == j) ? K[i].rr1 : Kj.rr1;
        Kj.rr2 = (i == j) ? K[i].rr2 : Kj.rr2;
    }
}

// zeros of this branch's rows in the other branches' columns
template <class I>
__device__ __forceinline__ void zero_fill(float* out0, float* out1, long mbase, int lane,
                                          int lanes)
{
    constexpr int B = I::S::B;
    constexpr int N = I::N;
    if constexpr (N > B) {
        for (int e = lane; e < B * N; e += lanes) {
            const int i = e / N, c2 = e % N;
            if (!I::contains(c2)) {
                const long o = mbase + (long)I::body_of(i) * N + c2;
                out0[o] = 0.0f;
                if (out1)
                    out1[o] = 0.0f;
            }
        }
    }
}

// ------------------------------------------------------------------ grid_fdgrad_quad

template <class I>
__device__ __forceinline__ void run_fused(const grid::Args& A, int block)
{
    using S = typename I::S;
    constexpr int B = S::B;
    constexpr int Q = S::Q;                   // quads per wavefront per problem
    constexpr int W = S::W;                   // wavefronts per problem
    constexpr int WB = GRID_WAVES;            // wavefronts per workgroup
    constexpr int PW = 16 / Q;                // problems per wavefront (W == 1)
    constexpr int P = (WB / W) * PW;          // problems per workgroup
    constexpr int N = I::N;
    __shared__ float s_M[P][B][B];
    __shared__ float4 s_tab[3 * B * 4];

    const int tid = (int)threadIdx.x;
    const int wave = tid / 64;
    const int lane = tid % 64;
    const int c = lane & 3;
    const Lane ln = lane_of(c == 3 ? 0 : c, I::a0());
    const int quad = (lane / 4) % Q;
    const int pslot = (wave / W) * PW + (lane / 4) / Q;     // problem in the workgroup
    const int s = quad + Q * (wave % W);                    // column slot in the problem
    const int kraw = block * P + pslot;
    const bool valid = kraw < A.nknots;
    const int knot = valid ? kraw : A.nknots - 1;           // tail slots recompute the last knot

    // roles: M column jm = s, derivative column (u, j): u = 0 -> d/dq, u = 1 -> d/dqd
    const int jm = s < B ? s : 0;
    const bool owns_m = s < B;
    const bool owns_col = s < 2 * B;
    const int u = owns_col ? s / B : 1;
    const int j = s % B;
    const long vbase = (long)knot * N;
    const long mbase = (long)knot * N * N;

    float qd[B];
    Rot E[B];
    LaneK K[B];
    load_bodies<I>(A.q, A.qd, vbase, ln, lane_table<I, 64 * WB>(s_tab, tid, c), qd, E, K);

    V v[B], gam[B], F[B], xa0[B];
    rnea0<I>(ln, qd, E, K, v, gam, F, xa0);
    float x[B];                               // tau - c, then qdd
#pragma unroll
    for (int i = 0; i < B; ++i)
        x[i] = A.tau[vbase + I::body[i]] - qperm<kZ>(s_half(prismatic<I>(i), F[i]));

    {
        V fm[B];
        m_column<I>(ln, E, K, jm, fm);
        if (owns_m && c == 2) {
#pragma unroll
            for (int i = 0; i < B; ++i)
                s_M[pslot][i][jm] = s_half(prismatic<I>(i), fm[i]);
        }
    }
    __syncthreads();
    float Lf[B][B], dinv[B];
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
        for (int b = 0; b <= i; ++b)
            if (b == i || is_anc<S>(b, i))
                Lf[i][b] = s_M[pslot][i][b];
    ltl_factor<S>(Lf, dinv);
    ltl_solve<S>(Lf, dinv, x);                // qdd

    V xd[B], Df[B];
    delta_rnea<I>(ln, E, K, x, xd, Df);
    const V xdj = pick<B>(xd, j), Dfj = pick<B>(Df, j);
    Rot Ej;
    LaneK Kj;
    pick_joint<I>(E, K, j, Ej, Kj);
    const V vj = pick<B>(v, j);
    const bool pj = prismatic<I>(j);
    // sources of column (u, j):
    //   u = q : dv += v_j x S, da += (X_j a_lambda(j)) x S, backward += X_j^T (S x* f_j)
    //   u = qd: dv += S,       da += v_j x S
    const V vxs = cross_s(ln, pj, vj);
    const V src_v = u == 0 ? vxs : s_vec(ln, pj, 1.0f);
    const V src_a = u == 0 ? cross_s(ln, pj, add(pick<B>(xa0, j), xdj)) : vxs;
    const V zeta = back_source(ln, pj, Ej, Kj, add(pick<B>(F, j), Dfj));
    const V src_f = u == 0 ? zeta : V{0.0f, 0.0f};

    float dx[B];
    drnea_column<I, true>(ln, qd, E, K, v, gam, j, src_v, src_a, src_f, dx);
    ltl_solve<S>(Lf, dinv, dx);               // M^-1 dtau/du_j
    float mc[B];                              // column jm of M^-1
#pragma unroll
    for (int i = 0; i < B; ++i)
        mc[i] = (i == jm) ? 1.0f : 0.0f;
    ltl_solve<S>(Lf, dinv, mc);
    if (!valid)
        return;
    // lane c of a quad stores the rows i with i % 4 == c
#pragma unroll
    for (int i = 0; i < B; ++i) {
        if ((i & 3) != c)
            continue;
        const int gi = I::body[i];
        if (s == 0)
            A.qdd[vbase + gi] = x[i];
        if (owns_col) {
            float* out = u == 0 ? A.dqdd_dq : A.dqdd_dqd;
            out[mbase + (long)gi * N + I::body_of(j)] = -dx[i];
        }
        // entry (i, jm) with i <= jm is written to both mirrored positions by the quad
        // owning column jm, so M^-1 comes out exactly symmetric
        if (owns_m && i <= jm) {
            const int gj = I::body_of(jm);
            A.Minv[mbase + (long)gi * N + gj] = mc[i];
            A.Minv[mbase + (long)gj * N + gi] = mc[i];
        }
    }
    const int lp = lane % (4 * Q) + 64 * (wave % W);        // lane within the problem
    zero_fill<I>(A.Minv, nullptr, mbase, lp, 4 * Q * W);
    zero_fill<I>(A.dqdd_dq, A.dqdd_dqd, mbase, lp, 4 * Q * W);
}

// ------------------------------------------------------------------ grid_fdgrad_pipe

// columns s and s + 16 (those below B) of M^-1 from the factor: to LDS (for the final
// products) and to the output, entries (i, jm), i <= jm, in both mirrored positions so that
// M^-1 comes out exactly symmetric; then this branch's zeros in other branches' columns
template <class I, int CB, int P, bool kLds = true>
__device__ __forceinline__ void minv_columns(float* Minv, const float (&Lf)[I::S::B][I::S::B],
                                             const float (&dinv)[I::S::B], int pslot, int s, int c,
                                             bool valid, long mbase, int lp, int lanes,
                                             float (&s_Mi)[P][I::S::B][I::S::B])
{
    using S = typename I::S;
    constexpr int B = S::B;
    constexpr int N = I::N;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const bool owns = s + 16 * cb < B;
        const int jm = owns ? s + 16 * cb : 0;
        float mc[B];
#pragma unroll
        for (int i = 0; i < B; ++i)
            mc[i] = (i == jm) ? 1.0f : 0.0f;
        ltl_solve<S>(Lf, dinv, mc);
        if (owns) {
#pragma unroll
            for (int i = 0; i < B; ++i) {
                if ((i & 3) != c)
                    continue;
                if constexpr (kLds)
                    s_Mi[pslot][i][jm] = mc[i];
                if (valid && i <= jm) {
                    const int gi = I::body[i];
                    const int gj = I::body_of(jm);
                    Minv[mbase + (long)gi * N + gj] = mc[i];
                    Minv[mbase + (long)gj * N + gi] = mc[i];
                }
            }
        }
    }
    if (valid)
        zero_fill<I>(Minv, nullptr, mbase, lp, lanes);
}

// x[r4 + c] for the lane's c (0..3) in an unrolled loop over r4 = 0, 4, ..; 0 past the end.
// The pick is a sum of the four candidates times the lane's 0/1 masks mk[k] = (c == k): a chain
// of selects folds into one indexed load, and the array then moves to scratch memory.
template <int B>
__device__ __forceinline__ float row_of_four(const float (&x)[B], int r4, const float (&mk)[4])
{
    float v = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (r4 + k < B)
            v += mk[k] * x[r4 + k];
    return v;
}

// Beyond 16 bodies (one problem per workgroup) the problem's rows of M^-1, dqdd/dq and
// dqdd/dqd are staged in LDS in local coordinates and the workgroup writes the B rows of N
// floats of each matrix, zeros outside the branch's columns included: consecutive threads take
// consecutive elements of a row, and no other pass writes those rows.
template <class I>
__device__ __forceinline__ void write_rows(const grid::Args& A, long mbase,
                                           const float (&tile)[3][I::S::B][I::S::B],
                                           const int* rowg, const int* locc, int t, int threads)
{
    constexpr int B = I::S::B;
    constexpr int N = I::N;
    for (int e = t; e < B * N; e += threads) {
        const int r = e / N, c2 = e - (e / N) * N;
        const int l = locc[c2];
        const long o = mbase + (long)rowg[r] * N + c2;
        float m = 0.0f, d = 0.0f, w = 0.0f;
        if (l >= 0) {
            m = tile[0][r][l];
            d = tile[1][r][l];
            w = tile[2][r][l];
        }
        A.Minv[o] = m;
        A.dqdd_dq[o] = d;
        A.dqdd_dqd[o] = w;
    }
}

template <int B>
struct PipeShape {
    static_assert(B >= 1 && B <= 32, "branches have at most 32 bodies");
    static constexpr int pow2(int x) { return x <= 1 ? 1 : 2 * pow2((x + 1) / 2); }
    static constexpr int CB = B <= 16 ? 1 : 2;            // role B: columns per quad
    static constexpr int QB = B <= 16 ? pow2(B) : 16;     // role B: quads per problem
    static constexpr int QA = 2 * B <= 16 ? 2 * QB : 16;  // role A: quads per wavefront
    static constexpr int WA = (2 * B + 15) / 16;          // role A: wavefronts per problem
    static constexpr int P = 16 / QB;                     // problems per workgroup
    static constexpr int PA = WA == 1 ? 16 / QA : 1;      // role A: problems per wavefront
    static constexpr int AW = WA == 1 ? 2 : WA;           // role A: wavefronts per workgroup
    // role C (M^-1 on its own wavefront) up to 16 bodies; beyond, role B computes M^-1 and
    // the workgroup stays at four wavefronts (one per SIMD, the full register file each)
    static constexpr bool HASC = B <= 16;
    static constexpr int WAVES = AW + 1 + (HASC ? 1 : 0);
    static_assert(WA > 1 || P == 2 * PA, "two role-A wavefronts serve the workgroup");
    static_assert(WA == 1 || P == 1, "one problem per workgroup beyond 8 bodies");
};

// kLoop: the call sits in a loop over blocks (the persistent mixed kernel). The thread index is
// then passed through an empty asm statement, so that nothing derived from it counts as loop
// invariant: hoisted out of the loop, the per-lane set-up would stay live across iterations
// beside the block's own state. The wavefront index is made uniform again explicitly.
template <class I, bool kLoop = false>
__device__ __forceinline__ void run_pipe(const grid::Args& A, int block)
{
    using S = typename I::S;
    constexpr int B = S::B;
    using PS = PipeShape<B>;
    constexpr int P = PS::P;
    constexpr int N = I::N;
    constexpr int BWAVE = PS::AW;             // role A on wavefronts 0 .. AW-1, then B, then C
    constexpr int CWAVE = PS::HASC ? PS::AW + 1 : -1;
    static_assert(P == S::PP, "problems per workgroup disagree with the generated shape");
    static_assert(PS::WAVES <= GRID_PIPE_WAVES, "workgroup too small for the shape");
    __shared__ float s_c[P][B];               // bias forces c (role A -> B)
    __shared__ float s_M[P][B][B];            // M columns (role B -> B, C)
    __shared__ float s_Mi[P][B][B];           // M^-1, row-major (role C -> A); beyond 16
                                              // bodies the factor L instead (B -> A)
    __shared__ float s_dinv[P][B];            // 1 / L_kk beyond 16 bodies (B -> A)
    __shared__ float s_D[P][B][B];            // qdd part of the q-columns, [column][row] (B -> A)
    // role B's weighted unit-acceleration responses, [problem][quad][body][component]: the
    // increments at qdd summed over the quads (branches of up to 16 bodies)
    __shared__ float4 s_red[B <= 16 ? P : 1][B <= 16 ? PS::QB : 1][B <= 16 ? B : 1][3];
    // beyond 16 bodies (one problem per workgroup, columns in two passes): role B's unweighted
    // unit-acceleration responses, [column k][body][component] = (a.a, a.l, f.a, f.l)
    __shared__ float4 s_resp[B > 16 ? B : 1][B > 16 ? B : 1][3];
    __shared__ float4 s_tab[3 * B * 4];       // the model's lane table (roles A, B)
    // beyond 16 bodies: the staged output rows (M^-1, dqdd/dq, dqdd/dqd in local coordinates),
    // local row -> global row, global column -> local column (-1: not in the branch)
    constexpr bool kStage = !PS::HASC;
    __shared__ float s_out[3][kStage ? B : 1][kStage ? B : 1];
    __shared__ int s_rowg[kStage ? B : 1];
    __shared__ int s_locc[kStage ? N : 1];
    // beyond 16 bodies role B publishes its factor after the first barrier and raises this
    // flag; role A needs the factor only after its dRNEA column and waits for the flag there
    __shared__ int s_lflag;

    int tid = (int)threadIdx.x;
    if constexpr (kLoop)
        asm volatile("" : "+v"(tid));
    const int wave = kLoop ? __builtin_amdgcn_readfirstlane(tid >> 6) : tid / 64;
    const int lane = kLoop ? (tid & 63) : tid % 64;
    const int c = lane & 3;
    const Lane ln = lane_of(c == 3 ? 0 : c, I::a0());
    if constexpr (kStage) {                   // ordered by the lane table's barrier
        if (tid == 0)
            s_lflag = 0;
        if (tid < B)
            s_rowg[tid] = I::body_of(tid);
        if (tid < N) {
            int l = -1;
#pragma unroll
            for (int k = 0; k < B; ++k)
                l = I::body[k] == tid ? k : l;
            s_locc[tid] = l;
        }
    }
    const float* tab = lane_table<I, 64 * GRID_PIPE_WAVES>(s_tab, tid, c);
    // the staged rows go out once the last tile is written (one problem per workgroup)
    const auto stage_out = [&]() {
        if constexpr (kStage) {
            __syncthreads();                  // the output tiles are complete
            if (block * P < A.nknots)
                write_rows<I>(A, (long)(block * P) * N * N, s_out, s_rowg, s_locc, tid,
                              64 * GRID_PIPE_WAVES);
        }
    };

    if (wave < PS::AW) {
        // -------------------------------------------------------- role A
        constexpr int QA = PS::QA;
        const int pslot = PS::WA == 1 ? wave * PS::PA + (lane / 4) / QA : 0;
        const int s = PS::WA == 1 ? (lane / 4) % QA : lane / 4 + 16 * wave;
        const int kraw = block * P + pslot;
        const bool valid = kraw < A.nknots;
        const int knot = valid ? kraw : A.nknots - 1;
        const bool owns_col = s < 2 * B;
        const int u = owns_col ? s / B : 1;
        const int j = s % B;
        const long vbase = (long)knot * N;
        const long mbase = (long)knot * N * N;

        float qd[B];
        Rot E[B];
        LaneK K[B];
        load_bodies<I>(A.q, A.qd, vbase, ln, tab, qd, E, K);
        V v[B], gam[B], F[B], xa0[B];
        rnea0<I>(ln, qd, E, K, v, gam, F, xa0);
        if (s == 0 && c == 2) {               // quad 0 of each problem publishes c
#pragma unroll
            for (int i = 0; i < B; ++i)
                s_c[pslot][i] = s_half(prismatic<I>(i), F[i]);
        }
        __syncthreads();                      // c published

        // (computed before the barrier, where this wavefront waits, these sources made every
        // launch 20-25% slower: after it they interleave with the start of the column sweep)
        Rot Ej;
        LaneK Kj;
        pick_joint<I>(E, K, j, Ej, Kj);
        const bool pj = prismatic<I>(j);
        const V vxs = cross_s(ln, pj, pick<B>(v, j));
        const V src_v = u == 0 ? vxs : s_vec(ln, pj, 1.0f);
        const V src_a = u == 0 ? cross_s(ln, pj, pick<B>(xa0, j)) : vxs;
        const V zeta = back_source(ln, pj, Ej, Kj, pick<B>(F, j));
        const V src_f = u == 0 ? zeta : V{0.0f, 0.0f};
        float dx[B];
        drnea_column<I, true>(ln, qd, E, K, v, gam, j, src_v, src_a, src_f, dx);
        const int lp = PS::WA == 1 ? lane % (4 * QA) : lane + 64 * wave;
        float Lf[B][B], dinv[B];              // beyond 16 bodies: role B's factor
        float mk[4];                          // this lane's c as 0/1 masks (staged rows)
#pragma unroll
        for (int k = 0; k < 4; ++k)
            mk[k] = c == k ? 1.0f : 0.0f;
        if constexpr (!PS::HASC) {
            // role B published the factor right after the first barrier (thousands of cycles
            // before this point); the wait is bounded so that it ends in any case. The quad
            // of column (qd, j) solves for column j of M^-1 while role B is still on the qdd
            // parts (entries (i, j), i <= j, to both mirrored positions: exactly symmetric)
            for (int spin = 0; spin < (1 << 20); ++spin) {
                if (__hip_atomic_load(&s_lflag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP))
                    break;
                __builtin_amdgcn_s_sleep(1);
            }
            float mc[B];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                dinv[i] = s_dinv[pslot][i];
                mc[i] = (i == j) ? 1.0f : 0.0f;
#pragma unroll
                for (int b = 0; b < i; ++b)
                    if (is_anc<S>(b, i))
                        Lf[i][b] = s_Mi[pslot][i][b];
            }
            ltl_solve<S>(Lf, dinv, mc);
            if (owns_col && u == 1) {
                // lane c of the quad takes rows c, c + 4, ..; entries (i, j), i <= j, to both
                // mirrored positions of the staged M^-1 (exactly symmetric)
#pragma unroll
                for (int r = 0; r < (B + 3) / 4; ++r) {
                    const int i = c + 4 * r;
                    const float m = row_of_four<B>(mc, 4 * r, mk);
                    if (i < B && i <= j) {
                        s_out[0][i][j] = m;
                        s_out[0][j][i] = m;
                    }
                }
            }
        }
        __syncthreads();                      // M^-1 and the qdd parts published

        const float qpart = u == 0 ? 1.0f : 0.0f;
#pragma unroll
        for (int i = 0; i < B; ++i)
            dx[i] += qpart * s_D[pslot][j][i];
        if constexpr (!PS::HASC) {
            // beyond 16 bodies: dqdd/du_j = -(L^T L)^-1 dtau/du_j by the two triangular solves
            ltl_solve<S>(Lf, dinv, dx);
            if (owns_col) {
#pragma unroll
                for (int r = 0; r < (B + 3) / 4; ++r) {
                    const int i = c + 4 * r;
                    const float d = row_of_four<B>(dx, 4 * r, mk);
                    if (i < B)
                        s_out[1 + u][i][j] = -d;
                }
            }
            stage_out();
            return;
        }
        if (!valid)
            return;
        // dqdd/du_j = -M^-1 dtau/du_j; lane c of the quad computes and stores rows c, c+4, ..
        if (owns_col) {
            float* out = u == 0 ? A.dqdd_dq : A.dqdd_dqd;
            const int gj = I::body_of(j);
#pragma unroll
            for (int r = 0; r < (B + 3) / 4; ++r) {
                const int i = c + 4 * r;
                if (i < B) {
                    float acc = 0.0f;
#pragma unroll
                    for (int k = 0; k < B; ++k)
                        acc += s_Mi[pslot][i][k] * dx[k];
                    out[mbase + (long)I::body_of(i) * N + gj] = -acc;
                }
            }
        }
        zero_fill<I>(A.dqdd_dq, A.dqdd_dqd, mbase, lp, PS::WA == 1 ? 4 * QA : 64 * PS::WA);
    } else if (wave == BWAVE) {
        // -------------------------------------------------------- role B
        constexpr int QB = PS::QB;
        constexpr int CB = PS::CB;
        const int pslot = (lane / 4) / QB;
        const int s = (lane / 4) % QB;        // columns s, s + 16: of M and q-columns
        const int kraw = block * P + pslot;
        const bool valid = kraw < A.nknots;
        const int knot = valid ? kraw : A.nknots - 1;
        int js[CB];
        bool owns[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            owns[cb] = s + 16 * cb < B;
            js[cb] = owns[cb] ? s + 16 * cb : 0;
        }
        const long vbase = (long)knot * N;

        float qd[B];
        Rot E[B];
        LaneK K[B];
        load_bodies<I>(A.q, A.qd, vbase, ln, tab, qd, E, K);
        // the unit-acceleration responses of this quad's columns of M, kept for the increments
        // (up to 16 bodies: see below)
        constexpr bool kLinear = B <= 16;
        V amk[kLinear ? CB : 1][B], fmk[kLinear ? CB : 1][B];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            V fm[B], am[B];
            if (cb == 0)
                m_column<I>(ln, E, K, js[cb], fm, am);
            else                              // columns 16.. only
                m_column<I, 16>(ln, E, K, js[cb], fm, am);
            if (owns[cb] && c == 2) {
#pragma unroll
                for (int i = 0; i < B; ++i)
                    s_M[pslot][i][js[cb]] = s_half(prismatic<I>(i), fm[i]);
            }
            if constexpr (kLinear) {
#pragma unroll
                for (int i = 0; i < B; ++i) {
                    amk[cb][i] = am[i];
                    fmk[cb][i] = fm[i];
                }
            } else {
                // beyond 16 bodies the responses go to LDS as they come (two passes would
                // hold twice the registers across the barrier)
                if (owns[cb] && c != 3) {
#pragma unroll
                    for (int i = 0; i < B; ++i)
                        s_resp[js[cb]][i][c] = float4{am[i].a, am[i].l, fm[i].a, fm[i].l};
                }
            }
        }
        // the exchange stays inside this wavefront: order its LDS traffic only
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
        // up to 16 bodies the factor is used only after the barrier, and the scheduler would
        // sink it there, onto the chain that follows the barrier; taking its values as operands
        // of an empty statement keeps it before, where this wavefront waits anyway (chain7:
        // 4.46 -> 4.37 us per launch; beyond 16 bodies the factor's LDS copy keeps it there)
        if constexpr (PS::HASC) {
#pragma unroll
            for (int i = 0; i < B; ++i) {
                asm volatile("" : "+v"(dinv[i]));
#pragma unroll
                for (int b = 0; b < i; ++b)
                    if (is_anc<S>(b, i))
                        asm volatile("" : "+v"(Lf[i][b]));
            }
        }
        __syncthreads();                      // c published
        if constexpr (!PS::HASC) {
            // no role C beyond 16 bodies: the factor goes to role A, which finishes with
            // triangular solves (and the columns of M^-1); published after the barrier, so
            // that the barrier does not wait for it, and released through the flag
            if (lane == 0) {
#pragma unroll
                for (int i = 0; i < B; ++i) {
                    s_dinv[pslot][i] = dinv[i];
#pragma unroll
                    for (int b = 0; b < i; ++b)
                        if (is_anc<S>(b, i))
                            s_Mi[pslot][i][b] = Lf[i][b];
                }
                __hip_atomic_store(&s_lflag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }

        float x[B];
#pragma unroll
        for (int i = 0; i < B; ++i)
            x[i] = A.tau[vbase + I::body[i]] - s_c[pslot][i];
        ltl_solve<S>(Lf, dinv, x);            // qdd
        if (valid && s == 0) {
#pragma unroll
            for (int i = 0; i < B; ++i)
                if ((i & 3) == c)
                    A.qdd[vbase + I::body[i]] = x[i];
        }
        // per column of this quad: xd_j = X_j Da_lambda(j) and Df_j, the sources of its sweep
        V xdj[CB], Dfj[CB];
        if constexpr (kLinear) {
            // RNEA is linear in qdd: Da_i = sum_k qdd_k a_i^(k) and Df_i = sum_k qdd_k f_i^(k)
            // over the unit-acceleration responses of the columns k of M (quad k holds column
            // k's), so the increments are a sum over the problem's quads instead of another
            // sweep down and up the tree; xd_j = Da_j - S_j qdd_j. Each quad writes its weighted
            // responses of every body to LDS and sums the ones of its own bodies j over the
            // quads. qdd_k of the quad's column k comes as a sum of x_k times a 0/1 mask (a
            // chain of selects of the array's elements folds into one indexed load, and the
            // array then moves to memory).
            float wk[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                wk[cb] = 0.0f;
#pragma unroll
                for (int k = 0; k < B; ++k)
                    wk[cb] += (owns[cb] && js[cb] == k ? 1.0f : 0.0f) * x[k];
            }
            const int cc = c == 3 ? 0 : c;
            if (c != 3) {
#pragma unroll
                for (int i = 0; i < B; ++i) {
                    V da{0.0f, 0.0f}, df{0.0f, 0.0f};
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        da = V{da.a + wk[cb] * amk[cb][i].a, da.l + wk[cb] * amk[cb][i].l};
                        df = V{df.a + wk[cb] * fmk[cb][i].a, df.l + wk[cb] * fmk[cb][i].l};
                    }
                    s_red[pslot][s][i][cc] = float4{da.a, da.l, df.a, df.l};
                }
            }
            // the exchange stays inside this wavefront: order its LDS traffic only
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                float4 t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int q = 0; q < QB; ++q) {
                    const float4 u = s_red[pslot][q][js[cb]][cc];
                    t = float4{t.x + u.x, t.y + u.y, t.z + u.z, t.w + u.w};
                }
                xdj[cb] = add_s(ln, prismatic<I>(js[cb]), V{t.x, t.y}, -wk[cb]);
                Dfj[cb] = V{t.z, t.w};
            }
        } else {
            // the same sum beyond 16 bodies, from the responses role B left in LDS before the
            // first barrier: Da_j = sum_k qdd_k a_j^(k), Df_j = sum_k qdd_k f_j^(k) for the
            // quad's own bodies j (one problem per workgroup)
            const int cc = c == 3 ? 0 : c;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                float4 t{0.0f, 0.0f, 0.0f, 0.0f};
                float w = 0.0f;
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    const float4 u = s_resp[k][js[cb]][cc];
                    t = float4{t.x + x[k] * u.x, t.y + x[k] * u.y, t.z + x[k] * u.z,
                               t.w + x[k] * u.w};
                    w += (js[cb] == k ? 1.0f : 0.0f) * x[k];
                }
                xdj[cb] = add_s(ln, prismatic<I>(js[cb]), V{t.x, t.y}, -w);
                Dfj[cb] = V{t.z, t.w};
            }
        }
        V none[B];                            // velocities do not enter the dv = 0 sweep
#pragma unroll
        for (int i = 0; i < B; ++i)
            none[i] = V{0.0f, 0.0f};
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int j = js[cb];
            Rot Ej;
            LaneK Kj;
            pick_joint<I>(E, K, j, Ej, Kj);
            const bool pj = prismatic<I>(j);
            const V src_a = cross_s(ln, pj, xdj[cb]);
            const V src_f = back_source(ln, pj, Ej, Kj, Dfj[cb]);
            float dxc[B];
            if (cb == 0)
                drnea_column<I, false>(ln, qd, E, K, none, none, j, V{0.0f, 0.0f}, src_a,
                                       src_f, dxc);
            else                              // columns 16.. only
                drnea_column<I, false, 16>(ln, qd, E, K, none, none, j, V{0.0f, 0.0f}, src_a,
                                           src_f, dxc);
            if (owns[cb]) {
#pragma unroll
                for (int i = 0; i < B; ++i)
                    if ((i & 3) == c)
                        s_D[pslot][j][i] = dxc[i];
            }
        }
        __syncthreads();                      // M^-1 and the qdd parts published
        stage_out();
    } else if (wave == CWAVE) {
        // -------------------------------------------------------- role C
        constexpr int QB = PS::QB;
        constexpr int CB = PS::CB;
        const int pslot = (lane / 4) / QB;
        const int s = (lane / 4) % QB;        // columns s, s + 16 of M^-1
        const int kraw = block * P + pslot;
        const bool valid = kraw < A.nknots;
        const int knot = valid ? kraw : A.nknots - 1;
        const long mbase = (long)knot * N * N;
        __syncthreads();                      // role B's columns of M are in LDS
        float Lf[B][B], dinv[B];
#pragma unroll
        for (int i = 0; i < B; ++i)
#pragma unroll
            for (int b = 0; b <= i; ++b)
                if (b == i || is_anc<S>(b, i))
                    Lf[i][b] = s_M[pslot][i][b];
        ltl_factor<S>(Lf, dinv);
        minv_columns<I, CB>(A.Minv, Lf, dinv, pslot, s, c, valid, mbase, lane % (4 * QB), 4 * QB, s_Mi);
        __syncthreads();                      // M^-1 published
    } else {
        // a wavefront this shape does not use still takes part in the barriers
        __syncthreads();
        __syncthreads();
        stage_out();
    }
}

}  // namespace gridq

// kernels of a one-robot module (a module of several robots defines GRID_PIPE_ONLY and its
// own entry point, grid_fdgrad_pipe_mixed)
#ifndef GRID_PIPE_ONLY

// defined by the generated epilogue: workgroup -> (branch, problem group)
__device__ void grid_dispatch_q(const grid::Args& args, int block);

// Fused kernel, quad layout: GRID_WAVES wavefronts per workgroup.
extern "C" __global__ void __launch_bounds__(64 * GRID_WAVES) grid_fdgrad_quad(grid::Args args)
{
    grid_dispatch_q(args, (int)blockIdx.x);
}

// The three-role kernel (grid_fdgrad_pipe) has an entry point only in the module generated
// for it alone, which is compiled with its own schedule.

#endif  // GRID_PIPE_ONLY
