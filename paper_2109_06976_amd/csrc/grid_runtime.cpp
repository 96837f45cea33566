// libgrid host runtime: the C ABI declared in include/grid.h.
#include "grid_internal.h"

#include <cmath>
#include <algorithm>
#include <cstring>
#include <new>

using namespace grid_impl;

namespace grid_impl {

static thread_local std::string t_last_error;

void set_error(const std::string& msg) { t_last_error = msg; }

static grid_status fail_to(std::string* err, grid_status s, const std::string& msg)
{
    *err = msg;
    return s;
}

static bool finite_all(const double* p, size_t k)
{
    for (size_t i = 0; i < k; ++i)
        if (!std::isfinite(p[i]))
            return false;
    return true;
}

grid_status validate_desc(const grid_model_desc* d, std::string* err)
{
    if (!d)
        return fail_to(err, GRID_EINVAL, "model description is NULL");
    if (d->n < 1)
        return fail_to(err, GRID_EINVAL, "n must be >= 1");
    if (d->n > kMaxBodies)
        return fail_to(err, GRID_EUNSUPPORTED, "n > " + std::to_string(kMaxBodies) + " is not supported");
    if (!d->parent || !d->tree_rot || !d->tree_pos || !d->mass || !d->com || !d->inertia_com)
        return fail_to(err, GRID_EINVAL, "a required model array is NULL");
    const int n = d->n;
    for (int i = 0; i < n; ++i) {
        if (d->parent[i] < -1 || d->parent[i] >= i)
            return fail_to(err, GRID_EINVAL, "parent[" + std::to_string(i) + "] = " +
                                                 std::to_string(d->parent[i]) +
                                                 " must satisfy -1 <= parent[i] < i");
        if (d->joint_type && d->joint_type[i] != GRID_JOINT_REVOLUTE &&
            d->joint_type[i] != GRID_JOINT_PRISMATIC && d->joint_type[i] != GRID_JOINT_FIXED)
            return fail_to(err, GRID_EINVAL, "joint_type[" + std::to_string(i) +
                                                 "] is not a joint type");
        if (d->axis) {
            const double* a = d->axis + 3 * i;
            const double nrm = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
            if (!(std::fabs(nrm - 1.0) <= 1e-6))
                return fail_to(err, GRID_EINVAL, "axis[" + std::to_string(i) +
                                                     "] must be a unit vector");
        }
    }
    if (!finite_all(d->tree_rot, 9 * n) || !finite_all(d->tree_pos, 3 * n) ||
        !finite_all(d->mass, n) || !finite_all(d->com, 3 * n) ||
        !finite_all(d->inertia_com, 6 * n) || !finite_all(d->gravity, 3))
        return fail_to(err, GRID_EINVAL, "model description holds a non-finite value");
    for (int i = 0; i < n; ++i) {
        if (!(d->mass[i] > 0))
            return fail_to(err, GRID_EINVAL, "mass[" + std::to_string(i) + "] must be > 0");
        const double* R = d->tree_rot + 9 * i;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double s = 0;
                for (int k = 0; k < 3; ++k)
                    s += R[a * 3 + k] * R[b * 3 + k];
                if (std::fabs(s - (a == b ? 1.0 : 0.0)) > 1e-5)
                    return fail_to(err, GRID_EINVAL, "tree_rot[" + std::to_string(i) + "] is not a rotation");
            }
        // inertia about the centre of mass must be positive definite (Sylvester)
        const double* J = d->inertia_com + 6 * i;
        const double xx = J[0], yy = J[1], zz = J[2], xy = J[3], xz = J[4], yz = J[5];
        const double m2 = xx * yy - xy * xy;
        const double m3 = xx * (yy * zz - yz * yz) - xy * (xy * zz - yz * xz) + xz * (xy * yz - yy * xz);
        if (!(xx > 0 && m2 > 0 && m3 > 0))
            return fail_to(err, GRID_EINVAL, "inertia_com[" + std::to_string(i) + "] is not positive definite");
    }
    return GRID_OK;
}

// device constants, branch by branch in local order, kConstStride floats per body:
// E_T, r, Ibar = Ic + m (|c|^2 1 - c c^T) about the body origin, h = m c, m
// A rotation R with R a = e_z for a unit vector a (rotation about a x e_z; a half turn
// about x when a = -e_z). Row-major.
static void align_to_z(const double* a, double* R)
{
    const double c = a[2];                                   // a . e_z
    const double v[3] = {a[1], -a[0], 0.0};                   // a x e_z
    const double s2 = v[0] * v[0] + v[1] * v[1];
    for (int k = 0; k < 9; ++k)
        R[k] = (k % 4 == 0) ? 1.0 : 0.0;
    if (s2 < 1e-24) {
        if (c < 0.0) {   // a = -e_z
            R[4] = -1.0;
            R[8] = -1.0;
        }
        return;
    }
    // R = 1 + [v]x + [v]x^2 / (1 + c)
    const double K[9] = {0.0, -v[2], v[1], v[2], 0.0, -v[0], -v[1], v[0], 0.0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k)
                acc += K[3 * i + k] * K[3 * k + j];
            K2[3 * i + j] = acc;
        }
    for (int k = 0; k < 9; ++k)
        R[k] += K[k] + K2[k] / (1.0 + c);
}

static void mat3(const double* A, const double* B, double* C, bool transB = false)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k)
                acc += A[3 * i + k] * (transB ? B[3 * j + k] : B[3 * k + j]);
            C[3 * i + j] = acc;
        }
}

// Body constants for the kernels, branch by branch: E_T, r, Ibar (about the body origin),
// h = m c, m. A joint axis a_i other than +z is turned into +z by re-expressing body i in
// the frame R_i (R_i a_i = e_z): E_T' = R_i E_T R_lambda^T, r' = R_lambda r, c' = R_i c,
// Ic' = R_i Ic R_i^T. Coordinates of body frames change; joint-space quantities do not.
std::vector<float> pack_constants(const grid_model_desc* d, const Topology& t)
{
    const int n = d->n;
    std::vector<double> R((size_t)9 * n);
    for (int i = 0; i < n; ++i) {
        double a[3] = {0.0, 0.0, 1.0};
        if (d->axis) {
            const double* ai = d->axis + 3 * i;
            const double nrm = std::sqrt(ai[0] * ai[0] + ai[1] * ai[1] + ai[2] * ai[2]);
            for (int k = 0; k < 3; ++k)
                a[k] = ai[k] / nrm;
        }
        align_to_z(a, R.data() + 9 * i);
    }
    static const double kI3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    std::vector<float> out((size_t)n * kConstStride, 0.0f);
    for (const BranchInst& inst : t.insts)
        for (size_t k = 0; k < inst.body.size(); ++k) {
            const int i = inst.body[k];
            const int p = d->parent[i];
            const double* Ri = R.data() + 9 * i;
            const double* Rp = p < 0 ? kI3 : R.data() + 9 * p;
            float* b = out.data() + inst.coff + k * kConstStride;
            double tmp[9], ET[9];
            mat3(Ri, d->tree_rot + 9 * i, tmp);
            mat3(tmp, Rp, ET, true);
            for (int e = 0; e < 9; ++e)
                b[e] = (float)ET[e];
            const double* r = d->tree_pos + 3 * i;
            for (int e = 0; e < 3; ++e)
                b[9 + e] = (float)(Rp[3 * e] * r[0] + Rp[3 * e + 1] * r[1] + Rp[3 * e + 2] * r[2]);
            const double m = d->mass[i];
            const double* c0 = d->com + 3 * i;
            double c[3];
            for (int e = 0; e < 3; ++e)
                c[e] = Ri[3 * e] * c0[0] + Ri[3 * e + 1] * c0[1] + Ri[3 * e + 2] * c0[2];
            const double* J0 = d->inertia_com + 6 * i;
            const double Jm[9] = {J0[0], J0[3], J0[4], J0[3], J0[1], J0[5], J0[4], J0[5], J0[2]};
            double RJ[9], Jr[9];
            mat3(Ri, Jm, RJ);
            mat3(RJ, Ri, Jr, true);
            const double J[6] = {Jr[0], Jr[4], Jr[8], Jr[1], Jr[2], Jr[5]};
            b[12] = (float)(J[0] + m * (c[1] * c[1] + c[2] * c[2]));
            b[13] = (float)(J[1] + m * (c[0] * c[0] + c[2] * c[2]));
            b[14] = (float)(J[2] + m * (c[0] * c[0] + c[1] * c[1]));
            b[15] = (float)(J[3] - m * c[0] * c[1]);
            b[16] = (float)(J[4] - m * c[0] * c[2]);
            b[17] = (float)(J[5] - m * c[1] * c[2]);
            b[18] = (float)(m * c[0]);
            b[19] = (float)(m * c[1]);
            b[20] = (float)(m * c[2]);
            b[21] = (float)m;
        }
    return out;
}

}  // namespace grid_impl

namespace {

grid_status fail(grid_status s, const std::string& msg)
{
    set_error(msg);
    return s;
}

grid_status hip_fail(hipError_t e, const char* what)
{
    return fail(GRID_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                  \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess)                          \
            return hip_fail(e_, #expr);                \
    } while (0)


grid_status launch(hipFunction_t fn, unsigned blocks, unsigned threads, int32_t N, float* work,
                   const float* q, const float* qd, const float* tau, float* qdd, float* Minv,
                   float* dq, float* dqd, hipStream_t stream)
{
    KernelArgs a;
    a.nknots = N;
    a.work = work;
    a.q = q;
    a.qd = qd;
    a.tau = tau;
    a.qdd = qdd;
    a.Minv = Minv;
    a.dqdd_dq = dq;
    a.dqdd_dqd = dqd;
    void* params[] = {&a};   // the kernel takes one argument: the Args block
    HIP_TRY(hipModuleLaunchKernel(fn, blocks, 1, 1, threads, 1, 1, 0, stream, params, nullptr));
    return GRID_OK;
}

}  // namespace

namespace grid_impl {

int fused_variant_for(grid_model m, int32_t N)
{
    for (const auto& e : m->tuned)
        if (N <= e.first)
            return e.second;
    if (!m->tuned.empty())
        return m->tuned.back().second;
    // untuned: the three-role kernel while its wavefronts fit one per SIMD of the device (the
    // lowest-latency form), the lane layout beyond (fewer instructions per knot), and from 64
    // knots per compute unit the forms with one problem per lane or four lanes (no repeated
    // sweeps; build 5 once it has 128 knots per compute unit, half a wavefront per SIMD at
    // least). A branch of more than 8 bodies makes the lane layout's repeated sweeps expensive,
    // and the tuner keeps the three-role kernel far beyond one wavefront per SIMD there
    // (humanoid30: up to 4096 knots, then build 6)
    const int64_t waves = workgroups_pipe(m->topo, N) * pipe_waves(m->topo);
    if (waves <= 4 * (int64_t)m->compute_units)
        return kVariantPipe;
    int largest = 0;
    for (const BranchShape& sh : m->topo.shapes)
        largest = std::max(largest, sh.B);
    if (largest > 8)
        return N <= 4096 ? kVariantPipe : kVariantSerial4;
    if (N >= 128 * (int64_t)m->compute_units)
        return kVariantSerial;
    if (N >= 64 * (int64_t)m->compute_units)
        return kVariantSerial4;
    return kVariantLane1;
}

grid_status launch_fused_variant(grid_model m, int variant, int32_t N, const float* q,
                                 const float* qd, const float* tau, float* qdd, float* Minv,
                                 float* dq, float* dqd, hipStream_t stream)
{
    if (variant < 0 || variant >= kNumVariants || !m->fused_variant[variant])
        return fail(GRID_EUNSUPPORTED, "the requested build of the fused kernel does not exist for the model");
    if (variant == kVariantQuad)
        return launch(m->fused_variant[variant], (unsigned)workgroups_quad(m->topo, N),
                      64u * (unsigned)m->topo.waves, N, nullptr, q, qd, tau, qdd, Minv, dq, dqd,
                      stream);
    if (variant == kVariantPipe)
        return launch(m->fused_variant[variant], (unsigned)workgroups_pipe(m->topo, N),
                      64u * (unsigned)pipe_waves(m->topo), N, nullptr, q, qd, tau, qdd, Minv, dq,
                      dqd, stream);
    if (variant == kVariantSerial || variant == kVariantSerial4 || variant == kVariantSerial2)
        return launch(m->fused_variant[variant],
                      (unsigned)workgroups_serial(m->topo, N, variant == kVariantSerial ? 64
                                                          : variant == kVariantSerial2 ? 32 : 16),
                      64u, N, nullptr, q, qd, tau, qdd, Minv, dq, dqd, stream);
    return launch(m->fused_variant[variant], (unsigned)workgroups_for(m->topo, N), 64u, N,
                  nullptr, q, qd, tau, qdd, Minv, dq, dqd, stream);
}

grid_status launch_fused(grid_model m, int32_t N, const float* q, const float* qd,
                         const float* tau, float* qdd, float* Minv, float* dq, float* dqd,
                         hipStream_t stream)
{
    return launch_fused_variant(m, fused_variant_for(m, N), N, q, qd, tau, qdd, Minv, dq, dqd,
                                stream);
}

}  // namespace grid_impl

extern "C" {

const char* grid_status_string(grid_status s)
{
    switch (s) {
    case GRID_OK: return "GRID_OK";
    case GRID_EINVAL: return "GRID_EINVAL";
    case GRID_ENOMEM: return "GRID_ENOMEM";
    case GRID_EDEVICE: return "GRID_EDEVICE";
    case GRID_EUNSUPPORTED: return "GRID_EUNSUPPORTED";
    case GRID_ECOMPILE: return "GRID_ECOMPILE";
    case GRID_EBUSY: return "GRID_EBUSY";
    case GRID_ETIMEDOUT: return "GRID_ETIMEDOUT";
    case GRID_ECANCELED: return "GRID_ECANCELED";
    default: return "GRID_UNKNOWN";
    }
}

const char* grid_last_error(void) { return t_last_error.c_str(); }

// validated description -> topology, packed constants and generated source
// The model without its fixed joints: every body on a fixed joint merges into its nearest
// ancestor on a movable (revolute or prismatic) joint (its owner; -1 when the chain of fixed
// joints reaches the base). Transforms are (E, r) with x_child = E (x_parent - r); the owner-to-body transform
// of a fixed body composes (E2, r2) after (E1, r1) as (E2 E1, r1 + E1^T r2). Inertias are
// summed about the owner's origin: mass, first moment and the rotational inertia there.
struct ReducedDesc {
    std::vector<int32_t> parent, joint_type;
    std::vector<double> axis, rot, pos, mass, com, inertia;
    grid_model_desc d{};
};

static void reduce_fixed(const grid_model_desc* src, ReducedDesc* out)
{
    const int n = src->n;
    std::vector<int> owner(n, -1), newidx(n, -1);
    std::vector<double> Eo((size_t)9 * n), ro((size_t)3 * n);   // owner frame -> body frame
    std::vector<double> M, H, IO;                                 // per movable body: m, m c, I_O
    int nd = 0;
    for (int i = 0; i < n; ++i) {
        const int p = src->parent[i];
        const double* ET = src->tree_rot + 9 * i;
        const double* rT = src->tree_pos + 3 * i;
        // owner frame -> this joint's frame (the parent's chain composed with X_T)
        double E[9], r[3];
        const int po = p < 0 ? -1 : owner[p];
        if (p < 0) {
            std::memcpy(E, ET, sizeof E);
            std::memcpy(r, rT, sizeof r);
        } else {
            const double* E1 = Eo.data() + 9 * p;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double acc = 0.0;
                    for (int k = 0; k < 3; ++k)
                        acc += ET[3 * a + k] * E1[3 * k + b];
                    E[3 * a + b] = acc;
                }
            for (int a = 0; a < 3; ++a)
                r[a] = ro[3 * p + a] + E1[a] * rT[0] + E1[3 + a] * rT[1] + E1[6 + a] * rT[2];
        }
        const bool fixed = src->joint_type && src->joint_type[i] == GRID_JOINT_FIXED;
        const double m = src->mass[i];
        const double* c = src->com + 3 * i;
        const double* J = src->inertia_com + 6 * i;
        const double Jm[9] = {J[0], J[3], J[4], J[3], J[1], J[5], J[4], J[5], J[2]};
        if (!fixed) {
            owner[i] = i;
            newidx[i] = nd++;
            out->parent.push_back(po < 0 ? -1 : newidx[po]);
            out->joint_type.push_back(src->joint_type ? src->joint_type[i] : GRID_JOINT_REVOLUTE);
            out->rot.insert(out->rot.end(), E, E + 9);
            out->pos.insert(out->pos.end(), r, r + 3);
            for (int k = 0; k < 3; ++k)
                out->axis.push_back(src->axis ? src->axis[3 * i + k] : (k == 2 ? 1.0 : 0.0));
            for (int k = 0; k < 9; ++k)
                Eo[9 * i + k] = (k % 4 == 0) ? 1.0 : 0.0;
            for (int k = 0; k < 3; ++k)
                ro[3 * i + k] = 0.0;
            // the body's own inertia about its origin
            M.push_back(m);
            for (int k = 0; k < 3; ++k)
                H.push_back(m * c[k]);
            const double cc = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    IO.push_back(Jm[3 * a + b] + m * ((a == b ? cc : 0.0) - c[a] * c[b]));
        } else {
            owner[i] = po;
            std::memcpy(Eo.data() + 9 * i, E, sizeof E);
            std::memcpy(ro.data() + 3 * i, r, sizeof r);
            if (po >= 0) {
                // this body in the owner's frame: centre r + E^T c, inertia E^T J E there
                const int o = newidx[po];
                double co[3], Jo[9];
                for (int a = 0; a < 3; ++a)
                    co[a] = r[a] + E[a] * c[0] + E[3 + a] * c[1] + E[6 + a] * c[2];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        double acc = 0.0;
                        for (int k = 0; k < 3; ++k)
                            for (int l = 0; l < 3; ++l)
                                acc += E[3 * k + a] * Jm[3 * k + l] * E[3 * l + b];
                        Jo[3 * a + b] = acc;
                    }
                const double cc = co[0] * co[0] + co[1] * co[1] + co[2] * co[2];
                M[o] += m;
                for (int k = 0; k < 3; ++k)
                    H[3 * o + k] += m * co[k];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        IO[9 * o + 3 * a + b] += Jo[3 * a + b] + m * ((a == b ? cc : 0.0) - co[a] * co[b]);
            }
        }
    }
    for (int o = 0; o < nd; ++o) {
        const double m = M[o];
        double c[3];
        for (int k = 0; k < 3; ++k)
            c[k] = H[3 * o + k] / m;
        const double cc = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        double Jc[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                Jc[3 * a + b] = IO[9 * o + 3 * a + b] - m * ((a == b ? cc : 0.0) - c[a] * c[b]);
        out->mass.push_back(m);
        out->com.insert(out->com.end(), c, c + 3);
        const double J6[6] = {Jc[0], Jc[4], Jc[8], Jc[1], Jc[2], Jc[5]};
        out->inertia.insert(out->inertia.end(), J6, J6 + 6);
    }
    grid_model_desc& d = out->d;
    d.n = nd;
    d.parent = out->parent.data();
    d.joint_type = out->joint_type.data();
    d.axis = src->axis ? out->axis.data() : nullptr;
    d.tree_rot = out->rot.data();
    d.tree_pos = out->pos.data();
    d.mass = out->mass.data();
    d.com = out->com.data();
    d.inertia_com = out->inertia.data();
    std::memcpy(d.gravity, src->gravity, sizeof d.gravity);
}

}  // extern "C"

namespace grid_impl {

// validated description -> topology of the model without its fixed joints, and its packed
// constants; the status and *err on failure
grid_status prepare_robot(const grid_model_desc* desc, Topology* topo,
                          std::vector<float>* consts, std::string* err)
{
    grid_status s = validate_desc(desc, err);
    if (s != GRID_OK)
        return s;
    ReducedDesc red;
    reduce_fixed(desc, &red);
    if (red.d.n < 1) {
        *err = "the model has no movable joint";
        return GRID_EINVAL;
    }
    if (!analyse_topology(red.d.parent, red.d.n, topo, err))
        return GRID_EINVAL;
    for (BranchInst& inst : topo->insts)
        for (size_t k = 0; k < inst.body.size(); ++k)
            if (red.d.joint_type[inst.body[k]] == GRID_JOINT_PRISMATIC)
                inst.prism |= 1ull << k;
    *consts = pack_constants(&red.d, *topo);
    return GRID_OK;
}

}  // namespace grid_impl

extern "C" {

// the model's two module sources: every kernel, and the pipe kernel alone (compiled with the
// ILP schedule); `allowed` are the flag bits the caller accepts
static grid_status prepare(const grid_model_desc* desc, uint32_t flags, uint32_t allowed,
                           Topology* topo, std::string* src, std::string* pipe_src)
{
    std::string err;
    std::vector<float> consts;
    grid_status s = prepare_robot(desc, topo, &consts, &err);
    if (s != GRID_OK)
        return fail(s, err);
    if (flags & ~allowed)
        return fail(GRID_EINVAL, "unknown flag bits");
    *src = generate_source(*topo, consts, desc->gravity, 0);
    *pipe_src = generate_pipe_source(*topo, consts, desc->gravity);
    return GRID_OK;
}

grid_status grid_codegen_source(const grid_model_desc* desc, uint32_t flags, char* buf,
                                size_t* len)
{
    if (!len)
        return fail(GRID_EINVAL, "len must not be NULL");
    Topology t;
    std::string main_src, pipe_src;
    grid_status s = prepare(desc, flags, GRID_CODEGEN_PIPE_MODULE, &t, &main_src, &pipe_src);
    if (s != GRID_OK)
        return s;
    const std::string& src = (flags & GRID_CODEGEN_PIPE_MODULE) ? pipe_src : main_src;
    const size_t need = src.size() + 1;
    const bool fits = buf && *len >= need;
    if (fits)
        std::memcpy(buf, src.c_str(), need);
    *len = need;
    if (buf && !fits)
        return fail(GRID_EINVAL, "buffer too small");
    return GRID_OK;
}

grid_status grid_codegen_precompile(const grid_model_desc* desc, uint32_t flags)
{
    Topology t;
    std::string src, pipe_src, err;
    grid_status s = prepare(desc, flags, 0, &t, &src, &pipe_src);
    if (s != GRID_OK)
        return s;
    std::vector<char> code;
    s = compile_cached(src, &code, &err);
    if (s == GRID_OK)
        s = compile_cached(pipe_src, &code, &err, true);
    if (s != GRID_OK)
        return fail(s, err);
    return GRID_OK;
}

grid_status grid_model_create(const grid_model_desc* desc, int32_t device, uint32_t flags,
                              grid_model* out)
{
    if (!out)
        return fail(GRID_EINVAL, "out must not be NULL");
    *out = nullptr;
    Topology topo;
    std::string src, pipe_src, err;
    grid_status s = prepare(desc, flags, 0, &topo, &src, &pipe_src);
    if (s != GRID_OK)
        return s;
    std::vector<char> code, pipe_code;
    s = compile_cached(src, &code, &err);
    if (s == GRID_OK)
        s = compile_cached(pipe_src, &pipe_code, &err, true);
    if (s != GRID_OK)
        return fail(s, err);

    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count)
        return fail(GRID_EINVAL, "device index out of range");
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(GRID_EUNSUPPORTED, std::string("device is ") + prop.gcnArchName +
                                           ", kernels are built for gfx950");

    s = noalloc_setup(device, &err);   // once per device: the scratch array's address
    if (s != GRID_OK)
        return fail(s, err);

    grid_model m = new (std::nothrow) grid_model_s;
    if (!m)
        return fail(GRID_ENOMEM, "host allocation failed");
    m->device = device;
    m->flags = flags;
    m->topo = std::move(topo);
    m->code_hash = source_hash(machine_code(code) + machine_code(pipe_code));
    static const char* const kStages[5] = {"grid_stage_rnea", "grid_stage_minv", "grid_stage_qdd",
                                           "grid_stage_drnea", "grid_stage_fdgrad"};
    static const char* const kVariants[kNumVariants] = {
        "grid_fdgrad_quad", "grid_fdgrad_fused", "grid_fdgrad_fused_w2", "grid_fdgrad_fused_w4",
        "grid_fdgrad_pipe", "grid_fdgrad_serial", "grid_fdgrad_serial4", "grid_fdgrad_serial2"};
    m->compute_units = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    hipError_t e = hipModuleLoadData(&m->module, code.data());
    for (int k = 0; k < kNumVariants && e == hipSuccess; ++k)
        if (k != kVariantPipe)   // build 4 lives in the pipe module alone
            e = hipModuleGetFunction(&m->fused_variant[k], m->module, kVariants[k]);
    static const char* const kOps[kNumOps] = {"grid_op_id", "grid_op_fd", "grid_op_minv",
                                              "grid_op_idgrad", "grid_op_vjp"};
    for (int k = 0; k < kNumOps && e == hipSuccess; ++k)
        e = hipModuleGetFunction(&m->op[k], m->module, kOps[k]);
    for (int k = 0; k < 5 && e == hipSuccess; ++k)
        e = hipModuleGetFunction(&m->stage[k], m->module, kStages[k]);
    static const char* const kMinvRoutes[2] = {"grid_minv_serial", "grid_minv_direct"};
    for (int k = 0; k < 2 && e == hipSuccess; ++k)
        e = hipModuleGetFunction(&m->minv_route[k], m->module, kMinvRoutes[k]);
    if (e == hipSuccess)
        e = hipModuleLoadData(&m->pipe_module, pipe_code.data());
    if (e == hipSuccess)   // build 4 from its own module
        e = hipModuleGetFunction(&m->fused_variant[kVariantPipe], m->pipe_module,
                                 "grid_fdgrad_pipe");
    if (e != hipSuccess) {
        grid_model_destroy(m);
        return hip_fail(e, "module load");
    }
    load_tuning(m);
    *out = m;
    return GRID_OK;
}

grid_status grid_model_destroy(grid_model m)
{
    if (!m)
        return GRID_OK;
    (void)hipSetDevice(m->device);
    if (m->module)
        (void)hipModuleUnload(m->module);
    if (m->pipe_module)
        (void)hipModuleUnload(m->pipe_module);
    delete m;
    return GRID_OK;
}

grid_status grid_model_info(grid_model m, int32_t* n, size_t* io_bytes_per_knot,
                            int32_t* lanes)
{
    if (!m)
        return fail(GRID_EINVAL, "model is NULL");
    const size_t nn = (size_t)m->topo.n;
    if (n)
        *n = m->topo.n;
    if (io_bytes_per_knot)
        *io_bytes_per_knot = sizeof(float) * (3 * nn + nn + 3 * nn * nn);
    if (lanes)
        *lanes = lanes_per_knot(m->topo);
    return GRID_OK;
}

grid_status grid_model_code_hash(grid_model m, uint64_t* hash)
{
    if (!m || !hash)
        return fail(GRID_EINVAL, "model and hash must not be NULL");
    *hash = m->code_hash;
    return GRID_OK;
}

grid_status grid_fd_grad(grid_model m, int32_t N, const float* q, const float* qd,
                         const float* tau, float* qdd, float* Minv, float* dqdd_dq,
                         float* dqdd_dqd, void* stream)
{
    if (!m)
        return fail(GRID_EINVAL, "model is NULL");
    if (N < 0)
        return fail(GRID_EINVAL, "N must be >= 0");
    if (N == 0)
        return GRID_OK;
    if (N > GRID_MAX_KNOTS)
        return fail(GRID_EINVAL, "N too large");
    if (!q || !qd || !tau || !qdd || !Minv || !dqdd_dq || !dqdd_dqd)
        return fail(GRID_EINVAL, "a data pointer is NULL");
    HIP_TRY(hipSetDevice(m->device));
    return launch_fused(m, N, q, qd, tau, qdd, Minv, dqdd_dq, dqdd_dqd, (hipStream_t)stream);
}

static grid_status launch_op(grid_model m, int op, int32_t N, const float* q, const float* qd,
                             const float* u, float* out0, float* out1, void* stream,
                             const float* u2 = nullptr, float* out2 = nullptr)
{
    if (!m)
        return fail(GRID_EINVAL, "model is NULL");
    if (N < 0)
        return fail(GRID_EINVAL, "N must be >= 0");
    if (N == 0)
        return GRID_OK;
    if (N > GRID_MAX_KNOTS)
        return fail(GRID_EINVAL, "N too large");
    const bool needs_qd = op != kOpMinv, needs_u = op != kOpMinv;
    const bool needs_out1 = op == kOpIdGrad || op == kOpVjp, vjp = op == kOpVjp;
    if (!q || (needs_qd && !qd) || (needs_u && !u) || !out0 || (needs_out1 && !out1) ||
        (vjp && (!u2 || !out2)))
        return fail(GRID_EINVAL, "a data pointer is NULL");
    HIP_TRY(hipSetDevice(m->device));
    OpArgs a;
    a.nknots = N;
    a.q = q;
    a.qd = needs_qd ? qd : nullptr;
    a.u = needs_u ? u : nullptr;
    a.u2 = vjp ? u2 : nullptr;
    a.out0 = out0;
    a.out1 = needs_out1 ? out1 : nullptr;
    a.out2 = vjp ? out2 : nullptr;
    const unsigned blocks = (unsigned)workgroups_op(m->topo, N, op);
    const unsigned threads = op == kOpIdGrad ? 64u * (unsigned)m->topo.waves : 64u;
    void* params[] = {&a};
    HIP_TRY(hipModuleLaunchKernel(m->op[op], blocks, 1, 1, threads, 1, 1, 0, (hipStream_t)stream,
                                  params, nullptr));
    return GRID_OK;
}

grid_status grid_id(grid_model m, int32_t N, const float* q, const float* qd, const float* qdd,
                    float* tau, void* stream)
{
    return launch_op(m, kOpId, N, q, qd, qdd, tau, nullptr, stream);
}

grid_status grid_fd(grid_model m, int32_t N, const float* q, const float* qd, const float* tau,
                    float* qdd, void* stream)
{
    return launch_op(m, kOpFd, N, q, qd, tau, qdd, nullptr, stream);
}

grid_status grid_minv(grid_model m, int32_t N, const float* q, float* Minv, void* stream)
{
    return launch_op(m, kOpMinv, N, q, nullptr, nullptr, Minv, nullptr, stream);
}

grid_status grid_minv_route(grid_model m, int32_t N, const float* q, float* Minv, int32_t route,
                            void* stream)
{
    if (route == GRID_MINV_QUAD)
        return grid_minv(m, N, q, Minv, stream);
    if (route != GRID_MINV_LANE_LTL && route != GRID_MINV_LANE_DIRECT)
        return fail(GRID_EINVAL, "unknown M^-1 route");
    if (!m)
        return fail(GRID_EINVAL, "model is NULL");
    if (N < 0)
        return fail(GRID_EINVAL, "N must be >= 0");
    if (N == 0)
        return GRID_OK;
    if (N > GRID_MAX_KNOTS)
        return fail(GRID_EINVAL, "N too large");
    if (!q || !Minv)
        return fail(GRID_EINVAL, "a data pointer is NULL");
    HIP_TRY(hipSetDevice(m->device));
    return launch(m->minv_route[route == GRID_MINV_LANE_DIRECT ? 1 : 0],
                  (unsigned)workgroups_serial(m->topo, N, 64), 64u, N, nullptr, q, nullptr,
                  nullptr, nullptr, Minv, nullptr, nullptr, (hipStream_t)stream);
}

grid_status grid_id_grad(grid_model m, int32_t N, const float* q, const float* qd,
                         const float* qdd, float* dtau_dq, float* dtau_dqd, void* stream)
{
    return launch_op(m, kOpIdGrad, N, q, qd, qdd, dtau_dq, dtau_dqd, stream);
}

grid_status grid_fd_vjp_adjoint(grid_model m, int32_t N, const float* q, const float* qd,
                                const float* qdd, const float* gbar, float* qbar, float* qdbar,
                                float* taubar, void* stream)
{
    return launch_op(m, kOpVjp, N, q, qd, qdd, qbar, qdbar, stream, gbar, taubar);
}

// the five stage kernels of the plain pipeline, intermediates in `work` (N x the model's
// workspace stride floats; every stage writes what a later one reads, so it needs no clearing)
static grid_status launch_staged(grid_model m, float* work, int32_t N, const float* q,
                                 const float* qd, const float* tau, float* qdd, float* Minv,
                                 float* dqdd_dq, float* dqdd_dqd, hipStream_t stream)
{
    for (int k = 0; k < 5; ++k) {
        grid_status s = launch(m->stage[k], (unsigned)workgroups_for(m->topo, N), 64u, N, work,
                               q, qd, tau, qdd, Minv, dqdd_dq, dqdd_dqd, stream);
        if (s != GRID_OK)
            return s;
    }
    return GRID_OK;
}

grid_status grid_fd_grad_staged(grid_model m, grid_workspace w, int32_t N, const float* q,
                                const float* qd, const float* tau, float* qdd, float* Minv,
                                float* dqdd_dq, float* dqdd_dqd, void* stream)
{
    if (!m || !w)
        return fail(GRID_EINVAL, "model and workspace must not be NULL");
    if (w->model != m)
        return fail(GRID_EINVAL, "workspace was created for another model");
    if (N < 0 || N > w->max_knots)
        return fail(GRID_EINVAL, "N must be in 0..max_knots of the workspace");
    if (N == 0)
        return GRID_OK;
    if (!q || !qd || !tau || !qdd || !Minv || !dqdd_dq || !dqdd_dqd)
        return fail(GRID_EINVAL, "a data pointer is NULL");
    HIP_TRY(hipSetDevice(m->device));
    return launch_staged(m, w->d_stage, N, q, qd, tau, qdd, Minv, dqdd_dq, dqdd_dqd,
                         (hipStream_t)stream);
}

grid_status grid_fd_grad_staged_noalloc(grid_model m, int32_t N, const float* q,
                                        const float* qd, const float* tau, float* qdd,
                                        float* Minv, float* dqdd_dq, float* dqdd_dqd,
                                        void* stream)
{
    if (!m)
        return fail(GRID_EINVAL, "model is NULL");
    if (N < 0)
        return fail(GRID_EINVAL, "N must be >= 0");
    const size_t per_knot = (size_t)workspace_layout(m->topo).stride * sizeof(float);
    if ((size_t)N * per_knot > (size_t)GRID_NOALLOC_SCRATCH_BYTES)
        return fail(GRID_EINVAL, "N = " + std::to_string(N) + " needs " +
                                     std::to_string((size_t)N * per_knot) +
                                     " bytes of scratch; the static array holds " +
                                     std::to_string((size_t)GRID_NOALLOC_SCRATCH_BYTES) +
                                     " (at most " +
                                     std::to_string(GRID_NOALLOC_SCRATCH_BYTES / per_knot) +
                                     " knots of this model)");
    if (N == 0)
        return GRID_OK;
    if (!q || !qd || !tau || !qdd || !Minv || !dqdd_dq || !dqdd_dqd)
        return fail(GRID_EINVAL, "a data pointer is NULL");
    float* work = noalloc_scratch(m->device);
    if (!work)
        return fail(GRID_EDEVICE, "the scratch array of this device has no address");
    HIP_TRY(hipSetDevice(m->device));
    return launch_staged(m, work, N, q, qd, tau, qdd, Minv, dqdd_dq, dqdd_dqd,
                         (hipStream_t)stream);
}

grid_status grid_fd_vjp(grid_model m, int32_t N, const float* dqdd_dq, const float* dqdd_dqd,
                        const float* Minv, const float* gbar, float* qbar, float* qdbar,
                        float* taubar, void* stream)
{
    if (!m)
        return fail(GRID_EINVAL, "model is NULL");
    if (N < 0 || N > GRID_MAX_KNOTS)
        return fail(GRID_EINVAL, "N out of range");
    if (N == 0)
        return GRID_OK;
    if (!dqdd_dq || !dqdd_dqd || !Minv || !gbar || !qbar || !qdbar || !taubar)
        return fail(GRID_EINVAL, "a data pointer is NULL");
    HIP_TRY(hipSetDevice(m->device));
    HIP_TRY(launch_vjp(N, m->topo.n, dqdd_dq, dqdd_dqd, Minv, gbar, qbar, qdbar, taubar,
                       (hipStream_t)stream));
    return GRID_OK;
}

grid_status grid_dt_jacobians(grid_model m, int32_t N, float dt, const float* dqdd_dq,
                              const float* dqdd_dqd, const float* Minv, float* A, float* B,
                              void* stream)
{
    if (!m)
        return fail(GRID_EINVAL, "model is NULL");
    if (N < 0 || N > GRID_MAX_KNOTS)
        return fail(GRID_EINVAL, "N out of range");
    if (!(dt > 0.0f) || !std::isfinite(dt))
        return fail(GRID_EINVAL, "dt must be positive and finite");
    if (N == 0)
        return GRID_OK;
    if ((long)N * 6L * m->topo.n * m->topo.n > (1L << 31) - 256)
        return fail(GRID_EINVAL, "N too large for one launch");
    if (!dqdd_dq || !dqdd_dqd || !Minv || !A || !B)
        return fail(GRID_EINVAL, "a data pointer is NULL");
    HIP_TRY(hipSetDevice(m->device));
    HIP_TRY(launch_dt(N, m->topo.n, dt, dqdd_dq, dqdd_dqd, Minv, A, B, (hipStream_t)stream));
    return GRID_OK;
}

grid_status grid_workspace_create(grid_model m, int32_t max_knots, grid_workspace* out)
{
    if (!m || !out)
        return fail(GRID_EINVAL, "model and out must not be NULL");
    *out = nullptr;
    if (max_knots < 1 || max_knots > GRID_MAX_KNOTS)
        return fail(GRID_EINVAL, "max_knots out of range");
    HIP_TRY(hipSetDevice(m->device));
    grid_workspace w = new (std::nothrow) grid_workspace_s;
    if (!w)
        return fail(GRID_ENOMEM, "host allocation failed");
    w->model = m;
    w->max_knots = max_knots;
    const size_t n = (size_t)m->topo.n;
    const size_t in_f = (size_t)max_knots * 3 * n;
    const size_t out_f = (size_t)max_knots * (n + 3 * n * n);
    hipError_t e = hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&w->stream2, hipStreamNonBlocking);
    for (int k = 0; k < 4 && e == hipSuccess; ++k)
        e = hipEventCreate(&w->ev[k]);
    if (e == hipSuccess)
        e = hipMalloc(&w->d_in, in_f * sizeof(float));
    if (e == hipSuccess)
        e = hipMalloc(&w->d_out, out_f * sizeof(float));
    if (e == hipSuccess)
        e = hipMalloc(&w->d_stage, (size_t)max_knots * workspace_layout(m->topo).stride *
                                       sizeof(float));
    if (e == hipSuccess)
        e = hipHostMalloc(&w->h_in, in_f * sizeof(float), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(&w->h_out, out_f * sizeof(float), hipHostMallocDefault);
    if (e != hipSuccess) {
        grid_workspace_destroy(w);
        return fail(GRID_ENOMEM, std::string("workspace allocation: ") + hipGetErrorString(e));
    }
    // the device's view of the pinned buffers, for the mapped call (optional)
    void* pin_in = nullptr;
    void* pin_out = nullptr;
    if (hipHostGetDevicePointer(&pin_in, w->h_in, 0) == hipSuccess &&
        hipHostGetDevicePointer(&pin_out, w->h_out, 0) == hipSuccess) {
        w->h_in_dev = static_cast<float*>(pin_in);
        w->h_out_dev = static_cast<float*>(pin_out);
    } else {
        (void)hipGetLastError();
    }
    *out = w;
    return GRID_OK;
}

grid_status grid_workspace_destroy(grid_workspace w)
{
    if (!w)
        return GRID_OK;
    (void)hipSetDevice(w->model->device);
    if (w->stream)
        (void)hipStreamSynchronize(w->stream);
    if (w->stream2)
        (void)hipStreamSynchronize(w->stream2);
    for (auto& ev : w->ev)
        if (ev)
            (void)hipEventDestroy(ev);
    if (w->stream)
        (void)hipStreamDestroy(w->stream);
    if (w->stream2)
        (void)hipStreamDestroy(w->stream2);
    (void)hipFree(w->d_in);
    (void)hipFree(w->d_out);
    (void)hipFree(w->d_stage);
    if (w->h_in)
        (void)hipHostFree(w->h_in);
    if (w->h_out)
        (void)hipHostFree(w->h_out);
    delete w;
    return GRID_OK;
}

// Knots [k0, k1) of a batch of N whose arrays sit packed in the workspace's pinned and device
// buffers (q | qd | tau, qdd | Minv | dqdd_dq | dqdd_dqd, each for N knots): their rows' H2D
// copies, one fused launch and the D2H copies of their outputs, on `s`.
static grid_status issue_piece(grid_model m, grid_workspace w, int32_t N, int32_t k0, int32_t k1,
                               hipStream_t s)
{
    const size_t n = (size_t)m->topo.n;
    const size_t vec = (size_t)N * n, mat = vec * n;
    const size_t ov = (size_t)k0 * n, om = ov * n;
    const size_t rv = (size_t)(k1 - k0) * n, rm = rv * n;
    for (int a = 0; a < 3; ++a)
        HIP_TRY(hipMemcpyAsync(w->d_in + a * vec + ov, w->h_in + a * vec + ov, rv * sizeof(float),
                               hipMemcpyHostToDevice, s));
    float* d_q = w->d_in;
    float* d_qdd = w->d_out;
    grid_status st = launch_fused(m, k1 - k0, d_q + ov, d_q + vec + ov, d_q + 2 * vec + ov,
                                  d_qdd + ov, d_qdd + vec + om, d_qdd + vec + mat + om,
                                  d_qdd + vec + 2 * mat + om, s);
    if (st != GRID_OK)
        return st;
    HIP_TRY(hipMemcpyAsync(w->h_out + ov, d_qdd + ov, rv * sizeof(float), hipMemcpyDeviceToHost,
                           s));
    for (int a = 0; a < 3; ++a)
        HIP_TRY(hipMemcpyAsync(w->h_out + vec + a * mat + om, d_qdd + vec + a * mat + om,
                               rm * sizeof(float), hipMemcpyDeviceToHost, s));
    return GRID_OK;
}

// H2D of the pinned inputs, the fused kernel and D2H into the pinned outputs for N knots, then
// a wait. One piece: one copy each way (the packed arrays are contiguous) on the workspace's
// stream, the three phases timed by events. Several pieces: issued on the two streams in turn,
// so that the copies of one overlap the kernel of another; only the total is timed.
static grid_status run_pinned(grid_model m, grid_workspace w, int32_t N, int32_t pieces,
                              grid_timing* timing)
{
    const size_t n = (size_t)m->topo.n;
    const size_t vec = (size_t)N * n, mat = vec * n;
    if (pieces <= 1) {
        float* d_q = w->d_in;
        float* d_qdd = w->d_out;
        HIP_TRY(hipEventRecord(w->ev[0], w->stream));
        HIP_TRY(hipMemcpyAsync(d_q, w->h_in, 3 * vec * sizeof(float), hipMemcpyHostToDevice,
                               w->stream));
        HIP_TRY(hipEventRecord(w->ev[1], w->stream));
        grid_status s = launch_fused(m, N, d_q, d_q + vec, d_q + 2 * vec, d_qdd, d_qdd + vec,
                                     d_qdd + vec + mat, d_qdd + vec + 2 * mat, w->stream);
        if (s != GRID_OK)
            return s;
        HIP_TRY(hipEventRecord(w->ev[2], w->stream));
        HIP_TRY(hipMemcpyAsync(w->h_out, d_qdd, (vec + 3 * mat) * sizeof(float),
                               hipMemcpyDeviceToHost, w->stream));
        HIP_TRY(hipEventRecord(w->ev[3], w->stream));
        HIP_TRY(hipStreamSynchronize(w->stream));
        if (timing) {
            HIP_TRY(hipEventElapsedTime(&timing->h2d_ms, w->ev[0], w->ev[1]));
            HIP_TRY(hipEventElapsedTime(&timing->kernel_ms, w->ev[1], w->ev[2]));
            HIP_TRY(hipEventElapsedTime(&timing->d2h_ms, w->ev[2], w->ev[3]));
            HIP_TRY(hipEventElapsedTime(&timing->total_ms, w->ev[0], w->ev[3]));
        }
        return GRID_OK;
    }
    HIP_TRY(hipEventRecord(w->ev[0], w->stream));
    HIP_TRY(hipStreamWaitEvent(w->stream2, w->ev[0], 0));
    for (int32_t c = 0; c < pieces; ++c) {
        const int32_t k0 = (int32_t)((int64_t)N * c / pieces);
        const int32_t k1 = (int32_t)((int64_t)N * (c + 1) / pieces);
        grid_status s = issue_piece(m, w, N, k0, k1, (c & 1) ? w->stream2 : w->stream);
        if (s != GRID_OK) {
            (void)hipStreamSynchronize(w->stream2);
            (void)hipStreamSynchronize(w->stream);
            return s;
        }
    }
    HIP_TRY(hipEventRecord(w->ev[1], w->stream2));
    HIP_TRY(hipStreamWaitEvent(w->stream, w->ev[1], 0));
    HIP_TRY(hipEventRecord(w->ev[3], w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    if (timing)
        HIP_TRY(hipEventElapsedTime(&timing->total_ms, w->ev[0], w->ev[3]));
    return GRID_OK;
}

grid_status grid_workspace_host_buffers(grid_workspace w, float** in, float** out)
{
    if (!w || !in || !out)
        return fail(GRID_EINVAL, "workspace and both output pointers are required");
    *in = w->h_in;
    *out = w->h_out;
    return GRID_OK;
}

grid_status grid_fd_grad_pinned(grid_model m, grid_workspace w, int32_t N, int32_t pieces,
                                grid_timing* timing)
{
    if (!m || !w)
        return fail(GRID_EINVAL, "model and workspace must not be NULL");
    if (w->model != m)
        return fail(GRID_EINVAL, "workspace was created for another model");
    if (N < 0 || N > w->max_knots)
        return fail(GRID_EINVAL, "N must be in 0..max_knots of the workspace");
    if (pieces < 1 || pieces > 64)
        return fail(GRID_EINVAL, "pieces must be in 1..64");
    if (timing)
        *timing = grid_timing{0, 0, 0, 0};
    if (N == 0)
        return GRID_OK;
    HIP_TRY(hipSetDevice(m->device));
    return run_pinned(m, w, N, std::min(pieces, N), timing);
}

grid_status grid_fd_grad_mapped(grid_model m, grid_workspace w, int32_t N, int32_t out_mode,
                                grid_timing* timing)
{
    if (!m || !w)
        return fail(GRID_EINVAL, "model and workspace must not be NULL");
    if (w->model != m)
        return fail(GRID_EINVAL, "workspace was created for another model");
    if (N < 0 || N > w->max_knots)
        return fail(GRID_EINVAL, "N must be in 0..max_knots of the workspace");
    if (out_mode != GRID_IO_COPY_KERNEL && out_mode != GRID_IO_DIRECT)
        return fail(GRID_EINVAL, "unknown output mode " + std::to_string(out_mode));
    if (timing)
        *timing = grid_timing{0, 0, 0, 0};
    if (N == 0)
        return GRID_OK;
    if (!w->h_in_dev || !w->h_out_dev)
        return fail(GRID_EUNSUPPORTED, "the runtime gave no device mapping of the pinned buffers");
    HIP_TRY(hipSetDevice(m->device));
    const size_t n = (size_t)m->topo.n;
    const size_t vec = (size_t)N * n, mat = vec * n;
    const float* q = w->h_in_dev;
    float* out = out_mode == GRID_IO_DIRECT ? w->h_out_dev : w->d_out;
    // events only where a phase boundary is timed (each record costs the stream microseconds)
    const bool copy = out_mode == GRID_IO_COPY_KERNEL;
    if (timing)
        HIP_TRY(hipEventRecord(w->ev[0], w->stream));
    grid_status s = launch_fused(m, N, q, q + vec, q + 2 * vec, out, out + vec, out + vec + mat,
                                 out + vec + 2 * mat, w->stream);
    if (s != GRID_OK)
        return s;
    if (timing)
        HIP_TRY(hipEventRecord(w->ev[1], w->stream));
    if (copy) {
        HIP_TRY(launch_copy_out(w->d_out, w->h_out_dev, vec + 3 * mat, w->stream));
        if (timing)
            HIP_TRY(hipEventRecord(w->ev[2], w->stream));
    }
    HIP_TRY(hipStreamSynchronize(w->stream));
    if (timing) {
        HIP_TRY(hipEventElapsedTime(&timing->kernel_ms, w->ev[0], w->ev[1]));
        if (copy)
            HIP_TRY(hipEventElapsedTime(&timing->d2h_ms, w->ev[1], w->ev[2]));
        HIP_TRY(hipEventElapsedTime(&timing->total_ms, w->ev[0], w->ev[copy ? 2 : 1]));
    }
    return GRID_OK;
}

grid_status grid_fd_grad_host(grid_model m, grid_workspace w, int32_t N, const float* q,
                              const float* qd, const float* tau, float* qdd, float* Minv,
                              float* dqdd_dq, float* dqdd_dqd, grid_timing* timing)
{
    if (!m || !w)
        return fail(GRID_EINVAL, "model and workspace must not be NULL");
    if (w->model != m)
        return fail(GRID_EINVAL, "workspace was created for another model");
    if (N < 0 || N > w->max_knots)
        return fail(GRID_EINVAL, "N must be in 0..max_knots of the workspace");
    if (timing)
        *timing = grid_timing{0, 0, 0, 0};
    if (N == 0)
        return GRID_OK;
    if (!q || !qd || !tau || !qdd || !Minv || !dqdd_dq || !dqdd_dqd)
        return fail(GRID_EINVAL, "a data pointer is NULL");
    HIP_TRY(hipSetDevice(m->device));
    const size_t n = (size_t)m->topo.n;
    const size_t vec = (size_t)N * n, mat = (size_t)N * n * n;
    std::memcpy(w->h_in, q, vec * sizeof(float));
    std::memcpy(w->h_in + vec, qd, vec * sizeof(float));
    std::memcpy(w->h_in + 2 * vec, tau, vec * sizeof(float));
    grid_status s = run_pinned(m, w, N, 1, timing);
    if (s != GRID_OK)
        return s;
    std::memcpy(qdd, w->h_out, vec * sizeof(float));
    std::memcpy(Minv, w->h_out + vec, mat * sizeof(float));
    std::memcpy(dqdd_dq, w->h_out + vec + mat, mat * sizeof(float));
    std::memcpy(dqdd_dqd, w->h_out + vec + 2 * mat, mat * sizeof(float));
    return GRID_OK;
}

}  // extern "C"
