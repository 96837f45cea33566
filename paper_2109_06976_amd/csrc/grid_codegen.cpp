// Per-robot code generation and compilation (paper Sec. IV-C: the robot's topology is
// known when code is generated, so offsets, parents, level structure and zero patterns
// become constants of the kernel instead of run-time lookups).
//
// A topology (parent array) is turned into a prelude of compile-time tables and
// prepended to the hand-written device source; hiprtc compiles the result for gfx950.
// Code objects are cached on disk under a hash of the full source and options.
#include "grid_internal.h"

#include <hip/hiprtc.h>

#include <dlfcn.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <fstream>
#include <iterator>
#include <mutex>
#include <sstream>

namespace grid_impl {

// embedded copies of grid_device.hip and grid_fused.hip (generated at build time)
#include "grid_device_src.inc"
#include "grid_fused_src.inc"
#include "grid_serial_src.inc"
#include "grid_ops_src.inc"

bool analyse_topology(const int32_t* parent, int32_t n, Topology* out, std::string* err)
{
    if (n < 1 || n > kMaxBodies) {
        *err = "n must be in 1.." + std::to_string(kMaxBodies);
        return false;
    }
    Topology t;
    t.n = n;
    t.parent.assign(parent, parent + n);
    std::vector<int> root(n, -1);
    for (int i = 0; i < n; ++i) {
        const int p = parent[i];
        if (p < -1 || p >= i) {
            *err = "parent[" + std::to_string(i) + "] = " + std::to_string(p) +
                   " must satisfy -1 <= parent[i] < i";
            return false;
        }
        root[i] = p < 0 ? i : root[p];
    }
    // one branch per body attached to the fixed base: that body and all its descendants,
    // in increasing robot index (so every local parent precedes its child)
    int coff = 0;
    for (int r = 0; r < n; ++r) {
        if (parent[r] >= 0)
            continue;
        BranchInst inst;
        std::vector<int> local(n, -1);
        for (int i = 0; i < n; ++i)
            if (root[i] == r) {
                local[i] = (int)inst.body.size();
                inst.body.push_back(i);
                inst.mask |= 1ull << i;
            }
        BranchShape shape;
        shape.B = (int)inst.body.size();
        for (int k = 0; k < shape.B; ++k) {
            const int p = parent[inst.body[k]];
            shape.parent.push_back(p < 0 ? -1 : local[p]);
            uint64_t anc = 0;
            for (int a = shape.parent[k]; a >= 0; a = shape.parent[a])
                anc |= 1ull << a;
            shape.anc.push_back(anc);
        }
        shape.L = 2;
        while (shape.L < 2 * shape.B)
            shape.L *= 2;
        // quad layout: one quad per derivative column; up to 16 quads per wavefront
        if (2 * shape.B <= 16) {
            shape.Q = shape.L;
            shape.W = 1;
        } else {
            shape.Q = 16;
            shape.W = 1;
            while (16 * shape.W < 2 * shape.B)
                shape.W *= 2;
        }
        int sid = -1;
        for (size_t s = 0; s < t.shapes.size(); ++s)
            if (t.shapes[s].parent == shape.parent)
                sid = (int)s;
        if (sid < 0) {
            sid = (int)t.shapes.size();
            t.shapes.push_back(shape);
        }
        inst.shape = sid;
        t.waves = std::max(t.waves, t.shapes[sid].W);
        inst.coff = coff;
        coff += shape.B * kConstStride;
        t.insts.push_back(inst);
    }
    *out = std::move(t);
    return true;
}

int64_t workgroups_for(const Topology& t, int64_t nknots)
{
    int64_t total = 0;
    for (const BranchInst& inst : t.insts) {
        const int K = 64 / t.shapes[inst.shape].L;
        total += (nknots + K - 1) / K;
    }
    return total;
}

// three-role quad kernel: roles B and C take the B columns of M and of M^-1 in QB quads (the
// power of two >= B, at most 16, two columns per quad beyond), so a workgroup holds 16 / QB
// problems; role A takes the 2B derivative columns in two wavefronts (B <= 16) or
// ceil(2B / 16)
int pipe_problems(int B)
{
    int qb = 1;
    while (qb < B && qb < 16)
        qb *= 2;
    return 16 / qb;
}

int pipe_waves(const Topology& t)
{
    int w = 3;
    for (const BranchShape& s : t.shapes) {
        const int wa = std::max(2, (2 * s.B + 15) / 16);   // role A
        w = std::max(w, wa + 1 + (s.B <= 16 ? 1 : 0));      // role B, role C up to 16 bodies
    }
    return w;
}

int64_t workgroups_pipe(const Topology& t, int64_t nknots)
{
    int64_t total = 0;
    for (const BranchInst& inst : t.insts) {
        const int P = pipe_problems(t.shapes[inst.shape].B);
        total += (nknots + P - 1) / P;
    }
    return total;
}

int64_t workgroups_serial(const Topology& t, int64_t nknots, int knots_per_wave)
{
    return (int64_t)t.insts.size() * ((nknots + knots_per_wave - 1) / knots_per_wave);
}

// standalone algorithms (ID, FD, M^-1, dID, VJP): problems per workgroup, as in grid_ops.hip
int64_t workgroups_op(const Topology& t, int64_t nknots, int op)
{
    int64_t total = 0;
    for (const BranchInst& inst : t.insts) {
        const BranchShape& sh = t.shapes[inst.shape];
        const int P = op == kOpId ? 16
                      : op == kOpIdGrad ? (t.waves / sh.W) * (16 / sh.Q)
                                        : pipe_problems(sh.B);   // FD, M^-1, VJP
        total += (nknots + P - 1) / P;
    }
    return total;
}

// problems (knot, branch) per workgroup of the quad-layout kernel
static int quad_problems(const Topology& t, const BranchShape& s)
{
    return (t.waves / s.W) * (16 / s.Q);
}

int64_t workgroups_quad(const Topology& t, int64_t nknots)
{
    int64_t total = 0;
    for (const BranchInst& inst : t.insts) {
        const int P = quad_problems(t, t.shapes[inst.shape]);
        total += (nknots + P - 1) / P;
    }
    return total;
}

WorkspaceLayout workspace_layout(const Topology& t)
{
    WorkspaceLayout w;
    w.c = 0;
    w.L = t.n;
    int total = 0;
    for (const BranchInst& inst : t.insts) {
        w.loff.push_back(total);
        total += (int)(inst.body.size() * inst.body.size());
    }
    w.dinv = w.L + total;
    w.dtau = w.dinv + t.n;
    w.stride = w.dtau + 2 * t.n * t.n;
    return w;
}

int lanes_per_knot(const Topology& t)
{
    int lanes = 0;
    for (const BranchInst& inst : t.insts)
        lanes += t.shapes[inst.shape].L;
    return lanes;
}

template <class T>
static void emit_list(std::ostringstream& os, const std::vector<T>& v, const char* suffix = "")
{
    os << "{";
    for (size_t i = 0; i < v.size(); ++i)
        os << (i ? ", " : "") << v[i] << suffix;
    os << "}";
}

static void emit_floats(std::ostringstream& os, const float* v, size_t k)
{
    // hexadecimal float literals: exact
    char buf[48];
    os << "{";
    for (size_t i = 0; i < k; ++i) {
        std::snprintf(buf, sizeof buf, "%a", (double)v[i]);
        os << (i ? ", " : "") << buf << "f";
    }
    os << "}";
}

// Compile-time structures of one or several robots: the workgroup-size macros (maxima over
// the robots), the distinct branch shapes, and one Inst<k> per branch (numbered across the
// robots) with its robot's joint count, gravity, constants and lane table. inst_base[r] is
// the first Inst index of robot r.
static void emit_prelude(std::ostringstream& os, const std::vector<RobotSource>& robots,
                         std::vector<int>* inst_base)
{
    const Topology& t0 = *robots[0].topo;
    const WorkspaceLayout ws = workspace_layout(t0);   // the staged pipeline: one robot only
    os << "#define GRID_WS_C " << ws.c << "\n#define GRID_WS_L " << ws.L << "\n#define GRID_WS_DINV "
       << ws.dinv << "\n#define GRID_WS_DTAU " << ws.dtau << "\n#define GRID_WS_STRIDE "
       << ws.stride << "\n";
    int waves = 1, pwaves = 1;
    for (const RobotSource& r : robots) {
        waves = std::max(waves, r.topo->waves);
        pwaves = std::max(pwaves, pipe_waves(*r.topo));
    }
    os << "#define GRID_WAVES " << waves << "\n";
    os << "#define GRID_PIPE_WAVES " << pwaves << "\n";
    os << "template <int s> struct Shape;\ntemplate <int k> struct Inst;\n";
    std::vector<BranchShape> shapes;   // distinct shapes over all robots
    auto shape_id = [&](const BranchShape& sh) {
        for (size_t s = 0; s < shapes.size(); ++s)
            if (shapes[s].parent == sh.parent)
                return (int)s;
        shapes.push_back(sh);
        const int s = (int)shapes.size() - 1;
        os << "template <> struct Shape<" << s << "> {\n";
        os << "    static constexpr int B = " << sh.B << ";\n";
        os << "    static constexpr int L = " << sh.L << ";\n";
        os << "    static constexpr int Q = " << sh.Q << ";\n";
        os << "    static constexpr int W = " << sh.W << ";\n";
        os << "    static constexpr int PP = " << pipe_problems(sh.B) << ";\n";
        os << "    static constexpr int parent[B] = ";
        emit_list(os, sh.parent);
        os << ";\n    static constexpr unsigned long long anc[B] = ";
        emit_list(os, sh.anc, "ull");
        os << ";\n};\n";
        return s;
    };
    int kk = 0;
    for (size_t ri = 0; ri < robots.size(); ++ri) {
        const Topology& t = *robots[ri].topo;
        const std::vector<float>& consts = *robots[ri].consts;
        const WorkspaceLayout wsr = workspace_layout(t);
        inst_base->push_back(kk);
        const float a0[3] = {(float)-robots[ri].gravity[0], (float)-robots[ri].gravity[1],
                             (float)-robots[ri].gravity[2]};
        os << "__device__ constexpr float grid_a0_" << ri << "[3] = ";
        emit_floats(os, a0, 3);
        os << ";\n";
        for (size_t k0 = 0; k0 < t.insts.size(); ++k0, ++kk) {
            const BranchInst& in = t.insts[k0];
            const int sid = shape_id(t.shapes[in.shape]);
            const int k = kk;
            // E_T (9), r (3), Ibar (6), h (3), m, 2 unused: per body in local order
            os << "__device__ constexpr float grid_const_" << k << "[" << in.body.size() * kConstStride
               << "] = ";
            emit_floats(os, consts.data() + in.coff, in.body.size() * kConstStride);
            os << ";\n";
            // per-lane constants of the quad layout for lane component c = 0, 1, 2, 16 floats
            // per (c, body): r_c+1, r_c+2, Ibar_cc, Ibar_c,c+1, Ibar_c+2,c, h_c+1, h_c+2, then
            // E_T[row][(c + col) % 3] for row, col = 0..2 (indices mod 3); read through LDS
            {
                const int B = (int)in.body.size();
                std::vector<float> lk((size_t)3 * B * 16);
                for (int c = 0; c < 3; ++c)
                    for (int i = 0; i < B; ++i) {
                        const float* b = consts.data() + in.coff + (size_t)i * kConstStride;
                        const float* r = b + 9;
                        const float* Ib = b + 12;   // xx yy zz xy xz yz
                        const float* h = b + 18;
                        const float ic1[3] = {Ib[3], Ib[5], Ib[4]};   // xy, yz, zx
                        float* o = lk.data() + ((size_t)c * B + i) * 16;
                        o[0] = r[(c + 1) % 3];
                        o[1] = r[(c + 2) % 3];
                        o[2] = Ib[c];
                        o[3] = ic1[c];
                        o[4] = ic1[(c + 2) % 3];
                        o[5] = h[(c + 1) % 3];
                        o[6] = h[(c + 2) % 3];
                        for (int row = 0; row < 3; ++row)
                            for (int col = 0; col < 3; ++col)
                                o[7 + 3 * row + col] = b[3 * row + (c + col) % 3];
                    }
                os << "__device__ alignas(16) const float grid_lk_" << k << "[" << lk.size() << "] = ";
                emit_floats(os, lk.data(), lk.size());
                os << ";\n";
            }
            os << "template <> struct Inst<" << k << "> {\n";
            os << "    using S = Shape<" << sid << ">;\n";
            os << "    static constexpr int N = " << t.n << ";\n";
            os << "    static constexpr int body[S::B] = ";
            emit_list(os, in.body);
            os << ";\n    static constexpr int loff = " << wsr.loff[k0] << ";\n";
            os << "    static constexpr unsigned long long mask = " << in.mask << "ull;\n";
            os << "    static constexpr unsigned long long prism = " << in.prism << "ull;\n";
            os << "    __device__ static int body_of(int i) {\n"
                  "        int r = body[0];\n"
                  "#pragma unroll\n"
                  "        for (int k = 1; k < S::B; ++k) r = (i == k) ? body[k] : r;\n"
                  "        return r;\n    }\n";
            os << "    __device__ static bool contains(int g) { return (mask >> g) & 1ull; }\n";
            os << "    __device__ static const float* consts() { return grid_const_" << k << "; }\n";
            os << "    __device__ static const float* lanek() { return grid_lk_" << k << "; }\n";
            os << "    __device__ static const float* a0() { return grid_a0_" << ri << "; }\n";
            os << "};\n";
        }
    }
}

// A dispatcher walks the branches: workgroups [0, nb_0) run branch 0, the next nb_1 run
// branch 1, and so on. The grid holds exactly sum nb_k workgroups, so the last branch takes
// the rest without a bound check: with one branch nothing waits for nknots before the other
// kernel arguments are loaded. (A workgroup past the end would still only recompute the last
// knot and store nothing: every store checks its knot.) `@` in per_block and call stands for
// the branch's Inst.
// `pool`, when given, is an expression in @ for the LDS floats one branch needs: the dispatch
// then holds one array of the largest such size, `pool`, that every branch's call shares
static void emit_dispatch(std::ostringstream& os, const Topology& t, const char* sig,
                          const std::string& per_block, const std::string& call,
                          const std::string& pool = "")
{
    auto inst = [](size_t k, std::string x) {
        const std::string K = "Inst<" + std::to_string(k) + ">";
        for (size_t at; (at = x.find("@")) != std::string::npos;)
            x.replace(at, 1, K);
        return x;
    };
    os << sig << "\n{\n    int b = block;\n";
    if (!pool.empty()) {
        os << "    __shared__ __align__(16) float pool[grids::cmax(";
        for (size_t k = 0; k < t.insts.size(); ++k)
            os << (k ? ", " : "") << inst(k, pool);
        os << ")];\n";
    }
    for (size_t k = 0; k < t.insts.size(); ++k) {
        auto sub = [&](const std::string& x) { return inst(k, x); };
        if (k + 1 == t.insts.size()) {
            os << "    " << sub(call) << ";\n";
            break;
        }
        os << "    {\n        const int P = " << sub(per_block) << ";\n"
           << "        const int nb = (a.nknots + P - 1) / P;\n"
           << "        if (b < nb) {\n            " << sub(call) << ";\n            return;\n"
           << "        }\n        b -= nb;\n    }\n";
    }
    os << "}\n";
}

std::string generate_source(const Topology& t, const std::vector<float>& consts,
                            const double gravity[3], uint32_t flags)
{
    (void)flags;
    std::ostringstream os;
    os << "// generated: one robot as compile-time structures and constants\n";
    std::vector<int> base;
    RobotSource rs{&t, &consts, {gravity[0], gravity[1], gravity[2]}};
    emit_prelude(os, {rs}, &base);
    os << "#line 1 \"grid_device.hip\"\n";
    os << grid_device_src;
    os << "\n// generated: workgroup -> (branch, knot group)\n";
    emit_dispatch(os, t, "template <int ST>\n__device__ void grid_dispatch(const grid::Args& a, int block)",
             "64 / @::S::L", "grid::run_branch<@, ST>(a, b)");
    os << "#line 1 \"grid_fused.hip\"\n";
    os << grid_fused_src;
    os << "\n// generated: workgroup -> (branch, problem group), quad layout\n";
    emit_dispatch(os, t, "__device__ void grid_dispatch_q(const grid::Args& a, int block)",
             "(GRID_WAVES / @::S::W) * (16 / @::S::Q)", "gridq::run_fused<@>(a, b)");
    os << "#line 1 \"grid_serial.hip\"\n";
    os << grid_serial_src;
    os << "\n// generated: workgroup -> (branch, 64 knots), one lane per knot\n";
    emit_dispatch(os, t, "__device__ void grid_dispatch_s(const grid::Args& a, int block)", "64",
             "grids::run_serial<@, 1, true>(a, b, pool)",
             "grids::serial_stage_floats<@, 1, true>()");
    os << "\n// generated: workgroup -> (branch, 16 or 32 knots), four or two lanes per knot; rows\n"
          "// staged only when every branch's fit\n";
    for (int L : {4, 2}) {
        os << "constexpr bool grid_rows" << L << " = true";
        for (size_t k = 0; k < t.insts.size(); ++k)
            os << " && grids::serial_rows_fit<Inst<" << k << ">, " << L << ">()";
        os << ";\n";
    }
    emit_dispatch(os, t, "__device__ void grid_dispatch_s4(const grid::Args& a, int block)", "16",
             "grids::run_serial<@, 4, grid_rows4>(a, b, pool)",
             "grids::serial_stage_floats<@, 4, grid_rows4>()");
    emit_dispatch(os, t, "__device__ void grid_dispatch_s2(const grid::Args& a, int block)", "32",
             "grids::run_serial<@, 2, grid_rows2>(a, b, pool)",
             "grids::serial_stage_floats<@, 2, grid_rows2>()");
    os << "\n// generated: workgroup -> (branch, 64 knots), M^-1 alone by either route\n";
    emit_dispatch(os, t, "template <bool D>\n__device__ void grid_dispatch_minv(const grid::Args& a, int block)",
             "64", "grids::run_minv<@, D>(a, b)");
    os << "#line 1 \"grid_ops.hip\"\n";
    os << grid_ops_src;
    os << "\n// generated: workgroup -> (branch, problem group), standalone algorithms\n";
    emit_dispatch(os, t, "template <int OP>\n__device__ void grid_dispatch_op(const gridq::OpArgs& a, int block)",
             "gridq::op_problems<@::S, OP>()", "gridq::run_op<@, OP>(a, b)");
    return os.str();
}

// The pipe kernel (build 4) alone, for its own module compiled with the ILP schedule.
std::string generate_pipe_source(const Topology& t, const std::vector<float>& consts,
                                 const double gravity[3])
{
    std::ostringstream os;
    os << "// generated: one robot as compile-time structures and constants, pipe kernel\n";
    os << "#define GRID_PIPE_ONLY 1\n";
    std::vector<int> base;
    RobotSource rs{&t, &consts, {gravity[0], gravity[1], gravity[2]}};
    emit_prelude(os, {rs}, &base);
    os << "#line 1 \"grid_device.hip\"\n";
    os << grid_device_src;
    os << "#line 1 \"grid_fused.hip\"\n";
    os << grid_fused_src;
    os << "\n// generated: workgroup -> (branch, problem group), pipe kernel\n";
    emit_dispatch(os, t, "__device__ void grid_dispatch_p(const grid::Args& a, int block)",
                  "@::S::PP", "gridq::run_pipe<@>(a, b)");
    os << "extern \"C\" __global__ void __launch_bounds__(64 * GRID_PIPE_WAVES) "
          "grid_fdgrad_pipe(grid::Args args)\n{\n"
          "    grid_dispatch_p(args, (int)blockIdx.x);\n}\n";
    return os.str();
}

// Several robots in one module holding only the fused pipe kernel: a launch runs a table of
// items, each one robot's knots with its own buffers. The host splits the grid into segments,
// one per (item, branch) with work, and passes their first workgroups; a workgroup finds its
// segment by a scan of that short table (uniform, scalar loads) and runs the segment's branch.
std::string generate_mixed_source(const std::vector<RobotSource>& robots,
                                  std::vector<int>* inst_base)
{
    std::ostringstream os;
    os << "// generated: " << robots.size() << " robots as compile-time structures and constants\n";
    os << "#define GRID_PIPE_ONLY 1\n";
    emit_prelude(os, robots, inst_base);
    os << "#line 1 \"grid_device.hip\"\n";
    os << grid_device_src;
    os << "#line 1 \"grid_fused.hip\"\n";
    os << grid_fused_src;
    int ninst = 0;
    for (const RobotSource& r : robots)
        ninst += (int)r.topo->insts.size();
    os << "\n// generated: workgroup -> (segment: item, branch), fused pipe kernel\n";
    os << "struct MixedArgs {\n    int nseg;\n    int nblocks;\n    int seg_start[" << kMixedSegs
       << "];\n    int seg_inst[" << kMixedSegs << "];\n    int seg_item[" << kMixedSegs
       << "];\n    int seg_blocks[" << kMixedSegs << "];\n    int seg_wgs[" << kMixedSegs
       << "];\n    grid::Args item[" << kMixedItems << "];\n};\n";
    // the segment of workgroup w: a uniform scan of the first workgroups of the segments
    os << "__device__ __forceinline__ int grid_mixed_segment(const MixedArgs& args, int w)\n{\n"
          "    int s = 0;\n"
          "    while (s + 1 < args.nseg && w >= args.seg_start[s + 1])\n"
          "        ++s;\n"
          "    return s;\n}\n";
    // one workgroup per block: workgroup w runs block w - seg_start of its segment's branch on
    // its item's buffers
    os << "extern \"C\" __global__ void __launch_bounds__(64 * GRID_PIPE_WAVES) "
          "grid_fdgrad_pipe_mixed(MixedArgs args)\n{\n"
          "    const int w = (int)blockIdx.x;\n"
          "    const int s = grid_mixed_segment(args, w);\n"
          "    const grid::Args& x = args.item[args.seg_item[s]];\n"
          "    const int lb = w - args.seg_start[s];\n"
          "    switch (args.seg_inst[s]) {\n";
    for (int k = 0; k < ninst; ++k)
        os << "    " << (k + 1 == ninst ? std::string("default") : "case " + std::to_string(k))
           << ": gridq::run_pipe<Inst<" << k << ">>(x, lb); break;\n";
    os << "    }\n}\n";
    // persistent: each segment owns seg_wgs resident workgroups, and each of them strides over
    // the segment's blocks. The loop sits inside the segment's case, so what the compiler keeps
    // live across iterations belongs to that one branch (a loop around the whole switch keeps
    // every branch's per-lane set-up live at once: 307 VGPRs against 168 for two robots). A
    // workgroup's blocks are uniform, so every wavefront takes each block's three barriers
    // (lane table T, bias forces C, products P). Reusing LDS for the next block is ordered by
    // those barriers: s_tab is written after P (read before C); s_c, s_M, the factor and s_D
    // after T or C of the next block (read before P, or just after P by a wavefront that then
    // reaches T); s_Mi after C (read after P).
    os << "extern \"C\" __global__ void __launch_bounds__(64 * GRID_PIPE_WAVES) "
          "grid_fdgrad_pipe_mixed_persistent(MixedArgs args)\n{\n"
          "    const int w = (int)blockIdx.x;\n"
          "    const int s = grid_mixed_segment(args, w);\n"
          "    const grid::Args& x = args.item[args.seg_item[s]];\n"
          "    const int lw = w - args.seg_start[s];\n"
          "    const int nb = args.seg_blocks[s];\n"
          "    const int nw = args.seg_wgs[s];\n"
          "    switch (args.seg_inst[s]) {\n";
    for (int k = 0; k < ninst; ++k)
        os << "    " << (k + 1 == ninst ? std::string("default") : "case " + std::to_string(k))
           << ":\n        for (int lb = lw; lb < nb; lb += nw)\n"
              "            gridq::run_pipe<Inst<" << k << ">, true>(x, lb);\n        break;\n";
    os << "    }\n}\n";
    return os.str();
}

static const char* const kCompileOptions[] = {
    "--offload-arch=gfx950", "-O3", "-std=c++17",
    // packed FP32 instructions are not generated (correctness of some packed forms)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
};

// the pipe kernel's own module: each of its wavefronts has a SIMD to itself and runs one long
// dependent chain, so it is scheduled for instruction-level parallelism rather than
// occupancy (chain7, N = 128: 4.65 against 4.97 us per launch; quad12 and humanoid30
// unchanged). The throughput builds keep the default (build 2 at N = 16384 lost 9% with it).
static const char* const kIlpOptions[] = {"-mllvm", "-amdgpu-sched-strategy=max-ilp"};

static uint64_t fnv1a(const std::string& s, uint64_t h = 1469598103934665603ull)
{
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

uint64_t source_hash(const std::string& source) { return fnv1a(source); }

// The machine code and constant data of an ELF64 code object: the .text, .rodata and .note
// sections (instructions, kernel descriptors and constant tables, kernel metadata), in that
// order, each behind its name. The symbol tables are left out: they carry an identifier of
// the compilation that changes with any edit of the source text, comments included, while the
// machine code stays the same. An object that does not parse as ELF64 is taken whole.
std::string machine_code(const std::vector<char>& elf)
{
    const std::string whole(elf.begin(), elf.end());
    auto rd = [&](size_t off, size_t n, uint64_t* v) {
        if (off + n > elf.size())
            return false;
        uint64_t x = 0;
        for (size_t k = 0; k < n; ++k)   // little endian
            x |= (uint64_t)(unsigned char)elf[off + k] << (8 * k);
        *v = x;
        return true;
    };
    if (elf.size() < 64 || elf[0] != 0x7f || elf[1] != 'E' || elf[2] != 'L' || elf[3] != 'F' ||
        elf[4] != 2)
        return whole;
    uint64_t shoff, shentsize, shnum, shstrndx;
    if (!rd(0x28, 8, &shoff) || !rd(0x3a, 2, &shentsize) || !rd(0x3c, 2, &shnum) ||
        !rd(0x3e, 2, &shstrndx) || shentsize < 64 || shstrndx >= shnum)
        return whole;
    auto sec = [&](uint64_t k, uint64_t* name, uint64_t* type, uint64_t* off, uint64_t* size) {
        const size_t h = (size_t)(shoff + k * shentsize);
        return rd(h, 4, name) && rd(h + 4, 4, type) && rd(h + 24, 8, off) && rd(h + 32, 8, size);
    };
    uint64_t sn, st, soff, ssize;
    if (!sec(shstrndx, &sn, &st, &soff, &ssize) || soff + ssize > elf.size())
        return whole;
    std::string out;
    for (const char* want : {".text", ".rodata", ".note"}) {
        for (uint64_t k = 0; k < shnum; ++k) {
            uint64_t name, type, off, size;
            if (!sec(k, &name, &type, &off, &size) || name >= ssize)
                return whole;
            const char* nm = elf.data() + soff + name;
            if (std::strncmp(nm, want, ssize - name) != 0)
                continue;
            if (type == 8)                    // SHT_NOBITS: nothing in the file
                continue;
            if (off + size > elf.size())
                return whole;
            out += want;
            out.append(elf.data() + off, (size_t)size);
        }
    }
    return out.empty() ? whole : out;
}

std::string cache_dir()
{
    if (const char* env = std::getenv("GRID_KERNEL_CACHE"))
        if (*env)
            return env;
    Dl_info info;
    if (dladdr(reinterpret_cast<void*>(&cache_dir), &info) && info.dli_fname) {
        std::string so = info.dli_fname;
        size_t slash = so.rfind('/');
        std::string dir = slash == std::string::npos ? "." : so.substr(0, slash);
        return dir + "/_kcache";
    }
    return "/tmp/grid_kcache";
}

static bool read_file(const std::string& path, std::vector<char>* out)
{
    std::ifstream f(path, std::ios::binary);
    if (!f)
        return false;
    out->assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
    return !out->empty();
}

static void write_file_atomic(const std::string& dir, const std::string& path,
                              const std::vector<char>& data)
{
    mkdir(dir.c_str(), 0755);
    std::string tmp = path + ".tmp" + std::to_string(getpid());
    {
        std::ofstream f(tmp, std::ios::binary);
        if (!f)
            return;   // cache is best effort
        f.write(data.data(), data.size());
        if (!f)
            return;
    }
    std::rename(tmp.c_str(), path.c_str());
}

static std::mutex g_compile_mutex;

grid_status compile_cached(const std::string& source, std::vector<char>* code, std::string* err,
                           bool ilp)
{
    std::vector<const char*> opts(std::begin(kCompileOptions), std::end(kCompileOptions));
    if (ilp)
        opts.insert(opts.end(), std::begin(kIlpOptions), std::end(kIlpOptions));
    std::string key_src = source;
    for (const char* o : opts)
        key_src += std::string("\n//opt ") + o;
    char name[64];
    std::snprintf(name, sizeof name, "grid_%016llx.hsaco", (unsigned long long)fnv1a(key_src));
    const std::string dir = cache_dir();
    const std::string path = dir + "/" + name;
    if (read_file(path, code))
        return GRID_OK;

    std::lock_guard<std::mutex> lock(g_compile_mutex);
    if (read_file(path, code))
        return GRID_OK;
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, source.c_str(), "grid_robot.hip", 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS) {
        *err = "hiprtcCreateProgram failed";
        return GRID_ECOMPILE;
    }
    hiprtcResult rc = hiprtcCompileProgram(prog, (int)opts.size(), opts.data());
    if (rc != HIPRTC_SUCCESS) {
        size_t log_size = 0;
        hiprtcGetProgramLogSize(prog, &log_size);
        std::string log(log_size, '\0');
        if (log_size)
            hiprtcGetProgramLog(prog, &log[0]);
        *err = std::string("kernel compilation failed: ") + hiprtcGetErrorString(rc) + "\n" + log;
        hiprtcDestroyProgram(&prog);
        return GRID_ECOMPILE;
    }
    size_t size = 0;
    hiprtcGetCodeSize(prog, &size);
    code->resize(size);
    hiprtcGetCode(prog, code->data());
    hiprtcDestroyProgram(&prog);
    write_file_atomic(dir, path, *code);
    return GRID_OK;
}

}  // namespace grid_impl
