// Internal declarations shared by the host-side translation units of libgrid.
#pragma once

#include "grid.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

namespace grid_impl {

constexpr int kMaxBodies = 32;      // the 2B derivative columns of a branch fit one wavefront
constexpr int kConstStride = 24;    // floats of device constants per body

// builds of the fused kernel: quad layout, lane layout at 1, 2, 4 wavefronts per SIMD,
// quad layout in three roles, one lane per knot, four lanes per knot, two lanes per knot
constexpr int kVariantQuad = 0;
constexpr int kVariantLane1 = 1;
constexpr int kVariantPipe = 4;
constexpr int kVariantSerial = 5;
constexpr int kVariantSerial4 = 6;
constexpr int kVariantSerial2 = 7;
constexpr int kNumVariants = 8;

// standalone algorithms (grid_ops.hip)
constexpr int kOpId = 0;
constexpr int kOpFd = 1;
constexpr int kOpMinv = 2;
constexpr int kOpIdGrad = 3;
constexpr int kOpVjp = 4;
constexpr int kNumOps = 5;

// argument block of the standalone kernels; must match gridq::OpArgs in grid_ops.hip
struct OpArgs {
    int nknots;
    const float* q;
    const float* qd;
    const float* u;
    const float* u2;
    float* out0;
    float* out1;
    float* out2;
};

// A branch hanging off the fixed base, in local numbering (parent before child).
struct BranchShape {
    int B = 0;                       // bodies
    int L = 0;                       // lanes per knot: power of two >= 2B
    int Q = 0;                       // quad layout: quads per wavefront per problem
    int W = 0;                       // quad layout: wavefronts per problem
    std::vector<int> parent;         // local parent, -1 = the fixed base
    std::vector<uint64_t> anc;       // strict ancestors (local bit masks)
};

// One base branch of a robot: its shape and where its bodies sit in the robot.
struct BranchInst {
    int shape = 0;
    std::vector<int> body;           // robot index of each local body
    int coff = 0;                    // float offset of the branch's constants
    uint64_t mask = 0;               // robot bodies in this branch
    uint64_t prism = 0;              // local bodies on prismatic joints
};

struct Topology {
    int n = 0;
    std::vector<int> parent;
    std::vector<BranchShape> shapes;
    std::vector<BranchInst> insts;
    int waves = 1;                   // quad layout: wavefronts per workgroup (max W)
};

// Staged pipeline workspace per knot (floats): c [n], the factors L of every branch
// [sum B^2], 1/L_kk [n], dtau/dq and dtau/dqd [2 n^2].
struct WorkspaceLayout {
    int c = 0, L = 0, dinv = 0, dtau = 0, stride = 0;
    std::vector<int> loff;           // per branch: offset of its B x B factor
};

// Kernel argument block; must match grid::Args in grid_device.hip.
struct KernelArgs {
    int nknots;
    float* work;
    const float* q;
    const float* qd;
    const float* tau;
    float* qdd;
    float* Minv;
    float* dqdd_dq;
    float* dqdd_dqd;
};

// A robot as the code generator sees it: topology, packed constants and gravity.
struct RobotSource {
    const Topology* topo;
    const std::vector<float>* consts;
    double gravity[3];
};

// One module for several robots (the fused pipe kernel only): workgroup segments of a launch
// name the item they serve and the branch (Inst index over all robots) they run.
constexpr int kMixedItems = 16;
constexpr int kMixedSegs = 64;

// Kernel argument block of the mixed kernel; must match MixedArgs of the generated source.
struct MixedArgs {
    int nseg;
    int nblocks;                     // blocks of the launch over all segments
    int seg_start[kMixedSegs];       // first workgroup of the segment, ascending
    int seg_inst[kMixedSegs];        // the branch the segment runs
    int seg_item[kMixedSegs];        // the item whose buffers it reads and writes
    int seg_blocks[kMixedSegs];      // blocks of the segment
    int seg_wgs[kMixedSegs];         // workgroups of the segment (= seg_blocks for one
                                     // workgroup per block; fewer in the persistent form)
    KernelArgs item[kMixedItems];
};

bool analyse_topology(const int32_t* parent, int32_t n, Topology* out, std::string* err);
std::vector<float> pack_constants(const grid_model_desc* d, const Topology& t);
std::string generate_source(const Topology& t, const std::vector<float>& consts,
                            const double gravity[3], uint32_t flags);
std::string generate_pipe_source(const Topology& t, const std::vector<float>& consts,
                                 const double gravity[3]);
std::string generate_mixed_source(const std::vector<RobotSource>& robots,
                                  std::vector<int>* inst_base);
grid_status prepare_robot(const grid_model_desc* desc, Topology* topo,
                          std::vector<float>* consts, std::string* err);
grid_status validate_desc(const grid_model_desc* d, std::string* err);
int64_t workgroups_for(const Topology& t, int64_t nknots);
int64_t workgroups_quad(const Topology& t, int64_t nknots);
int64_t workgroups_pipe(const Topology& t, int64_t nknots);
int64_t workgroups_serial(const Topology& t, int64_t nknots, int knots_per_wave = 64);
int64_t workgroups_op(const Topology& t, int64_t nknots, int op);
int pipe_problems(int B);
int pipe_waves(const Topology& t);
int lanes_per_knot(const Topology& t);
WorkspaceLayout workspace_layout(const Topology& t);
// ilp: the instruction-level-parallelism schedule (the pipe kernel's module)
grid_status compile_cached(const std::string& source, std::vector<char>* code, std::string* err,
                           bool ilp = false);
uint64_t source_hash(const std::string& source);
std::string machine_code(const std::vector<char>& elf);
grid_status launch_fused(grid_model m, int32_t N, const float* q, const float* qd,
                         const float* tau, float* qdd, float* Minv, float* dq, float* dqd,
                         hipStream_t stream);
grid_status launch_fused_variant(grid_model m, int variant, int32_t N, const float* q,
                                 const float* qd, const float* tau, float* qdd, float* Minv,
                                 float* dq, float* dqd, hipStream_t stream);
int fused_variant_for(grid_model m, int32_t N);
void load_tuning(grid_model m);
std::string cache_dir();

void set_error(const std::string& msg);

hipError_t launch_vjp(int nknots, int n, const float* dq, const float* dqd, const float* Minv,
                      const float* g, float* qbar, float* qdbar, float* taubar, hipStream_t stream);
hipError_t launch_dt(int nknots, int n, float dt, const float* dq, const float* dqd,
                     const float* Minv, float* A, float* B, hipStream_t stream);

// device -> pinned host copy of n floats by a kernel (16-byte stores; both 16-byte aligned)
hipError_t launch_copy_out(const float* src, float* dst, size_t n, hipStream_t stream);

// the library's static scratch array (grid_noalloc.hip): its device address on `device`, taken
// once with that device current; noalloc_scratch returns it (NULL before the setup)
grid_status noalloc_setup(int device, std::string* err);
float* noalloc_scratch(int device);

}  // namespace grid_impl

struct grid_model_s {
    int device = 0;
    uint32_t flags = 0;
    grid_impl::Topology topo;
    uint64_t code_hash = 0;             // of the two loaded code objects, in that order:
                                        // keys tuning tables
    int compute_units = 256;
    hipFunction_t fused_variant[grid_impl::kNumVariants] = {};   // see kVariantQuad
    hipFunction_t op[grid_impl::kNumOps] = {};                    // see kOpId
    hipFunction_t minv_route[2] = {};   // M^-1 one lane per knot: L^T L, direct
    std::vector<std::pair<int32_t, int>> tuned;   // (largest N, variant), ascending N
    hipModule_t module = nullptr;
    hipModule_t pipe_module = nullptr;  // build 4 alone, compiled with the ILP schedule
    hipFunction_t stage[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

struct grid_workspace_s {
    grid_model model = nullptr;
    int32_t max_knots = 0;
    hipStream_t stream = nullptr;
    hipStream_t stream2 = nullptr;      // second stream of the pieces of a pinned call
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    float* d_in = nullptr;              // q | qd | tau
    float* d_out = nullptr;             // qdd | Minv | dqdd_dq | dqdd_dqd
    float* d_stage = nullptr;           // staged pipeline intermediates
    float* h_in = nullptr;              // pinned staging
    float* h_out = nullptr;
    float* h_in_dev = nullptr;          // the device's mapping of h_in and h_out (NULL if the
    float* h_out_dev = nullptr;         // runtime gives none: the mapped call is unsupported)
};
