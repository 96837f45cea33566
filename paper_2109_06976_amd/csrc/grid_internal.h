// Internal declarations shared by the host-side translation units of libgrid.
#pragma once

#include "grid.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

namespace grid_impl {

constexpr int kMaxBodies = 32;      // 2n derivative columns fit one wavefront
constexpr int kBodyStride = 24;     // doubles of device constants per body

struct Topology {
    int n = 0;
    int nlev = 0;
    int max_anc = 0;
    int lanes = 0;                       // lanes per knot (power of two >= 2n)
    std::vector<int> parent, level, branch;
    std::vector<uint64_t> level_mask;    // bodies per tree level
    std::vector<uint64_t> round_mask;    // inward accumulation rounds, deepest first
    std::vector<uint64_t> related;       // per body: ancestors, descendants and itself
};

// Kernel argument block; must match grid::Args in grid_device.hip.
struct KernelArgs {
    const double* model;
    double a0[3];
    int nknots;
    const float* q;
    const float* qd;
    const float* tau;
    float* qdd;
    float* Minv;
    float* dqdd_dq;
    float* dqdd_dqd;
};

bool analyse_topology(const int32_t* parent, int32_t n, Topology* out, std::string* err);
std::string generate_source(const Topology& t, uint32_t flags);
grid_status compile_cached(const std::string& source, std::vector<char>* code, std::string* err);
std::string cache_dir();

void set_error(const std::string& msg);

}  // namespace grid_impl

struct grid_model_s {
    int device = 0;
    uint32_t flags = 0;
    grid_impl::Topology topo;
    double a0[3] = {0, 0, 0};
    double* d_model = nullptr;          // n * kBodyStride doubles
    hipModule_t module = nullptr;
    hipFunction_t fused = nullptr;
};

struct grid_workspace_s {
    grid_model model = nullptr;
    int32_t max_knots = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    float* d_in = nullptr;              // q | qd | tau
    float* d_out = nullptr;             // qdd | Minv | dqdd_dq | dqdd_dqd
    float* h_in = nullptr;              // pinned staging
    float* h_out = nullptr;
};
