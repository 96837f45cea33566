// Mixed-robot batches (one launch per item, or one hipGraph replay for all items) and the
// autotuner that picks a build of the fused kernel per batch size (include/grid.h).
#include "grid_internal.h"

#include <algorithm>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>

using namespace grid_impl;

namespace {

constexpr int kMaxItems = 64;

grid_status fail(grid_status s, const std::string& msg)
{
    set_error(msg);
    return s;
}

#define HIP_TRY(expr)                                                          \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess)                                                  \
            return fail(GRID_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

grid_status check_items(const grid_item* items, int32_t count)
{
    if (!items || count < 1 || count > kMaxItems)
        return fail(GRID_EINVAL, "items must hold 1..64 entries");
    for (int k = 0; k < count; ++k) {
        const grid_item& it = items[k];
        if (!it.model || it.N < 0 || it.N > GRID_MAX_KNOTS)
            return fail(GRID_EINVAL, "item " + std::to_string(k) +
                                         ": NULL model or N outside 0..GRID_MAX_KNOTS");
        if (it.model->device != items[0].model->device)
            return fail(GRID_EINVAL, "all items must be on one device");
        if (it.N > 0 && (!it.q || !it.qd || !it.tau || !it.qdd || !it.Minv || !it.dqdd_dq ||
                         !it.dqdd_dqd))
            return fail(GRID_EINVAL, "item " + std::to_string(k) + ": a data pointer is NULL");
    }
    return GRID_OK;
}

}  // namespace

struct grid_graph_s {
    int device = 0;
    int count = 0;
    grid_mixed mx = nullptr;    // a graph of one mixed launch (grid_mixed_graph_create)
    int mode = -1;              // its launch mode (-1: the tuned one at each capture)
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// `issue` enqueues the graph's work on the capture stream. The items' kernels in sequence
// make a chain of kernel nodes. (A first version forked every item onto a side stream so that
// the nodes had no edges between them; on ROCm 7.2 launching that graph took 39 us of host
// time for two nodes, the chain 14 us.)
template <class Issue>
grid_status capture_with(grid_graph g, Issue issue, hipGraph_t* out)
{
    HIP_TRY(hipStreamBeginCapture(g->capture, hipStreamCaptureModeThreadLocal));
    grid_status st = issue(g->capture);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(g->capture, &graph);
    if (st != GRID_OK) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return st;
    }
    if (e2 != hipSuccess) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return fail(GRID_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e2));
    }
    *out = graph;
    return GRID_OK;
}

grid_status capture(grid_graph g, const grid_item* items, int32_t count, hipGraph_t* out)
{
    return capture_with(g, [&](hipStream_t s) {
        grid_status st = GRID_OK;
        for (int k = 0; k < count && st == GRID_OK; ++k)
            if (items[k].N > 0)
                st = launch_fused(items[k].model, items[k].N, items[k].q, items[k].qd,
                                  items[k].tau, items[k].qdd, items[k].Minv, items[k].dqdd_dq,
                                  items[k].dqdd_dqd, s);
        return st;
    }, out);
}

// replace the graph's executable by one of `fresh`: updated in place, or re-instantiated if
// the update is refused; takes ownership of `fresh`
grid_status swap_in(grid_graph g, hipGraph_t fresh)
{
    hipGraphNode_t err_node = nullptr;
    hipGraphExecUpdateResult res;
    if (hipGraphExecUpdate(g->exec, fresh, &err_node, &res) != hipSuccess ||
        res != hipGraphExecUpdateSuccess) {
        (void)hipGetLastError();
        hipGraphExec_t exec = nullptr;
        hipError_t e = hipGraphInstantiate(&exec, fresh, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(fresh);
            return fail(GRID_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        (void)hipGraphExecDestroy(g->exec);
        g->exec = exec;
    }
    (void)hipGraphDestroy(g->graph);
    g->graph = fresh;
    return GRID_OK;
}

void destroy_graph(grid_graph g)
{
    if (g->exec)
        (void)hipGraphExecDestroy(g->exec);
    if (g->graph)
        (void)hipGraphDestroy(g->graph);
    if (g->capture)
        (void)hipStreamDestroy(g->capture);
    delete g;
}

}  // namespace

extern "C" {

grid_status grid_fd_grad_batch(const grid_item* items, int32_t count, void* stream)
{
    grid_status st = check_items(items, count);
    if (st != GRID_OK)
        return st;
    HIP_TRY(hipSetDevice(items[0].model->device));
    for (int k = 0; k < count; ++k) {
        const grid_item& it = items[k];
        if (it.N == 0)
            continue;
        st = launch_fused(it.model, it.N, it.q, it.qd, it.tau, it.qdd, it.Minv, it.dqdd_dq,
                          it.dqdd_dqd, (hipStream_t)stream);
        if (st != GRID_OK)
            return st;
    }
    return GRID_OK;
}

grid_status grid_graph_create(const grid_item* items, int32_t count, grid_graph* out)
{
    if (!out)
        return fail(GRID_EINVAL, "out must not be NULL");
    *out = nullptr;
    grid_status st = check_items(items, count);
    if (st != GRID_OK)
        return st;
    HIP_TRY(hipSetDevice(items[0].model->device));
    grid_graph g = new (std::nothrow) grid_graph_s;
    if (!g)
        return fail(GRID_ENOMEM, "host allocation failed");
    g->device = items[0].model->device;
    g->count = count;
    hipError_t e = hipStreamCreateWithFlags(&g->capture, hipStreamNonBlocking);
    if (e != hipSuccess) {
        destroy_graph(g);
        return fail(GRID_EDEVICE, std::string("graph stream: ") + hipGetErrorString(e));
    }
    st = capture(g, items, count, &g->graph);
    if (st == GRID_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess)
            st = fail(GRID_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    if (st != GRID_OK) {
        destroy_graph(g);
        return st;
    }
    *out = g;
    return GRID_OK;
}

grid_status grid_graph_launch(grid_graph g, void* stream)
{
    if (!g)
        return fail(GRID_EINVAL, "graph is NULL");
    HIP_TRY(hipSetDevice(g->device));
    HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return GRID_OK;
}

grid_status grid_graph_update(grid_graph g, const grid_item* items, int32_t count)
{
    if (!g)
        return fail(GRID_EINVAL, "graph is NULL");
    grid_status st = check_items(items, count);
    if (st != GRID_OK)
        return st;
    if (g->mx)
        return fail(GRID_EINVAL, "a graph of a mixed launch is updated by grid_mixed_graph_update");
    if (count != g->count || items[0].model->device != g->device)
        return fail(GRID_EINVAL, "an update keeps the item count and the device");
    HIP_TRY(hipSetDevice(g->device));
    hipGraph_t fresh = nullptr;
    st = capture(g, items, count, &fresh);
    if (st != GRID_OK)
        return st;
    return swap_in(g, fresh);
}

grid_status grid_graph_destroy(grid_graph g)
{
    if (!g)
        return GRID_OK;
    (void)hipSetDevice(g->device);
    (void)hipStreamSynchronize(g->capture);
    destroy_graph(g);
    return GRID_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ one launch, several robots

// the block is passed by value as the kernel's only argument: its host layout must be the
// device one (ints, then 8-byte aligned argument blocks of the same field order)
static_assert(sizeof(KernelArgs) == 72, "Args: an int and eight pointers");
static_assert(offsetof(MixedArgs, item) == 8 + 5 * 4 * kMixedSegs &&
                  sizeof(MixedArgs) == offsetof(MixedArgs, item) + kMixedItems * sizeof(KernelArgs),
              "MixedArgs layout");

struct grid_mixed_s {
    int device = 0;
    std::vector<Topology> topo;       // per robot
    std::vector<int> inst_base;       // per robot: index of its first branch in the module
    int waves = 1;                    // wavefronts per workgroup (the largest robot's)
    hipModule_t module = nullptr;
    hipFunction_t fn = nullptr;             // one workgroup per block
    hipFunction_t fn_persistent = nullptr;  // resident workgroups striding over the blocks
    int resident = 0;                       // workgroups of fn_persistent resident at once
    std::vector<grid_model> models;         // per robot: its own modules (per-robot launches)
    // (blocks of the largest tuned plan, mode): a launch of B blocks uses the mode tuned for
    // the smallest entry >= B (the last one beyond); untuned: one workgroup per block
    std::vector<std::pair<int64_t, int>> tuned;
};

namespace {

// the robots' topologies, constants and the module source
grid_status mixed_source(const grid_model_desc* descs, int32_t count, std::vector<Topology>* topo,
                         std::vector<int>* inst_base, std::string* src)
{
    if (!descs || count < 1 || count > kMixedItems)
        return fail(GRID_EINVAL, "descs must hold 1.." + std::to_string(kMixedItems) + " models");
    topo->assign(count, Topology());
    std::vector<std::vector<float>> consts(count);
    std::vector<RobotSource> rs;
    for (int r = 0; r < count; ++r) {
        std::string err;
        const grid_status st = prepare_robot(&descs[r], &(*topo)[r], &consts[r], &err);
        if (st != GRID_OK)
            return fail(st, "model " + std::to_string(r) + ": " + err);
    }
    for (int r = 0; r < count; ++r)
        rs.push_back(RobotSource{&(*topo)[r], &consts[r],
                                 {descs[r].gravity[0], descs[r].gravity[1], descs[r].gravity[2]}});
    inst_base->clear();
    *src = generate_mixed_source(rs, inst_base);
    return GRID_OK;
}

}  // namespace

extern "C" {

grid_status grid_mixed_source(const grid_model_desc* descs, int32_t count, char* buf, size_t* len)
{
    if (!len)
        return fail(GRID_EINVAL, "len must not be NULL");
    std::vector<Topology> topo;
    std::vector<int> base;
    std::string src;
    const grid_status st = mixed_source(descs, count, &topo, &base, &src);
    if (st != GRID_OK)
        return st;
    const size_t need = src.size() + 1;
    const bool fits = buf && *len >= need;
    if (fits)
        std::memcpy(buf, src.c_str(), need);
    *len = need;
    if (buf && !fits)
        return fail(GRID_EINVAL, "buffer too small");
    return GRID_OK;
}

grid_status grid_mixed_precompile(const grid_model_desc* descs, int32_t count)
{
    std::vector<Topology> topo;
    std::vector<int> base;
    std::string src, err;
    grid_status st = mixed_source(descs, count, &topo, &base, &src);
    if (st != GRID_OK)
        return st;
    std::vector<char> code;
    st = compile_cached(src, &code, &err);
    return st == GRID_OK ? GRID_OK : fail(st, err);
}

grid_status grid_mixed_create(const grid_model_desc* descs, int32_t count, int32_t device,
                              grid_mixed* out)
{
    if (!out)
        return fail(GRID_EINVAL, "out must not be NULL");
    *out = nullptr;
    std::vector<Topology> topo;
    std::vector<int> base;
    std::string src, err;
    grid_status st = mixed_source(descs, count, &topo, &base, &src);
    if (st != GRID_OK)
        return st;
    std::vector<char> code;
    st = compile_cached(src, &code, &err);
    if (st != GRID_OK)
        return fail(st, err);
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev)
        return fail(GRID_EINVAL, "device index out of range");
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(GRID_EUNSUPPORTED, std::string("device is ") + prop.gcnArchName +
                                           ", kernels are built for gfx950");
    grid_mixed mx = new (std::nothrow) grid_mixed_s;
    if (!mx)
        return fail(GRID_ENOMEM, "host allocation failed");
    mx->device = device;
    mx->topo = std::move(topo);
    mx->inst_base = std::move(base);
    for (const Topology& t : mx->topo)
        mx->waves = std::max(mx->waves, pipe_waves(t));
    hipError_t e = hipModuleLoadData(&mx->module, code.data());
    if (e == hipSuccess)
        e = hipModuleGetFunction(&mx->fn, mx->module, "grid_fdgrad_pipe_mixed");
    if (e == hipSuccess)
        e = hipModuleGetFunction(&mx->fn_persistent, mx->module,
                                 "grid_fdgrad_pipe_mixed_persistent");
    int per_cu = 0, cus = 0;
    if (e == hipSuccess)
        e = hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mx->fn_persistent,
                                                               64 * mx->waves, 0);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) {
        grid_mixed_destroy(mx);
        return fail(GRID_EDEVICE, std::string("mixed module load: ") + hipGetErrorString(e));
    }
    mx->resident = std::max(1, per_cu) * std::max(1, cus);
    for (int r = 0; r < count; ++r) {
        grid_model m = nullptr;
        st = grid_model_create(&descs[r], device, 0, &m);
        if (st != GRID_OK) {
            grid_mixed_destroy(mx);
            return st;
        }
        mx->models.push_back(m);
    }
    *out = mx;
    return GRID_OK;
}

}  // extern "C"

namespace {

// Checks the items and builds the segment table of a launch: one segment per (item, branch)
// with knots, each with its first workgroup, its blocks and its workgroups. One workgroup per
// block: in item order. Persistent (`resident` > 0): ordered by the branch's bodies, largest
// first, and the resident workgroups (at most one per block) shared among the segments in
// proportion to their blocks times a per-block cost of (bodies + 4), at least one each.
// *blocks: the blocks of the launch; *wgs: its workgroups.
grid_status mixed_args(grid_mixed mx, const grid_mixed_item* items, int32_t count,
                       int64_t resident, MixedArgs* a, int64_t* blocks, int64_t* wgs = nullptr)
{
    if (!mx)
        return fail(GRID_EINVAL, "mixed module is NULL");
    if (!items || count < 1 || count > kMixedItems)
        return fail(GRID_EINVAL, "items must hold 1.." + std::to_string(kMixedItems) + " entries");
    std::memset(a, 0, sizeof *a);
    struct Seg {
        int inst, item, B;
        int64_t nb;
    };
    std::vector<Seg> segs;
    for (int j = 0; j < count; ++j) {
        const grid_mixed_item& it = items[j];
        if (it.robot < 0 || it.robot >= (int)mx->topo.size())
            return fail(GRID_EINVAL, "item " + std::to_string(j) + ": robot index out of range");
        if (it.N < 0 || it.N > GRID_MAX_KNOTS)
            return fail(GRID_EINVAL, "item " + std::to_string(j) + ": N out of range");
        if (it.N > 0 && (!it.q || !it.qd || !it.tau || !it.qdd || !it.Minv || !it.dqdd_dq ||
                         !it.dqdd_dqd))
            return fail(GRID_EINVAL, "item " + std::to_string(j) + ": a data pointer is NULL");
        KernelArgs& k = a->item[j];
        k.nknots = it.N;
        k.work = nullptr;
        k.q = it.q;
        k.qd = it.qd;
        k.tau = it.tau;
        k.qdd = it.qdd;
        k.Minv = it.Minv;
        k.dqdd_dq = it.dqdd_dq;
        k.dqdd_dqd = it.dqdd_dqd;
        if (it.N == 0)
            continue;
        const Topology& t = mx->topo[it.robot];
        for (size_t b = 0; b < t.insts.size(); ++b) {
            if ((int)segs.size() == kMixedSegs)
                return fail(GRID_EINVAL, "more than " + std::to_string(kMixedSegs) +
                                             " (item, branch) segments in one launch");
            const int B = t.shapes[t.insts[b].shape].B;
            const int P = pipe_problems(B);
            segs.push_back(Seg{mx->inst_base[it.robot] + (int)b, j, B, (it.N + P - 1) / P});
        }
    }
    const bool pers = resident > 0;
    if (pers)
        std::stable_sort(segs.begin(), segs.end(),
                         [](const Seg& x, const Seg& y) { return x.B > y.B; });
    int64_t total = 0;
    for (const Seg& g : segs)
        total += g.nb;
    if (total > INT32_MAX)
        return fail(GRID_EINVAL, "too many knots in one launch");
    std::vector<int64_t> w(segs.size());
    for (size_t k = 0; k < segs.size(); ++k)
        w[k] = segs[k].nb;
    if (pers && total > 0) {
        const int64_t W = std::min<int64_t>(total, resident);
        double cost = 0;
        for (const Seg& g : segs)
            cost += (double)g.nb * (g.B + 4);
        int64_t used = 0;
        for (size_t k = 0; k < segs.size(); ++k) {
            const double share = (double)W * segs[k].nb * (segs[k].B + 4) / cost;
            w[k] = std::max<int64_t>(1, std::min<int64_t>(segs[k].nb, (int64_t)share));
            used += w[k];
        }
        // the rest of the resident workgroups to the segments with the most cost per workgroup
        for (; used < W; ++used) {
            size_t best = segs.size();
            double most = 0;
            for (size_t k = 0; k < segs.size(); ++k) {
                const double per = (double)segs[k].nb * (segs[k].B + 4) / (double)w[k];
                if (w[k] < segs[k].nb && per > most) {
                    most = per;
                    best = k;
                }
            }
            if (best == segs.size())
                break;
            ++w[best];
        }
    }
    int64_t start = 0;
    for (size_t k = 0; k < segs.size(); ++k) {
        a->seg_start[a->nseg] = (int)start;
        a->seg_inst[a->nseg] = segs[k].inst;
        a->seg_item[a->nseg] = segs[k].item;
        a->seg_blocks[a->nseg] = (int)segs[k].nb;
        a->seg_wgs[a->nseg] = (int)w[k];
        ++a->nseg;
        start += w[k];
    }
    a->nblocks = (int)total;
    *blocks = total;
    if (wgs)
        *wgs = start;
    return GRID_OK;
}

grid_status mixed_launch_mode(grid_mixed mx, const grid_mixed_item* items, int32_t count,
                              int mode, hipStream_t stream)
{
    if (mode < GRID_MIXED_ONE_LAUNCH || mode > GRID_MIXED_PER_ROBOT)
        return fail(GRID_EINVAL, "unknown mixed launch mode " + std::to_string(mode));
    MixedArgs a;
    int64_t blocks = 0, wgs = 0;
    const bool pers = mode == GRID_MIXED_PERSISTENT;
    grid_status st = mixed_args(mx, items, count, pers ? mx->resident : 0, &a, &blocks, &wgs);
    if (st != GRID_OK)
        return st;
    if (blocks == 0)
        return GRID_OK;
    HIP_TRY(hipSetDevice(mx->device));
    if (mode == GRID_MIXED_PER_ROBOT) {
        for (int j = 0; j < count; ++j) {
            const grid_mixed_item& it = items[j];
            if (it.N == 0)
                continue;
            st = launch_fused(mx->models[it.robot], it.N, it.q, it.qd, it.tau, it.qdd, it.Minv,
                              it.dqdd_dq, it.dqdd_dqd, stream);
            if (st != GRID_OK)
                return st;
        }
        return GRID_OK;
    }
    const unsigned grid = (unsigned)wgs;
    void* params[] = {&a};   // the kernel takes one argument: the MixedArgs block
    HIP_TRY(hipModuleLaunchKernel(pers ? mx->fn_persistent : mx->fn, grid, 1, 1,
                                  64u * (unsigned)mx->waves, 1, 1, 0, stream, params, nullptr));
    return GRID_OK;
}

// the mode tuned for a launch of `blocks` blocks
int mixed_mode_for(grid_mixed mx, int64_t blocks)
{
    for (const auto& e : mx->tuned)
        if (blocks <= e.first)
            return e.second;
    return mx->tuned.empty() ? GRID_MIXED_ONE_LAUNCH : mx->tuned.back().second;
}

// the launch a mixed graph records: `mode`, or the tuned mode for this many blocks (-1); an
// empty batch records nothing (the graph then has no nodes)
grid_status mixed_capture_launch(grid_mixed mx, const grid_mixed_item* items, int32_t count,
                                 int mode, int64_t blocks, hipStream_t s)
{
    if (blocks == 0)
        return GRID_OK;
    return mixed_launch_mode(mx, items, count, mode >= 0 ? mode : mixed_mode_for(mx, blocks), s);
}

}  // namespace

extern "C" {

grid_status grid_mixed_launch(grid_mixed mx, const grid_mixed_item* items, int32_t count,
                              void* stream)
{
    MixedArgs a;
    int64_t blocks = 0;
    grid_status st = mixed_args(mx, items, count, 0, &a, &blocks);
    if (st != GRID_OK)
        return st;
    if (blocks == 0)
        return GRID_OK;
    return mixed_launch_mode(mx, items, count, mixed_mode_for(mx, blocks), (hipStream_t)stream);
}

grid_status grid_mixed_launch_mode(grid_mixed mx, const grid_mixed_item* items, int32_t count,
                                   int32_t mode, void* stream)
{
    return mixed_launch_mode(mx, items, count, mode, (hipStream_t)stream);
}

grid_status grid_mixed_graph_create(grid_mixed mx, const grid_mixed_item* items, int32_t count,
                                    int32_t mode, grid_graph* out)
{
    if (!out)
        return fail(GRID_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (mode < -1 || mode > GRID_MIXED_PER_ROBOT)
        return fail(GRID_EINVAL, "unknown mixed launch mode " + std::to_string(mode));
    MixedArgs a;
    int64_t blocks = 0;
    grid_status st = mixed_args(mx, items, count, 0, &a, &blocks);
    if (st != GRID_OK)
        return st;
    HIP_TRY(hipSetDevice(mx->device));
    grid_graph g = new (std::nothrow) grid_graph_s;
    if (!g)
        return fail(GRID_ENOMEM, "host allocation failed");
    g->device = mx->device;
    g->count = count;
    g->mx = mx;
    g->mode = mode;
    hipError_t e = hipStreamCreateWithFlags(&g->capture, hipStreamNonBlocking);
    if (e != hipSuccess) {
        destroy_graph(g);
        return fail(GRID_EDEVICE, std::string("graph stream: ") + hipGetErrorString(e));
    }
    st = capture_with(g, [&](hipStream_t s) {
        return mixed_capture_launch(mx, items, count, g->mode, blocks, s);
    }, &g->graph);
    if (st == GRID_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess)
            st = fail(GRID_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    if (st != GRID_OK) {
        destroy_graph(g);
        return st;
    }
    *out = g;
    return GRID_OK;
}

grid_status grid_mixed_graph_update(grid_graph g, const grid_mixed_item* items, int32_t count)
{
    if (!g)
        return fail(GRID_EINVAL, "graph is NULL");
    if (!g->mx)
        return fail(GRID_EINVAL, "not a graph of a mixed launch (grid_graph_update updates it)");
    MixedArgs a;
    int64_t blocks = 0;
    grid_status st = mixed_args(g->mx, items, count, 0, &a, &blocks);
    if (st != GRID_OK)
        return st;
    HIP_TRY(hipSetDevice(g->device));
    hipGraph_t fresh = nullptr;
    st = capture_with(g, [&](hipStream_t s) {
        return mixed_capture_launch(g->mx, items, count, g->mode, blocks, s);
    }, &fresh);
    if (st != GRID_OK)
        return st;
    g->count = count;
    return swap_in(g, fresh);
}

grid_status grid_mixed_tune(grid_mixed mx, const grid_mixed_item* items, int32_t count,
                            int32_t* chosen, float* us)
{
    MixedArgs a;
    int64_t blocks = 0;
    grid_status st = mixed_args(mx, items, count, 0, &a, &blocks);
    if (st != GRID_OK)
        return st;
    if (blocks == 0)
        return fail(GRID_EINVAL, "the items hold no knots");
    HIP_TRY(hipSetDevice(mx->device));
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    auto cleanup = [&]() {
        if (s)
            (void)hipStreamSynchronize(s);
        if (e0)
            (void)hipEventDestroy(e0);
        if (e1)
            (void)hipEventDestroy(e1);
        if (s)
            (void)hipStreamDestroy(s);
    };
    if (e != hipSuccess) {
        cleanup();
        return fail(GRID_EDEVICE, std::string("mixed tuning: ") + hipGetErrorString(e));
    }
    // per-robot mode runs each robot's own build for the item's N: tune every robot's model
    // for the knot counts it has here first, so that the modes are compared at their best
    for (size_t r = 0; r < mx->models.size() && st == GRID_OK; ++r) {
        std::vector<int32_t> Ns;
        for (int j = 0; j < count; ++j)
            if (items[j].robot == (int)r && items[j].N > 0 &&
                std::find(Ns.begin(), Ns.end(), items[j].N) == Ns.end())
                Ns.push_back(items[j].N);
        if (!Ns.empty())
            st = grid_tune(mx->models[r], Ns.data(), (int32_t)Ns.size(), nullptr, nullptr);
    }
    if (st != GRID_OK) {
        cleanup();
        return st;
    }
    int best = GRID_MIXED_ONE_LAUNCH;
    float best_us = 1e30f;
    for (int mode = GRID_MIXED_ONE_LAUNCH; mode <= GRID_MIXED_PER_ROBOT; ++mode) {
        const int reps = 20;
        float times[5];
        for (int trial = 0; trial < 5; ++trial) {
            for (int w = 0; w < 3 && st == GRID_OK; ++w)
                st = mixed_launch_mode(mx, items, count, mode, s);
            e = hipEventRecord(e0, s);
            for (int r = 0; r < reps && st == GRID_OK; ++r)
                st = mixed_launch_mode(mx, items, count, mode, s);
            if (e == hipSuccess)
                e = hipEventRecord(e1, s);
            if (e == hipSuccess)
                e = hipEventSynchronize(e1);
            if (st != GRID_OK || e != hipSuccess) {
                cleanup();
                return st != GRID_OK ? st
                                     : fail(GRID_EDEVICE, std::string("mixed tuning: ") +
                                                              hipGetErrorString(e));
            }
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            times[trial] = 1e3f * ms / reps;
        }
        std::sort(times, times + 5);
        if (us)
            us[mode] = times[2];
        if (times[2] < best_us) {
            best_us = times[2];
            best = mode;
        }
    }
    cleanup();
    bool replaced = false;
    for (auto& t : mx->tuned)
        if (t.first == blocks) {
            t.second = best;
            replaced = true;
        }
    if (!replaced) {
        mx->tuned.emplace_back(blocks, best);
        std::sort(mx->tuned.begin(), mx->tuned.end());
    }
    if (chosen)
        *chosen = best;
    return GRID_OK;
}

grid_status grid_mixed_destroy(grid_mixed mx)
{
    if (!mx)
        return GRID_OK;
    (void)hipSetDevice(mx->device);
    for (grid_model m : mx->models)
        grid_model_destroy(m);
    if (mx->module)
        (void)hipModuleUnload(mx->module);
    delete mx;
    return GRID_OK;
}

grid_status grid_tune(grid_model m, const int32_t* Ns, int32_t count, const char* table_path,
                      int32_t* chosen)
{
    if (!m || !Ns || count < 1 || count > 64)
        return fail(GRID_EINVAL, "model and 1..64 knot counts are required");
    int32_t maxN = 0;
    for (int k = 0; k < count; ++k) {
        if (Ns[k] < 1 || Ns[k] > (1 << 22))
            return fail(GRID_EINVAL, "knot counts must be in 1..2^22");
        maxN = std::max(maxN, Ns[k]);
    }
    HIP_TRY(hipSetDevice(m->device));
    const size_t n = (size_t)m->topo.n;
    float *in = nullptr, *outb = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (s)
            (void)hipStreamSynchronize(s);
        (void)hipFree(in);
        (void)hipFree(outb);
        if (e0)
            (void)hipEventDestroy(e0);
        if (e1)
            (void)hipEventDestroy(e1);
        if (s)
            (void)hipStreamDestroy(s);
    };
    hipError_t e = hipMalloc(&in, (size_t)maxN * 3 * n * sizeof(float));
    if (e == hipSuccess)
        e = hipMalloc(&outb, (size_t)maxN * (n + 3 * n * n) * sizeof(float));
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    if (e == hipSuccess)   // q = qd = tau = 0: a valid state; the timing does not depend on values
        e = hipMemsetAsync(in, 0, (size_t)maxN * 3 * n * sizeof(float), s);
    if (e != hipSuccess) {
        cleanup();
        return fail(GRID_ENOMEM, std::string("tuning buffers: ") + hipGetErrorString(e));
    }
    std::vector<std::pair<int32_t, int>> table;
    for (int k = 0; k < count; ++k) {
        const int32_t N = Ns[k];
        const size_t vec = (size_t)N * n, mat = vec * n;
        float *q = in, *qd = in + vec, *tau = in + 2 * vec;
        float *qdd = outb, *Mi = outb + vec, *dq = Mi + mat, *dqd = dq + mat;
        int best = 0;
        float best_ms = 1e30f;
        for (int v = 0; v < grid_impl::kNumVariants; ++v) {
            if (!m->fused_variant[v])
                continue;   // not built for this model
            const int reps = 30;
            float times[5];
            for (int trial = 0; trial < 5; ++trial) {
                grid_status st = GRID_OK;
                for (int w = 0; w < 3 && st == GRID_OK; ++w)
                    st = grid_impl::launch_fused_variant(m, v, N, q, qd, tau, qdd, Mi, dq, dqd, s);
                e = hipEventRecord(e0, s);
                for (int r = 0; r < reps && st == GRID_OK; ++r)
                    st = grid_impl::launch_fused_variant(m, v, N, q, qd, tau, qdd, Mi, dq, dqd, s);
                if (e == hipSuccess)
                    e = hipEventRecord(e1, s);
                if (e == hipSuccess)
                    e = hipEventSynchronize(e1);
                if (st != GRID_OK || e != hipSuccess) {
                    cleanup();
                    return st != GRID_OK ? st
                                         : fail(GRID_EDEVICE, std::string("tuning: ") +
                                                                  hipGetErrorString(e));
                }
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                times[trial] = ms / reps;
            }
            std::sort(times, times + 5);
            if (times[2] < best_ms) {
                best_ms = times[2];
                best = v;
            }
        }
        table.emplace_back(N, best);
        if (chosen)
            chosen[k] = best;
    }
    cleanup();
    std::sort(table.begin(), table.end());
    m->tuned = table;
    if (table_path) {
        std::ofstream f(table_path, std::ios::app);
        if (!f)
            return fail(GRID_EINVAL, std::string("cannot write ") + table_path);
        f << "{\"arch\": \"gfx950\", \"model\": \"" << std::hex << m->code_hash << std::dec
          << "\", \"buckets\": [";
        for (size_t i = 0; i < table.size(); ++i)
            f << (i ? ", " : "") << "[" << table[i].first << ", " << table[i].second << "]";
        f << "]}\n";
    }
    return GRID_OK;
}

grid_status grid_tune_apply(grid_model m, const int32_t* Ns, const int32_t* builds,
                            int32_t count)
{
    if (!m || count < 0 || count > 64 || (count > 0 && (!Ns || !builds)))
        return fail(GRID_EINVAL, "model and 0..64 (N, build) pairs are required");
    std::vector<std::pair<int32_t, int>> table;
    for (int k = 0; k < count; ++k) {
        if (Ns[k] < 1 || Ns[k] > (1 << 22) || (k > 0 && Ns[k] <= Ns[k - 1]))
            return fail(GRID_EINVAL, "knot counts must ascend within 1..2^22");
        if (builds[k] < 0 || builds[k] >= grid_impl::kNumVariants ||
            !m->fused_variant[builds[k]])
            return fail(GRID_EUNSUPPORTED, "build " + std::to_string(builds[k]) +
                                               " does not exist for this model");
        table.emplace_back(Ns[k], builds[k]);
    }
    m->tuned = table;
    return GRID_OK;
}

grid_status grid_build_for(grid_model m, int32_t N, int32_t* build)
{
    if (!m || N < 1 || !build)
        return fail(GRID_EINVAL, "model, N >= 1 and an output pointer are required");
    *build = grid_impl::fused_variant_for(m, N);
    return GRID_OK;
}

}  // extern "C"

namespace grid_impl {

// Apply the last line of $GRID_TUNE_TABLE whose model hash matches this model's code objects
// (a table tuned on other machine code is not applied).
void load_tuning(grid_model m)
{
    const char* path = std::getenv("GRID_TUNE_TABLE");
    if (!path || !*path)
        return;
    std::ifstream f(path);
    if (!f)
        return;
    char key[32];
    std::snprintf(key, sizeof key, "\"model\": \"%llx\"", (unsigned long long)m->code_hash);
    std::string line, last;
    while (std::getline(f, line))
        if (line.find(key) != std::string::npos)
            last = line;
    if (last.empty())
        return;
    std::vector<std::pair<int32_t, int>> table;
    size_t p = last.find("\"buckets\": [");
    if (p == std::string::npos)
        return;
    p += 12;
    while (true) {
        p = last.find('[', p);
        if (p == std::string::npos)
            break;
        long Nk = 0, v = 0;
        if (std::sscanf(last.c_str() + p, "[%ld, %ld]", &Nk, &v) != 2 || v < 0 ||
            v >= kNumVariants || !m->fused_variant[v])
            break;
        table.emplace_back((int32_t)Nk, (int)v);
        ++p;
    }
    std::sort(table.begin(), table.end());
    m->tuned = table;
}

}  // namespace grid_impl
