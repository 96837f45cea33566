// Continuous-batching dFD server and its open-loop load generator (include/grid.h).
//
// Threads:
//   clients   grid_server_submit queues a request and wakes the scheduler; grid_server_wait
//             sleeps on a condition variable until the request is final;
//   scheduler admits pending requests while the in-flight bytes fit the budget, packs
//             admitted requests of one model into a free batch context (pinned staging,
//             device buffers, its own stream) under the batching policy, and enqueues H2D
//             copy, one launch and D2H copy with events around each phase; it sleeps until a
//             request arrives, a context frees up or a batch window closes;
//   workers   one per context: waits for its batch on the device (polling the last event for
//             a short while, then a blocking wait), copies the outputs from pinned staging into
//             the requests' host buffers, publishes them and frees the context and its
//             admission bytes.
#include "grid_internal.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <random>
#include <thread>
#include <unordered_map>

using namespace grid_impl;

namespace {

using Clock = std::chrono::steady_clock;

enum ReqState : int { kQueued = 0, kLaunched = 1, kDone = 2, kCanceled = 3 };

// how long a worker polls its batch's last event before it blocks on it
constexpr auto kPollBeforeBlock = std::chrono::microseconds(60);

struct Request {
    uint64_t ticket = 0;
    int model = 0;
    int N = 0;
    const float *q = nullptr, *qd = nullptr, *tau = nullptr;
    float *qdd = nullptr, *Minv = nullptr, *dq = nullptr, *dqd = nullptr;
    size_t bytes = 0;
    // with GRID_SERVER_DIRECT_PINNED: the seven arrays as the device sees them, when all of them
    // lie inside pinned host allocations mapped into the device (else direct = false)
    bool direct = false;
    float* dev[7] = {};
    std::atomic<int> state{kQueued};
    // timeline (host clock) and the device phases of its batch (ms)
    Clock::time_point t_admit, t_launch, t_seen, t_done;
    float h2d_ms = 0, kernel_ms = 0, d2h_ms = 0;
};

struct BatchCtx {
    int model = 0;
    int n = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev[4] = {};                     // before H2D, after H2D, after kernel, after D2H
    float *d_in = nullptr, *d_out = nullptr, *h_in = nullptr, *h_out = nullptr;
    float *h_in_dev = nullptr, *h_out_dev = nullptr;   // device mapping (mapped I/O)
    grid_workspace ws = nullptr;               // staged (per-request) mode only
    std::vector<Request*> reqs;
    int knots = 0;
    bool inplace = false;                      // this batch runs on its request's own arrays
    bool mapped = false;                       // and without copy-engine phases
    std::atomic<bool> busy{false};             // set by the scheduler, cleared by its worker
    std::thread worker;
    std::mutex mu;                             // launched, quit
    std::condition_variable cv;
    bool launched = false, quit = false;
};

size_t request_bytes(int n, int N) { return sizeof(float) * (size_t)N * (4 * n + 3 * n * n); }

// Host array for the load generator: ordinary memory, or pinned and mapped into the device.
struct HostArray {
    float* ptr = nullptr;
    size_t len = 0;
    bool pinned = false;
    HostArray() = default;
    HostArray(const HostArray&) = delete;
    HostArray& operator=(const HostArray&) = delete;
    ~HostArray()
    {
        if (pinned)
            (void)hipHostFree(ptr);
        else
            delete[] ptr;
    }
    bool alloc(size_t n, bool pin)
    {
        len = n;
        pinned = pin;
        if (pin) {
            void* p = nullptr;
            if (hipHostMalloc(&p, n * sizeof(float), hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                pinned = false;
                return false;
            }
            ptr = static_cast<float*>(p);
        } else {
            ptr = new (std::nothrow) float[n]();
        }
        return ptr != nullptr;
    }
    float* data() { return ptr; }
    size_t size() const { return len; }
    float& operator[](size_t i) { return ptr[i]; }
};

// The device address of host array [p, p + bytes) when the whole range lies inside one pinned
// host allocation mapped into the device; NULL otherwise (pageable memory, a range that runs
// past its allocation, or a failed query).
float* mapped_range(const void* p, size_t bytes)
{
    hipDeviceptr_t start = nullptr;
    size_t size = 0;
    hipPointerAttribute_t at{};
    const hipDeviceptr_t hp = const_cast<void*>(p);
    if (hipPointerGetAttribute(&start, HIP_POINTER_ATTRIBUTE_RANGE_START_ADDR, hp) != hipSuccess ||
        hipPointerGetAttribute(&size, HIP_POINTER_ATTRIBUTE_RANGE_SIZE, hp) != hipSuccess ||
        hipPointerGetAttributes(&at, start) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    const char* s0 = static_cast<const char*>(start);
    const char* c = static_cast<const char*>(p);
    if (at.type != hipMemoryTypeHost || !at.devicePointer || c < s0 ||
        (size_t)(c - s0) + bytes > size)
        return nullptr;
    return reinterpret_cast<float*>(static_cast<char*>(at.devicePointer) + (c - s0));
}

}  // namespace

struct grid_server_s {
    std::vector<grid_model> models;
    grid_server_config cfg{};
    int device = 0;
    std::vector<std::unique_ptr<BatchCtx>> ctx;

    std::mutex mu;                             // everything below up to `stop`
    std::condition_variable sched_cv;          // a request arrived, a context freed, stop
    std::condition_variable done_cv;           // a request reached a final state
    std::deque<Request*> pending;
    std::unordered_map<uint64_t, Request*> tickets;
    uint64_t next_ticket = 1;
    uint64_t wake_seq = 0;                     // bumped with every scheduler wake-up
    bool accepting = true;
    bool stop = false;                         // scheduler: drain and exit

    std::atomic<size_t> inflight_bytes{0};
    std::thread scheduler;

    std::atomic<uint64_t> submitted{0}, completed_n{0}, canceled{0}, knots_done{0}, launches{0};
    std::atomic<uint64_t> max_inflight{0}, inplace_launches{0};
    std::atomic<bool> device_error{false};

    // pinned host ranges the caller registered for in-place requests: host start, length,
    // the device's address of the start
    struct PinRange {
        const char* start;
        size_t len;
        char* dev;
    };
    std::mutex pin_mu;
    std::vector<PinRange> pins;
};

namespace {

grid_status fail(grid_status s, const std::string& msg)
{
    set_error(msg);
    return s;
}

void wake_scheduler(grid_server s)
{
    {
        std::lock_guard<std::mutex> lk(s->mu);
        ++s->wake_seq;
    }
    s->sched_cv.notify_one();
}

// Return a context and its requests' admission bytes. Requests are published (done or
// canceled) only after the context no longer refers to them: a waiter may free a
// request as soon as it sees the final state.
void finish_ctx(grid_server s, BatchCtx* c, int final_state)
{
    std::vector<Request*> reqs;
    reqs.swap(c->reqs);
    size_t freed = 0;
    for (Request* r : reqs)
        freed += r->bytes;
    c->knots = 0;
    s->inflight_bytes.fetch_sub(freed);
    c->busy.store(false, std::memory_order_release);
    for (Request* r : reqs) {
        if (final_state == kCanceled)
            s->canceled.fetch_add(1);
        r->state.store(final_state, std::memory_order_release);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);   // orders the stores before any waiter's check
        ++s->wake_seq;
    }
    s->done_cv.notify_all();
    s->sched_cv.notify_one();
}

// wait for the batch's last event: poll for a short while (most batches finish within tens of
// microseconds), then block in the runtime
hipError_t wait_batch(BatchCtx* c)
{
    const auto t0 = Clock::now();
    for (;;) {
        const hipError_t q = hipEventQuery(c->ev[3]);
        if (q != hipErrorNotReady)
            return q;
        if (Clock::now() - t0 > kPollBeforeBlock)
            return hipEventSynchronize(c->ev[3]);
        std::this_thread::yield();
    }
}

void worker_loop(grid_server s, BatchCtx* c)
{
    (void)hipSetDevice(s->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(c->mu);
            c->cv.wait(lk, [&] { return c->launched || c->quit; });
            if (!c->launched)
                return;
            c->launched = false;
        }
        const hipError_t e = wait_batch(c);
        const auto t_seen = Clock::now();
        float ph[3] = {0, 0, 0};
        if (e != hipSuccess) {
            s->device_error.store(true);
        } else if (c->mapped) {
            (void)hipEventElapsedTime(&ph[1], c->ev[0], c->ev[3]);   // the kernel alone
        } else {
            for (int k = 0; k < 3; ++k)
                (void)hipEventElapsedTime(&ph[k], c->ev[k], c->ev[k + 1]);
        }
        const size_t n = (size_t)c->n, K = (size_t)c->knots;
        const float* oq = c->h_out;
        const float* oM = oq + K * n;
        const float* oD = oM + K * n * n;
        const float* oV = oD + K * n * n;
        size_t off = 0;
        for (Request* r : c->reqs) {
            const size_t N = (size_t)r->N;
            r->t_seen = t_seen;
            r->h2d_ms = ph[0];
            r->kernel_ms = ph[1];
            r->d2h_ms = ph[2];
            if (!c->inplace) {                 // in place, the kernel wrote the caller's arrays
                std::memcpy(r->qdd, oq + off * n, N * n * sizeof(float));
                std::memcpy(r->Minv, oM + off * n * n, N * n * n * sizeof(float));
                std::memcpy(r->dq, oD + off * n * n, N * n * n * sizeof(float));
                std::memcpy(r->dqd, oV + off * n * n, N * n * n * sizeof(float));
            }
            off += N;
            r->t_done = Clock::now();
            s->knots_done.fetch_add(N);
            s->completed_n.fetch_add(1);
        }
        finish_ctx(s, c, kDone);
    }
}

bool ctx_busy(BatchCtx* c) { return c->busy.load(std::memory_order_acquire); }

// stage inputs, enqueue copy-in, launch, copy-out and the events around them
bool launch_ctx(grid_server s, BatchCtx* c)
{
    grid_model m = s->models[c->model];
    const size_t n = (size_t)c->n, K = (size_t)c->knots;
    float* iq = c->h_in;
    float* iqd = iq + K * n;
    float* itau = iqd + K * n;
    size_t off = 0;
    const auto now = Clock::now();
    c->inplace = c->reqs.size() == 1 && c->reqs[0]->direct;
    for (Request* r : c->reqs) {
        const size_t N = (size_t)r->N;
        if (!c->inplace) {
            std::memcpy(iq + off * n, r->q, N * n * sizeof(float));
            std::memcpy(iqd + off * n, r->qd, N * n * sizeof(float));
            std::memcpy(itau + off * n, r->tau, N * n * sizeof(float));
        }
        r->t_launch = now;
        r->state.store(kLaunched, std::memory_order_relaxed);
        off += N;
    }
    // mapped I/O: the kernel reads the pinned inputs and writes the pinned outputs through the
    // device's mapping (no copy-engine transfers; no H2D and D2H phases, and no events for
    // them: an event record costs a few microseconds of the stream's time). In place: a batch
    // of one request whose arrays are all pinned and mapped runs on them directly.
    const bool mapped = c->inplace || (s->cfg.flags & GRID_SERVER_MAPPED_IO) != 0;
    c->mapped = mapped;
    float* const* rd = c->reqs[0]->dev;
    float* dq = c->inplace ? rd[0] : mapped ? c->h_in_dev : c->d_in;
    float* dqd = c->inplace ? rd[1] : dq + K * n;
    float* dtau = c->inplace ? rd[2] : dqd + K * n;
    float* oq = c->inplace ? rd[3] : mapped ? c->h_out_dev : c->d_out;
    float* oM = c->inplace ? rd[4] : oq + K * n;
    float* oD = c->inplace ? rd[5] : oM + K * n * n;
    float* oV = c->inplace ? rd[6] : oD + K * n * n;
    if (hipEventRecord(c->ev[0], c->stream) != hipSuccess ||
        (!mapped && (hipMemcpyAsync(dq, iq, 3 * K * n * sizeof(float), hipMemcpyHostToDevice,
                                    c->stream) != hipSuccess ||
                     hipEventRecord(c->ev[1], c->stream) != hipSuccess)))
        return false;
    grid_status st;
    if (s->cfg.flags & GRID_SERVER_PER_REQUEST)
        st = grid_fd_grad_staged(m, c->ws, (int32_t)K, dq, dqd, dtau, oq, oM, oD, oV, c->stream);
    else
        st = grid_fd_grad(m, (int32_t)K, dq, dqd, dtau, oq, oM, oD, oV, c->stream);
    if (st != GRID_OK)
        return false;
    if ((!mapped && (hipEventRecord(c->ev[2], c->stream) != hipSuccess ||
                     hipMemcpyAsync(c->h_out, c->d_out, K * (n + 3 * n * n) * sizeof(float),
                                    hipMemcpyDeviceToHost, c->stream) != hipSuccess)) ||
        hipEventRecord(c->ev[3], c->stream) != hipSuccess)
        return false;
    s->launches.fetch_add(1);
    if (c->inplace)
        s->inplace_launches.fetch_add(1);
    {
        std::lock_guard<std::mutex> lk(c->mu);
        c->launched = true;
    }
    c->cv.notify_one();
    return true;
}

void scheduler_loop(grid_server s)
{
    (void)hipSetDevice(s->device);
    const int nm = (int)s->models.size();
    const bool per_request = (s->cfg.flags & GRID_SERVER_PER_REQUEST) != 0;
    const auto window = std::chrono::microseconds(per_request ? 0 : s->cfg.batch_window_us);
    const int min_fill = per_request ? 0 : s->cfg.min_batch_knots;
    std::vector<std::deque<Request*>> admitted(nm);
    std::vector<int> admitted_knots(nm, 0);
    uint64_t seen = 0;
    for (;;) {
        bool stopping = false;
        // admission: FIFO while the bytes fit
        {
            std::lock_guard<std::mutex> lk(s->mu);
            seen = s->wake_seq;
            stopping = s->stop;
            const auto now = Clock::now();
            while (!s->pending.empty()) {
                Request* r = s->pending.front();
                const size_t cur = s->inflight_bytes.load();
                if (cur + r->bytes > s->cfg.device_budget_bytes)
                    break;
                s->inflight_bytes.fetch_add(r->bytes);
                size_t now_b = cur + r->bytes, top = s->max_inflight.load();
                while (now_b > top && !s->max_inflight.compare_exchange_weak(top, now_b)) {
                }
                s->pending.pop_front();
                r->t_admit = now;
                admitted[r->model].push_back(r);
                admitted_knots[r->model] += r->N;
            }
        }
        // packing under the batching policy
        Clock::time_point deadline = Clock::time_point::max();
        for (int k = 0; k < nm; ++k) {
            auto& q = admitted[k];
            while (!q.empty()) {
                BatchCtx* free_ctx = nullptr;
                int busy = 0;
                for (auto& cp : s->ctx) {
                    if (cp->model != k)
                        continue;
                    if (ctx_busy(cp.get()))
                        ++busy;
                    else if (!free_ctx)
                        free_ctx = cp.get();
                }
                if (!free_ctx)
                    break;
                if (busy > 0 && !stopping && admitted_knots[k] < min_fill) {
                    const auto due = q.front()->t_admit + window;
                    if (Clock::now() < due) {
                        deadline = std::min(deadline, due);
                        break;
                    }
                }
                BatchCtx* c = free_ctx;
                int knots = 0;
                while (!q.empty()) {
                    Request* r = q.front();
                    if (knots > 0 && (per_request || knots + r->N > s->cfg.max_batch_knots))
                        break;
                    c->reqs.push_back(r);
                    knots += r->N;
                    q.pop_front();
                }
                admitted_knots[k] -= knots;
                c->knots = knots;
                c->busy.store(true, std::memory_order_release);
                if (!launch_ctx(s, c)) {
                    s->device_error.store(true);
                    (void)hipStreamSynchronize(c->stream);
                    finish_ctx(s, c, kCanceled);
                }
            }
        }
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop) {
            bool idle = true;
            for (auto& q : admitted)
                idle = idle && q.empty();
            for (auto& cp : s->ctx)
                idle = idle && !ctx_busy(cp.get());
            if (idle && s->pending.empty())
                break;
        }
        // sleep until a request arrives, a context frees up or a batch window closes
        auto woken = [&] { return s->wake_seq != seen; };
        if (deadline == Clock::time_point::max())
            s->sched_cv.wait(lk, woken);
        else
            s->sched_cv.wait_until(lk, deadline, woken);
    }
}

void destroy_ctx(BatchCtx* c)
{
    if (c->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(c->mu);
            c->quit = true;
        }
        c->cv.notify_one();
        c->worker.join();
    }
    if (c->stream)
        (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t e : c->ev)
        if (e)
            (void)hipEventDestroy(e);
    if (c->stream)
        (void)hipStreamDestroy(c->stream);
    (void)hipFree(c->d_in);
    (void)hipFree(c->d_out);
    if (c->h_in)
        (void)hipHostFree(c->h_in);
    if (c->h_out)
        (void)hipHostFree(c->h_out);
    if (c->ws)
        grid_workspace_destroy(c->ws);
}

}  // namespace

extern "C" {

grid_status grid_server_create(const grid_model* models, int32_t count,
                               const grid_server_config* cfg, grid_server* out)
{
    if (!out)
        return fail(GRID_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!models || count < 1 || !cfg)
        return fail(GRID_EINVAL, "models, count and config are required");
    if (cfg->max_batch_knots < 1 || cfg->max_batch_knots > (1 << 20) || cfg->contexts_per_model < 1 ||
        cfg->contexts_per_model > 64 ||
        (cfg->flags & ~(uint32_t)(GRID_SERVER_PER_REQUEST | GRID_SERVER_MAPPED_IO |
                                  GRID_SERVER_DIRECT_PINNED)) ||
        cfg->batch_window_us < 0 || cfg->batch_window_us > 1000000 || cfg->min_batch_knots < 0 ||
        cfg->min_batch_knots > cfg->max_batch_knots)
        return fail(GRID_EINVAL, "bad server configuration");
    for (int k = 0; k < count; ++k)
        if (!models[k] || models[k]->device != models[0]->device)
            return fail(GRID_EINVAL, "models must be non-NULL and on one device");
    grid_server s = new (std::nothrow) grid_server_s;
    if (!s)
        return fail(GRID_ENOMEM, "host allocation failed");
    s->models.assign(models, models + count);
    s->cfg = *cfg;
    s->device = models[0]->device;
    if (hipSetDevice(s->device) != hipSuccess) {
        delete s;
        return fail(GRID_EDEVICE, "hipSetDevice failed");
    }
    for (int k = 0; k < count; ++k)
        for (int c = 0; c < cfg->contexts_per_model; ++c) {
            auto b = std::make_unique<BatchCtx>();
            b->model = k;
            b->n = models[k]->topo.n;
            const size_t n = (size_t)b->n, K = (size_t)cfg->max_batch_knots;
            hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
            for (int v = 0; v < 4 && e == hipSuccess; ++v)   // the last one is waited on
                e = hipEventCreateWithFlags(&b->ev[v], v == 3 ? hipEventBlockingSync
                                                              : hipEventDefault);
            if (e == hipSuccess)
                e = hipMalloc(&b->d_in, 3 * K * n * sizeof(float));
            if (e == hipSuccess)
                e = hipMalloc(&b->d_out, K * (n + 3 * n * n) * sizeof(float));
            if (e == hipSuccess)
                e = hipHostMalloc(&b->h_in, 3 * K * n * sizeof(float), hipHostMallocDefault);
            if (e == hipSuccess)
                e = hipHostMalloc(&b->h_out, K * (n + 3 * n * n) * sizeof(float), hipHostMallocDefault);
            if (e == hipSuccess && (cfg->flags & GRID_SERVER_MAPPED_IO)) {
                void* pi = nullptr;
                void* po = nullptr;
                e = hipHostGetDevicePointer(&pi, b->h_in, 0);
                if (e == hipSuccess)
                    e = hipHostGetDevicePointer(&po, b->h_out, 0);
                b->h_in_dev = static_cast<float*>(pi);
                b->h_out_dev = static_cast<float*>(po);
            }
            grid_status st = GRID_OK;
            if (e == hipSuccess && (cfg->flags & GRID_SERVER_PER_REQUEST))
                st = grid_workspace_create(models[k], cfg->max_batch_knots, &b->ws);
            s->ctx.push_back(std::move(b));
            if (e != hipSuccess || st != GRID_OK) {
                for (auto& cp : s->ctx)
                    destroy_ctx(cp.get());
                delete s;
                return fail(GRID_ENOMEM, "server buffer allocation failed");
            }
        }
    for (auto& cp : s->ctx)
        cp->worker = std::thread(worker_loop, s, cp.get());
    s->scheduler = std::thread(scheduler_loop, s);
    *out = s;
    return GRID_OK;
}

grid_status grid_server_submit(grid_server s, int32_t model_index, int32_t N, const float* q,
                               const float* qd, const float* tau, float* qdd, float* Minv,
                               float* dqdd_dq, float* dqdd_dqd, uint64_t* ticket)
{
    if (!s || !ticket)
        return fail(GRID_EINVAL, "server and ticket must not be NULL");
    if (model_index < 0 || model_index >= (int32_t)s->models.size())
        return fail(GRID_EINVAL, "model index out of range");
    if (N < 1 || N > s->cfg.max_batch_knots)
        return fail(GRID_EINVAL, "N must be in 1..max_batch_knots");
    if (!q || !qd || !tau || !qdd || !Minv || !dqdd_dq || !dqdd_dqd)
        return fail(GRID_EINVAL, "a data pointer is NULL");
    const size_t bytes = request_bytes(s->models[model_index]->topo.n, N);
    if (bytes > s->cfg.device_budget_bytes)
        return fail(GRID_EBUSY, "request exceeds the admission budget");
    Request* r = new (std::nothrow) Request;
    if (!r)
        return fail(GRID_ENOMEM, "host allocation failed");
    r->model = model_index;
    r->N = N;
    r->q = q;
    r->qd = qd;
    r->tau = tau;
    r->qdd = qdd;
    r->Minv = Minv;
    r->dq = dqdd_dq;
    r->dqd = dqdd_dqd;
    r->bytes = bytes;
    if (s->cfg.flags & GRID_SERVER_DIRECT_PINNED) {
        // every array inside a registered pinned range: the request can run in place
        const size_t n = (size_t)s->models[model_index]->topo.n, v = N * n * sizeof(float);
        const void* a[7] = {q, qd, tau, qdd, Minv, dqdd_dq, dqdd_dqd};
        const size_t len[7] = {v, v, v, v, v * n, v * n, v * n};
        std::lock_guard<std::mutex> lk(s->pin_mu);
        r->direct = !s->pins.empty();
        for (int k = 0; k < 7 && r->direct; ++k) {
            const char* c = static_cast<const char*>(a[k]);
            r->dev[k] = nullptr;
            for (const auto& pr : s->pins)
                if (c >= pr.start && (size_t)(c - pr.start) + len[k] <= pr.len) {
                    r->dev[k] = reinterpret_cast<float*>(pr.dev + (c - pr.start));
                    break;
                }
            r->direct = r->dev[k] != nullptr;
        }
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->accepting) {
            delete r;
            return fail(GRID_ECANCELED, "server is shutting down");
        }
        r->ticket = s->next_ticket++;
        s->tickets[r->ticket] = r;
        s->pending.push_back(r);
        ++s->wake_seq;
    }
    s->sched_cv.notify_one();
    s->submitted.fetch_add(1);
    *ticket = r->ticket;
    return GRID_OK;
}

grid_status grid_server_pin_range(grid_server s, const void* p, size_t bytes)
{
    if (!s || !p || bytes == 0)
        return fail(GRID_EINVAL, "server, pointer and a nonzero length are required");
    float* dev = mapped_range(p, bytes);
    if (!dev)
        return fail(GRID_EINVAL, "the range is not inside one pinned host allocation mapped "
                                 "into the device");
    std::lock_guard<std::mutex> lk(s->pin_mu);
    if (s->pins.size() >= 64)
        return fail(GRID_EINVAL, "at most 64 pinned ranges per server");
    s->pins.push_back({static_cast<const char*>(p), bytes, reinterpret_cast<char*>(dev)});
    return GRID_OK;
}

grid_status grid_server_unpin_range(grid_server s, const void* p)
{
    if (!s || !p)
        return fail(GRID_EINVAL, "server and pointer are required");
    std::lock_guard<std::mutex> lk(s->pin_mu);
    for (size_t k = 0; k < s->pins.size(); ++k)
        if (s->pins[k].start == static_cast<const char*>(p)) {
            s->pins.erase(s->pins.begin() + (long)k);
            return GRID_OK;
        }
    return fail(GRID_EINVAL, "no registered range starts at this pointer");
}

static Request* find_request(grid_server s, uint64_t ticket)
{
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    return it == s->tickets.end() ? nullptr : it->second;
}

static void drop_ticket(grid_server s, Request* r)
{
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->tickets.erase(r->ticket);
    }
    delete r;
}

// sleep until the request is final or the timeout passes (timeout_us < 0: no limit); true if
// final
static bool wait_final(grid_server s, Request* r, int64_t timeout_us)
{
    auto final_ = [&] { return r->state.load(std::memory_order_acquire) >= kDone; };
    std::unique_lock<std::mutex> lk(s->mu);
    if (timeout_us < 0) {
        s->done_cv.wait(lk, final_);
        return true;
    }
    return s->done_cv.wait_for(lk, std::chrono::microseconds(timeout_us), final_);
}

grid_status grid_server_wait(grid_server s, uint64_t ticket, int64_t timeout_us)
{
    if (!s)
        return fail(GRID_EINVAL, "server is NULL");
    Request* r = find_request(s, ticket);
    if (!r)
        return fail(GRID_EINVAL, "unknown ticket");
    if (!wait_final(s, r, timeout_us))
        return fail(GRID_ETIMEDOUT, "request still running");
    const int st = r->state.load(std::memory_order_acquire);
    drop_ticket(s, r);
    if (st == kCanceled)
        return fail(GRID_ECANCELED, "request canceled");
    if (s->device_error.load())
        return fail(GRID_EDEVICE, "a device operation of the server failed");
    return GRID_OK;
}

grid_status grid_server_stats_get(grid_server s, grid_server_stats* out)
{
    if (!s || !out)
        return fail(GRID_EINVAL, "server and out must not be NULL");
    out->submitted = s->submitted.load();
    out->completed = s->completed_n.load();
    out->canceled = s->canceled.load();
    out->knots_completed = s->knots_done.load();
    out->launches = s->launches.load();
    out->max_inflight_bytes = s->max_inflight.load();
    out->inplace_launches = s->inplace_launches.load();
    return GRID_OK;
}

grid_status grid_server_destroy(grid_server s)
{
    if (!s)
        return GRID_OK;
    std::deque<Request*> dropped;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->accepting = false;
        dropped.swap(s->pending);
    }
    for (Request* r : dropped) {
        s->canceled.fetch_add(1);
        r->state.store(kCanceled, std::memory_order_release);   // the waiter frees it
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        ++s->wake_seq;
    }
    s->done_cv.notify_all();
    s->sched_cv.notify_one();
    // the scheduler launches what it admitted and returns once every context is free
    if (s->scheduler.joinable())
        s->scheduler.join();
    for (auto& c : s->ctx)
        destroy_ctx(c.get());
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto& kv : s->tickets)
            delete kv.second;
        s->tickets.clear();
    }
    delete s;
    return GRID_OK;
}

grid_status grid_server_loadgen(grid_server s, const grid_loadgen_config* cfg,
                                grid_loadgen_result* out)
{
    if (!s || !cfg || !out || !cfg->model_prob)
        return fail(GRID_EINVAL, "server, config, model_prob and out are required");
    if (!(cfg->rate_per_s > 0) || !(cfg->duration_s > 0) || cfg->warmup_s < 0 || cfg->n_min < 1 ||
        cfg->n_max < cfg->n_min || cfg->n_max > s->cfg.max_batch_knots)
        return fail(GRID_EINVAL, "bad load generator configuration");
    const int nm = (int)s->models.size();
    std::vector<double> cdf(nm);
    double acc = 0;
    for (int k = 0; k < nm; ++k) {
        acc += cfg->model_prob[k];
        cdf[k] = acc;
    }
    if (std::fabs(acc - 1.0) > 1e-6)
        return fail(GRID_EINVAL, "model probabilities must sum to 1");
    std::memset(out, 0, sizeof *out);
    std::mt19937_64 rng(cfg->seed);
    std::uniform_real_distribution<double> uni(0.0, 1.0);
    std::normal_distribution<float> gauss(0.0f, 1.0f);
    // input pools and output rings per model: ordinary host memory, or pinned host memory
    // mapped into the device (cfg->pinned: the clients' arrays then qualify for in-place
    // batches on a GRID_SERVER_DIRECT_PINNED server; a smaller ring keeps the pinned total
    // modest)
    const int pool_knots = 8192, ring = cfg->pinned ? 64 : 256;
    struct Pool {
        int n;
        HostArray q, qd, tau;
        HostArray qdd, M, D, V;                // ring of output slots
    };
    std::vector<Pool> pools(nm);
    for (int k = 0; k < nm; ++k) {
        Pool& p = pools[k];
        p.n = s->models[k]->topo.n;
        const size_t n = (size_t)p.n, slot = (size_t)cfg->n_max;
        const bool pin = cfg->pinned != 0;
        if (!p.q.alloc(pool_knots * n, pin) || !p.qd.alloc(pool_knots * n, pin) ||
            !p.tau.alloc(pool_knots * n, pin) || !p.qdd.alloc(ring * slot * n, pin) ||
            !p.M.alloc(ring * slot * n * n, pin) || !p.D.alloc(ring * slot * n * n, pin) ||
            !p.V.alloc(ring * slot * n * n, pin))
            return fail(GRID_ENOMEM, "load generator buffers");
        for (size_t i = 0; i < p.q.size(); ++i) {
            p.q[i] = (float)(M_PI * (2.0 * uni(rng) - 1.0));
            p.qd[i] = gauss(rng);
            p.tau[i] = 5.0f * gauss(rng);
        }
    }
    // pinned client arrays are registered with the server for the run (in-place requests on a
    // GRID_SERVER_DIRECT_PINNED server) and unregistered on every way out
    std::vector<const void*> pinned_ranges;
    struct Unpin {
        grid_server s;
        std::vector<const void*>* r;
        ~Unpin()
        {
            for (const void* p : *r)
                (void)grid_server_unpin_range(s, p);
        }
    } unpin{s, &pinned_ranges};
    if (cfg->pinned && (s->cfg.flags & GRID_SERVER_DIRECT_PINNED)) {
        for (Pool& p : pools)
            for (HostArray* a : {&p.q, &p.qd, &p.tau, &p.qdd, &p.M, &p.D, &p.V}) {
                const grid_status st = grid_server_pin_range(s, a->data(), a->size() * sizeof(float));
                if (st != GRID_OK)
                    return st;
                pinned_ranges.push_back(a->data());
            }
    }
    struct Sent {
        uint64_t ticket;
        Clock::time_point t_sched;
        int model, N, slot;
        bool counted;
    };
    std::vector<Sent> sent;
    sent.reserve((size_t)(cfg->rate_per_s * (cfg->duration_s + cfg->warmup_s) * 1.2) + 16);
    std::vector<std::vector<int64_t>> slot_owner(nm, std::vector<int64_t>(ring, -1));
    std::vector<int> next_slot(nm, 0);
    std::exponential_distribution<double> gap(cfg->rate_per_s);
    const auto start = Clock::now();
    const double total_s = cfg->warmup_s + cfg->duration_s;
    double t_arr = 0.0;
    std::vector<double> lat;
    std::vector<std::vector<double>> lat_model(std::min(nm, GRID_LOADGEN_MODELS));
    std::vector<double> split[6];   // queue, h2d, kernel, d2h, complete, copyout (us)
    uint64_t knots = 0;
    const uint64_t launches0 = s->launches.load();
    auto us = [](Clock::time_point a, Clock::time_point b) {
        return std::chrono::duration<double, std::micro>(b - a).count();
    };
    auto settle = [&](size_t idx) -> grid_status {
        Sent& e = sent[idx];
        // the request's timeline is read once it is final and before wait releases it
        Request* r = find_request(s, e.ticket);
        if (r && wait_final(s, r, -1) && e.counted &&
            r->state.load(std::memory_order_acquire) == kDone) {
            lat.push_back(us(e.t_sched, r->t_done));
            if (e.model < GRID_LOADGEN_MODELS)
                lat_model[e.model].push_back(lat.back());
            split[0].push_back(us(e.t_sched, r->t_launch));
            split[1].push_back(1e3 * r->h2d_ms);
            split[2].push_back(1e3 * r->kernel_ms);
            split[3].push_back(1e3 * r->d2h_ms);
            split[4].push_back(us(r->t_launch, r->t_seen));
            split[5].push_back(us(r->t_seen, r->t_done));
            knots += (uint64_t)e.N;
        }
        return grid_server_wait(s, e.ticket, -1);
    };
    size_t settled = 0;
    for (;;) {
        t_arr += gap(rng);
        if (t_arr >= total_s)
            break;
        const auto t_sched = start + std::chrono::duration_cast<Clock::duration>(
                                         std::chrono::duration<double>(t_arr));
        const double u = uni(rng);
        int k = 0;
        while (k < nm - 1 && u > cdf[k])
            ++k;
        const int N = cfg->n_min + (int)(uni(rng) * (cfg->n_max - cfg->n_min + 1));
        const int Nc = std::min(N, cfg->n_max);
        Pool& p = pools[k];
        const size_t n = (size_t)p.n;
        const int o = (int)(uni(rng) * (pool_knots - Nc));
        // an output slot no in-flight request of this model still owns
        const int slot = next_slot[k];
        next_slot[k] = (slot + 1) % ring;
        if (slot_owner[k][slot] >= 0) {
            const size_t owner = (size_t)slot_owner[k][slot];
            while (settled <= owner) {
                grid_status st = settle(settled);
                if (st != GRID_OK)
                    return st;
                ++settled;
            }
        }
        // sleep through most of the gap, then spin to the scheduled instant
        if (t_sched - Clock::now() > std::chrono::microseconds(200))
            std::this_thread::sleep_until(t_sched - std::chrono::microseconds(100));
        while (Clock::now() < t_sched) {
        }
        uint64_t ticket = 0;
        const size_t so = (size_t)slot * cfg->n_max;
        grid_status st = grid_server_submit(
            s, k, Nc, p.q.data() + o * n, p.qd.data() + o * n, p.tau.data() + o * n,
            p.qdd.data() + so * n, p.M.data() + so * n * n, p.D.data() + so * n * n,
            p.V.data() + so * n * n, &ticket);
        if (st != GRID_OK)
            return st;
        slot_owner[k][slot] = (int64_t)sent.size();
        sent.push_back(Sent{ticket, t_sched, k, Nc, slot, t_arr >= cfg->warmup_s});
    }
    while (settled < sent.size()) {
        grid_status st = settle(settled);
        if (st != GRID_OK)
            return st;
        ++settled;
    }
    const uint64_t nlaunch = s->launches.load() - launches0;
    std::sort(lat.begin(), lat.end());
    auto pct_of = [](const std::vector<double>& v, double p) {
        if (v.empty())
            return 0.0;
        const size_t i = std::min(v.size() - 1, (size_t)std::floor(p * (v.size() - 1) + 0.5));
        return v[i];
    };
    auto pct = [&](double p) { return pct_of(lat, p); };
    double* p50f[6] = {&out->p50.queue_us, &out->p50.h2d_us, &out->p50.kernel_us,
                       &out->p50.d2h_us, &out->p50.complete_us, &out->p50.copyout_us};
    double* p99f[6] = {&out->p99.queue_us, &out->p99.h2d_us, &out->p99.kernel_us,
                       &out->p99.d2h_us, &out->p99.complete_us, &out->p99.copyout_us};
    for (int k = 0; k < 6; ++k) {
        std::sort(split[k].begin(), split[k].end());
        *p50f[k] = pct_of(split[k], 0.50);
        *p99f[k] = pct_of(split[k], 0.99);
    }
    out->requests_per_launch = nlaunch ? (double)sent.size() / (double)nlaunch : 0.0;
    for (size_t k = 0; k < lat_model.size(); ++k) {
        std::sort(lat_model[k].begin(), lat_model[k].end());
        out->model_requests[k] = lat_model[k].size();
        out->model_p50_us[k] = pct_of(lat_model[k], 0.50);
        out->model_p99_us[k] = pct_of(lat_model[k], 0.99);
    }
    double mean = 0;
    for (double x : lat)
        mean += x;
    out->requests = lat.size();
    out->knots = knots;
    out->seconds = cfg->duration_s;
    out->p50_us = pct(0.50);
    out->p90_us = pct(0.90);
    out->p99_us = pct(0.99);
    out->max_us = lat.empty() ? 0.0 : lat.back();
    out->mean_us = lat.empty() ? 0.0 : mean / lat.size();
    out->offered_rate_per_s = cfg->rate_per_s;
    return GRID_OK;
}

}  // extern "C"
