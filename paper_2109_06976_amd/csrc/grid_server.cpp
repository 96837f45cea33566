// Continuous-batching dFD server and its open-loop load generator (include/grid.h).
//
// Threads:
//   clients   grid_server_submit pushes a request onto the pending queue;
//   scheduler admits pending requests while the in-flight bytes fit the budget, packs
//             admitted requests of one model into a free batch context (pinned staging,
//             device buffers, its own stream), enqueues H2D copy, one launch, D2H copy and
//             an event, and polls the events of busy contexts;
//   copiers   scatter a completed context's outputs from pinned staging into the
//             requests' host buffers, mark the requests done, and free the context and
//             its admission bytes.
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

struct Request {
    uint64_t ticket = 0;
    int model = 0;
    int N = 0;
    const float *q = nullptr, *qd = nullptr, *tau = nullptr;
    float *qdd = nullptr, *Minv = nullptr, *dq = nullptr, *dqd = nullptr;
    size_t bytes = 0;
    std::atomic<int> state{kQueued};
    Clock::time_point t_done;
};

struct BatchCtx {
    int model = 0;
    int n = 0;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    float *d_in = nullptr, *d_out = nullptr, *h_in = nullptr, *h_out = nullptr;
    grid_workspace ws = nullptr;               // staged (per-request) mode only
    std::vector<Request*> reqs;
    int knots = 0;
    std::atomic<bool> busy{false};             // set by the scheduler, cleared by a copier
};

size_t request_bytes(int n, int N) { return sizeof(float) * (size_t)N * (4 * n + 3 * n * n); }

}  // namespace

struct grid_server_s {
    std::vector<grid_model> models;
    grid_server_config cfg{};
    int device = 0;
    std::vector<std::unique_ptr<BatchCtx>> ctx;

    std::mutex mu;                             // pending, tickets, next_ticket, accepting
    std::deque<Request*> pending;
    std::unordered_map<uint64_t, Request*> tickets;
    uint64_t next_ticket = 1;
    bool accepting = true;

    std::mutex done_mu;                        // completed contexts for the copiers
    std::condition_variable done_cv;
    std::deque<BatchCtx*> completed;
    std::atomic<int> free_events{0};           // contexts released by copiers (wake-up hint)

    std::atomic<bool> stop{false};             // scheduler: drain and exit
    std::atomic<bool> copiers_stop{false};     // copiers: exit once nothing is left
    std::atomic<size_t> inflight_bytes{0};
    std::thread scheduler;
    std::vector<std::thread> copiers;

    std::atomic<uint64_t> submitted{0}, completed_n{0}, canceled{0}, knots_done{0}, launches{0};
    std::atomic<uint64_t> max_inflight{0};
    std::atomic<bool> device_error{false};
};

namespace {

grid_status fail(grid_status s, const std::string& msg)
{
    set_error(msg);
    return s;
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
    s->free_events.fetch_add(1);
    for (Request* r : reqs) {
        if (final_state == kCanceled)
            s->canceled.fetch_add(1);
        r->state.store(final_state, std::memory_order_release);
    }
}

void copier_loop(grid_server s)
{
    for (;;) {
        BatchCtx* c = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->done_mu);
            s->done_cv.wait(lk, [&] { return !s->completed.empty() || s->copiers_stop.load(); });
            if (s->completed.empty())
                return;
            c = s->completed.front();
            s->completed.pop_front();
        }
        const size_t n = (size_t)c->n, K = (size_t)c->knots;
        const float* oq = c->h_out;
        const float* oM = oq + K * n;
        const float* oD = oM + K * n * n;
        const float* oV = oD + K * n * n;
        size_t off = 0;
        for (Request* r : c->reqs) {
            const size_t N = (size_t)r->N;
            std::memcpy(r->qdd, oq + off * n, N * n * sizeof(float));
            std::memcpy(r->Minv, oM + off * n * n, N * n * n * sizeof(float));
            std::memcpy(r->dq, oD + off * n * n, N * n * n * sizeof(float));
            std::memcpy(r->dqd, oV + off * n * n, N * n * n * sizeof(float));
            off += N;
            r->t_done = Clock::now();
            s->knots_done.fetch_add(N);
            s->completed_n.fetch_add(1);
        }
        finish_ctx(s, c, kDone);
    }
}

bool ctx_busy(BatchCtx* c) { return c->busy.load(std::memory_order_acquire); }

// stage inputs, enqueue copy-in, launch, copy-out and the completion event
bool launch_ctx(grid_server s, BatchCtx* c)
{
    grid_model m = s->models[c->model];
    const size_t n = (size_t)c->n, K = (size_t)c->knots;
    float* iq = c->h_in;
    float* iqd = iq + K * n;
    float* itau = iqd + K * n;
    size_t off = 0;
    for (Request* r : c->reqs) {
        const size_t N = (size_t)r->N;
        std::memcpy(iq + off * n, r->q, N * n * sizeof(float));
        std::memcpy(iqd + off * n, r->qd, N * n * sizeof(float));
        std::memcpy(itau + off * n, r->tau, N * n * sizeof(float));
        r->state.store(kLaunched, std::memory_order_relaxed);
        off += N;
    }
    float* dq = c->d_in;
    float* dqd = dq + K * n;
    float* dtau = dqd + K * n;
    float* oq = c->d_out;
    float* oM = oq + K * n;
    float* oD = oM + K * n * n;
    float* oV = oD + K * n * n;
    if (hipMemcpyAsync(dq, iq, 3 * K * n * sizeof(float), hipMemcpyHostToDevice, c->stream) !=
        hipSuccess)
        return false;
    grid_status st;
    if (s->cfg.flags & GRID_SERVER_PER_REQUEST)
        st = grid_fd_grad_staged(m, c->ws, (int32_t)K, dq, dqd, dtau, oq, oM, oD, oV, c->stream);
    else
        st = grid_fd_grad(m, (int32_t)K, dq, dqd, dtau, oq, oM, oD, oV, c->stream);
    if (st != GRID_OK)
        return false;
    if (hipMemcpyAsync(c->h_out, c->d_out, K * (n + 3 * n * n) * sizeof(float),
                       hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return false;
    if (hipEventRecord(c->done, c->stream) != hipSuccess)
        return false;
    s->launches.fetch_add(1);
    return true;
}

void scheduler_loop(grid_server s)
{
    (void)hipSetDevice(s->device);
    const int nm = (int)s->models.size();
    std::vector<std::deque<Request*>> admitted(nm);
    std::vector<BatchCtx*> inflight;
    for (;;) {
        bool progress = false;
        // completions: hand finished contexts to the copiers
        for (size_t k = 0; k < inflight.size();) {
            BatchCtx* c = inflight[k];
            hipError_t q = hipEventQuery(c->done);
            if (q == hipErrorNotReady) {
                ++k;
                continue;
            }
            if (q != hipSuccess)
                s->device_error.store(true);
            {
                std::lock_guard<std::mutex> lk(s->done_mu);
                s->completed.push_back(c);
            }
            s->done_cv.notify_one();
            inflight[k] = inflight.back();
            inflight.pop_back();
            progress = true;
        }
        // admission: FIFO while the bytes fit
        {
            std::lock_guard<std::mutex> lk(s->mu);
            while (!s->pending.empty()) {
                Request* r = s->pending.front();
                const size_t cur = s->inflight_bytes.load();
                if (cur + r->bytes > s->cfg.device_budget_bytes)
                    break;
                s->inflight_bytes.fetch_add(r->bytes);
                size_t now = cur + r->bytes, seen = s->max_inflight.load();
                while (now > seen && !s->max_inflight.compare_exchange_weak(seen, now)) {
                }
                s->pending.pop_front();
                admitted[r->model].push_back(r);
                progress = true;
            }
        }
        // packing: each free context of a model takes admitted requests up to the limit
        for (auto& cp : s->ctx) {
            BatchCtx* c = cp.get();
            auto& q = admitted[c->model];
            if (q.empty() || ctx_busy(c))
                continue;
            int knots = 0;
            while (!q.empty()) {
                Request* r = q.front();
                if (knots > 0 && ((s->cfg.flags & GRID_SERVER_PER_REQUEST) ||
                                  knots + r->N > s->cfg.max_batch_knots))
                    break;
                c->reqs.push_back(r);
                knots += r->N;
                q.pop_front();
            }
            c->knots = knots;
            c->busy.store(true, std::memory_order_release);
            if (!launch_ctx(s, c)) {
                s->device_error.store(true);
                (void)hipStreamSynchronize(c->stream);
                finish_ctx(s, c, kCanceled);
                continue;
            }
            inflight.push_back(c);
            progress = true;
        }
        if (s->stop.load()) {
            bool idle = inflight.empty();
            for (auto& q : admitted)
                idle = idle && q.empty();
            if (idle)
                break;
        }
        if (!progress)
            std::this_thread::yield();
    }
}

void destroy_ctx(BatchCtx* c)
{
    if (c->stream)
        (void)hipStreamSynchronize(c->stream);
    if (c->done)
        (void)hipEventDestroy(c->done);
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
        cfg->contexts_per_model > 64 || (cfg->flags & ~(uint32_t)GRID_SERVER_PER_REQUEST))
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
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
            if (e == hipSuccess)
                e = hipMalloc(&b->d_in, 3 * K * n * sizeof(float));
            if (e == hipSuccess)
                e = hipMalloc(&b->d_out, K * (n + 3 * n * n) * sizeof(float));
            if (e == hipSuccess)
                e = hipHostMalloc(&b->h_in, 3 * K * n * sizeof(float), hipHostMallocDefault);
            if (e == hipSuccess)
                e = hipHostMalloc(&b->h_out, K * (n + 3 * n * n) * sizeof(float), hipHostMallocDefault);
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
    const int ncopy = 4;
    for (int k = 0; k < ncopy; ++k)
        s->copiers.emplace_back(copier_loop, s);
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
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->accepting) {
            delete r;
            return fail(GRID_ECANCELED, "server is shutting down");
        }
        r->ticket = s->next_ticket++;
        s->tickets[r->ticket] = r;
        s->pending.push_back(r);
    }
    s->submitted.fetch_add(1);
    *ticket = r->ticket;
    return GRID_OK;
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

grid_status grid_server_wait(grid_server s, uint64_t ticket, int64_t timeout_us)
{
    if (!s)
        return fail(GRID_EINVAL, "server is NULL");
    Request* r = find_request(s, ticket);
    if (!r)
        return fail(GRID_EINVAL, "unknown ticket");
    const auto t0 = Clock::now();
    for (;;) {
        const int st = r->state.load(std::memory_order_acquire);
        if (st == kDone || st == kCanceled) {
            drop_ticket(s, r);
            if (st == kCanceled)
                return fail(GRID_ECANCELED, "request canceled");
            if (s->device_error.load())
                return fail(GRID_EDEVICE, "a device operation of the server failed");
            return GRID_OK;
        }
        if (timeout_us >= 0 &&
            std::chrono::duration_cast<std::chrono::microseconds>(Clock::now() - t0).count() >=
                timeout_us)
            return fail(GRID_ETIMEDOUT, "request still running");
        std::this_thread::yield();
    }
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
    s->stop.store(true);
    if (s->scheduler.joinable())
        s->scheduler.join();
    // the scheduler has handed every launched context to the copiers; let them drain
    for (;;) {
        bool busy = false;
        for (auto& c : s->ctx)
            busy = busy || ctx_busy(c.get());
        if (!busy)
            break;
        std::this_thread::yield();
    }
    {
        std::lock_guard<std::mutex> lk(s->done_mu);
        s->copiers_stop.store(true);
    }
    s->done_cv.notify_all();
    for (auto& t : s->copiers)
        t.join();
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
    std::mt19937_64 rng(cfg->seed);
    std::uniform_real_distribution<double> uni(0.0, 1.0);
    std::normal_distribution<float> gauss(0.0f, 1.0f);
    // input pools and output rings per model
    const int pool_knots = 8192, ring = 256;
    struct Pool {
        int n;
        std::vector<float> q, qd, tau;
        std::vector<float> qdd, M, D, V;       // ring of output slots
    };
    std::vector<Pool> pools(nm);
    for (int k = 0; k < nm; ++k) {
        Pool& p = pools[k];
        p.n = s->models[k]->topo.n;
        const size_t n = (size_t)p.n;
        p.q.resize(pool_knots * n);
        p.qd.resize(pool_knots * n);
        p.tau.resize(pool_knots * n);
        for (size_t i = 0; i < p.q.size(); ++i) {
            p.q[i] = (float)(M_PI * (2.0 * uni(rng) - 1.0));
            p.qd[i] = gauss(rng);
            p.tau[i] = 5.0f * gauss(rng);
        }
        const size_t slot = (size_t)cfg->n_max;
        p.qdd.resize(ring * slot * n);
        p.M.resize(ring * slot * n * n);
        p.D.resize(ring * slot * n * n);
        p.V.resize(ring * slot * n * n);
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
    uint64_t knots = 0;
    auto settle = [&](size_t idx) -> grid_status {
        Sent& e = sent[idx];
        // the caller owns the request until wait reports completion
        Request* r = find_request(s, e.ticket);
        Clock::time_point t_done;
        if (r) {
            while (r->state.load(std::memory_order_acquire) < kDone)
                std::this_thread::yield();
            t_done = r->t_done;
        }
        grid_status st = grid_server_wait(s, e.ticket, -1);
        if (st != GRID_OK)
            return st;
        if (e.counted) {
            lat.push_back(std::chrono::duration<double, std::micro>(t_done - e.t_sched).count());
            knots += (uint64_t)e.N;
        }
        return GRID_OK;
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
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double p) {
        if (lat.empty())
            return 0.0;
        const size_t i = std::min(lat.size() - 1, (size_t)std::floor(p * (lat.size() - 1) + 0.5));
        return lat[i];
    };
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
