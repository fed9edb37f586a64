// Replanning server: the request loop around the batched kernel.
//
// One host thread runs control cycles.  Each cycle takes every active request's
// next quantum of steps as one job of a gmapp_batch graph replay on the compute
// stream; while it runs, the loop admits waiting requests (FIFO, while a slot is
// free and their bytes fit the device budget) and uploads their worlds and
// agents on the copy stream, so they join the next cycle.  When the cycle ends,
// requests that reached the end of their horizon download their costs, choice
// and trajectory, release their memory and are reported.  The scheduling logic
// (allocator, FIFO, slots, quanta, deadlines, statistics) is in sched.h.
//
// Every admitted request holds one cancel word in mapped, coherent host memory
// (one per slot), which its job of each cycle carries: cancelling a request that
// is on the device raises the word, and the running cycle skips or stops that
// request's work (the batched kernel reads the word at every work item and every
// 64 steps), so the completion comes without waiting for the request's quantum.
#include "gmapp_internal.h"
#include "sched.h"

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>

using namespace gm;

namespace {

// Device block of one request: offsets of its pieces from the block start.
struct Layout {
    size_t x, y, z, seg_begin, seg_vel, agent[6], cost, best, state, traj, total;
};

Layout layout_of(const gmapp_request &r)
{
    using sched::round_up;
    Layout l{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += round_up(bytes);
        return at;
    };
    const size_t np = (size_t)std::max<int64_t>(r.n_points, 0), na = (size_t)std::max(r.n_agents, 0);
    l.x = take(4 * np);
    l.y = take(4 * np);
    l.z = take(4 * np);
    l.seg_begin = take(4 * ((size_t)r.n_seg + 1));
    l.seg_vel = take(12 * (size_t)r.n_seg);
    for (int i = 0; i < 5; ++i) l.agent[i] = take(4 * na);
    l.agent[5] = take(12 * na);
    l.cost = take(20 * na);
    l.best = take(4);
    l.state = take(4 * (size_t)kStateFloats * na);
    l.traj = r.traj ? take(12 * na * ((size_t)r.params.n_steps + 1)) : 0;
    l.total = o;
    return l;
}

struct Item {
    sched::Req req;
    gmapp_request in;
    Layout lay;
    int best = -1;
    int word = -1;      // cancel word while admitted
};

}  // namespace

struct gmapp_server {
    gmapp_ctx *ctx = nullptr;
    gmapp_server_config cfg{};
    char *arena = nullptr;
    gmapp_batch *batch = nullptr;
    hipStream_t comp = nullptr, copy = nullptr;
    hipEvent_t uploaded = nullptr;
    std::unique_ptr<sched::Core> core;
    std::mutex m;                 // core, items, completions
    std::mutex m_ctx;             // library calls that use the context (validation and launches)
    std::condition_variable cv_work, cv_done;
    std::unordered_map<int64_t, std::unique_ptr<Item>> items;
    std::deque<gmapp_completion> done;
    int64_t next_id = 1;
    bool stop = false;
    gmapp_status fault = GMAPP_OK;
    unsigned *cancel_host = nullptr;   // [max_active] cancel words, mapped and coherent
    unsigned *cancel_dev = nullptr;    // their device address
    std::vector<int> free_words;
    std::thread worker;
    std::chrono::steady_clock::time_point t0;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
    void run();
    gmapp_status upload(Item &it);
    gmapp_status download(Item &it);
    void report(std::vector<sched::Req *> &fin);
};

gmapp_status gmapp_server::upload(Item &it)
{
    const gmapp_request &r = it.in;
    char *b = arena + it.req.off;
    const Layout &l = it.lay;
    const size_t np = (size_t)r.n_points, na = (size_t)r.n_agents;
    auto put = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(b + off, src, bytes, hipMemcpyHostToDevice, copy);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = put(l.x, r.x, 4 * np);
    if (e == hipSuccess) e = put(l.y, r.y, 4 * np);
    if (e == hipSuccess) e = put(l.z, r.z, 4 * np);
    if (r.n_seg > 0) {
        if (e == hipSuccess) e = put(l.seg_begin, r.seg_begin, 4 * ((size_t)r.n_seg + 1));
        if (e == hipSuccess) e = put(l.seg_vel, r.seg_vel, 12 * (size_t)r.n_seg);
    }
    const float *src[6] = {r.k_a, r.d_a, r.k_f, r.r_d, r.r_a, r.omega};
    for (int i = 0; i < 6 && e == hipSuccess; ++i) e = put(l.agent[i], src[i], (i == 5 ? 12 : 4) * na);
    if (e != hipSuccess) return hip_fail(ctx, e, "request upload");
    return GMAPP_OK;
}

gmapp_status gmapp_server::download(Item &it)
{
    const gmapp_request &r = it.in;
    const char *b = arena + it.req.off;
    const size_t na = (size_t)r.n_agents;
    hipError_t e = hipMemcpyAsync(&it.best, b + it.lay.best, 4, hipMemcpyDeviceToHost, copy);
    if (e == hipSuccess && r.cost && na) e = hipMemcpyAsync(r.cost, b + it.lay.cost, 20 * na, hipMemcpyDeviceToHost, copy);
    if (e == hipSuccess && r.traj && na)
        e = hipMemcpyAsync(r.traj, b + it.lay.traj, 12 * na * ((size_t)r.params.n_steps + 1), hipMemcpyDeviceToHost,
                           copy);
    if (e == hipSuccess) e = hipStreamSynchronize(copy);
    if (e != hipSuccess) return hip_fail(ctx, e, "result download");
    return GMAPP_OK;
}

void gmapp_server::report(std::vector<sched::Req *> &fin)
{
    for (sched::Req *q : fin) {
        Item &it = *static_cast<Item *>(q->user);
        gmapp_completion c;
        c.id = q->id;
        c.status = q->status;
        c.best = q->status == 0 ? it.best : -1;
        c.queue_s = q->t_admit >= 0 ? q->t_admit - q->t_submit : -1.0;
        c.latency_s = q->t_finish - q->t_submit;
        done.push_back(c);
        if (it.word >= 0) free_words.push_back(it.word);
        items.erase(q->id);
    }
    fin.clear();
    cv_done.notify_all();
}

void gmapp_server::run()
{
    (void)hipSetDevice(ctx->device);
    std::vector<sched::Req *> fin;
    std::vector<gmapp_job> jobs;
    bool pending_upload = false;
    while (true) {
        std::vector<sched::Slice> slices;
        {
            std::unique_lock<std::mutex> lk(m);
            cv_work.wait(lk, [&] { return stop || !core->idle(); });
            if (stop) break;
            slices = core->plan();
        }
        // ---- launch the cycle (every active request's next quantum)
        const double c0 = now();
        bool launched = false;
        if (!slices.empty()) {
            jobs.clear();
            for (const sched::Slice &s : slices) {
                Item &it = *static_cast<Item *>(s.r->user);
                const gmapp_request &r = it.in;
                char *b = arena + s.r->off;
                auto f = [&](size_t o) { return reinterpret_cast<float *>(b + o); };
                gmapp_job j{};
                j.scene = gmapp_scene{f(it.lay.x), f(it.lay.y), f(it.lay.z), r.n_points, nullptr, r.r_obs, r.n_seg,
                                      reinterpret_cast<const int32_t *>(b + it.lay.seg_begin), f(it.lay.seg_vel)};
                j.agents = gmapp_agents{f(it.lay.agent[0]), f(it.lay.agent[1]), f(it.lay.agent[2]),
                                        f(it.lay.agent[3]), f(it.lay.agent[4]), f(it.lay.agent[5]), r.n_agents,
                                        nullptr};
                j.query = r.query;
                j.params = r.params;
                j.out = gmapp_outputs{r.traj ? f(it.lay.traj) : nullptr, f(it.lay.cost), nullptr,
                                      reinterpret_cast<int32_t *>(b + it.lay.best)};
                j.state = f(it.lay.state);
                j.k_begin = s.k_begin;
                j.k_end = s.k_end;
                j.cancel = it.word >= 0 ? cancel_dev + it.word : nullptr;
                jobs.push_back(j);
            }
            gmapp_status st;
            {
                std::lock_guard<std::mutex> g(m_ctx);
                if (pending_upload) (void)hipStreamWaitEvent(comp, uploaded, 0);
                st = gmapp_batch_set_jobs(batch, jobs.data(), (int)jobs.size());
                if (st == GMAPP_OK) st = gmapp_batch_launch(batch, comp);
            }
            pending_upload = false;
            if (st != GMAPP_OK) {
                std::lock_guard<std::mutex> lk(m);
                fault = st;
                for (const sched::Slice &s : slices) s.r->cancel = true;   // leave the loop's state consistent
                for (sched::Slice &s : slices) s.r->status = st;
            } else {
                launched = true;
            }
        }
        // ---- meanwhile: admit waiting requests and upload them (copy stream)
        std::vector<sched::Req *> in;
        {
            std::lock_guard<std::mutex> lk(m);
            in = core->admit(now(), fin);
            report(fin);
            for (sched::Req *q : in) {          // a lowered cancel word for each (slots bound them)
                Item &it = *static_cast<Item *>(q->user);
                if (!free_words.empty()) {
                    it.word = free_words.back();
                    free_words.pop_back();
                    __atomic_store_n(cancel_host + it.word, 0u, __ATOMIC_SEQ_CST);
                }
            }
        }
        if (!in.empty()) {
            std::lock_guard<std::mutex> g(m_ctx);
            for (sched::Req *q : in) {
                gmapp_status st = upload(*static_cast<Item *>(q->user));
                if (st != GMAPP_OK) {
                    std::lock_guard<std::mutex> lk(m);
                    q->cancel = true;
                    q->status = st;
                    fault = st;
                }
            }
            (void)hipEventRecord(uploaded, copy);
            pending_upload = true;
        }
        // ---- end of the cycle
        if (launched) {
            hipError_t e = hipStreamSynchronize(comp);
            if (e != hipSuccess) {
                std::lock_guard<std::mutex> lk(m);
                fault = GMAPP_EDEVICE;
                for (sched::Slice &s : slices) {
                    s.r->cancel = true;
                    s.r->status = GMAPP_EDEVICE;
                }
            }
        }
        const double c1 = now();
        {
            std::lock_guard<std::mutex> lk(m);
            core->complete(slices, c0, c1, fin);
        }
        // results of requests that finished their horizon (memory is reused only after this)
        for (sched::Req *q : fin)
            if (q->status == 0) {
                gmapp_status st = download(*static_cast<Item *>(q->user));
                if (st != GMAPP_OK) q->status = st;
            }
        {
            std::lock_guard<std::mutex> lk(m);
            report(fin);
        }
    }
}

namespace {

gmapp_status check_request(gmapp_ctx *ctx, const gmapp_request *r)
{
    if (!r) return fail(ctx, GMAPP_EINVAL, "request is NULL");
    gmapp_scene sc{r->x, r->y, r->z, r->n_points, nullptr, r->r_obs, r->n_seg, r->seg_begin, r->seg_vel};
    gmapp_agents ag{r->k_a, r->d_a, r->k_f, r->r_d, r->r_a, r->omega, r->n_agents, nullptr};
    gmapp_status st;
    if ((st = check_scene(ctx, &sc)) || (st = check_agents(ctx, &ag)) || (st = check_params(ctx, &r->params, true)) ||
        (st = check_query(ctx, &r->query)))
        return st;
    if (r->n_seg > kBatchMaxSegments)
        return fail(ctx, GMAPP_EINVAL, "request has %d segments (at most %d)", r->n_seg, kBatchMaxSegments);
    if (!(r->deadline_s >= 0)) return fail(ctx, GMAPP_EINVAL, "deadline_s must be >= 0");
    return GMAPP_OK;
}

}  // namespace

extern "C" {

gmapp_status gmapp_server_create(gmapp_ctx *ctx, const gmapp_server_config *cfg, gmapp_server **out)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if (!out) return fail(ctx, GMAPP_EINVAL, "out is NULL");
    *out = nullptr;
    gmapp_server_config c = cfg ? *cfg : gmapp_server_config{0, 0, 0, 0};
    if (c.max_active < 0 || c.max_active > kMaxBatchJobs || c.quantum_steps < 0 || c.max_queue < 0)
        return fail(ctx, GMAPP_EINVAL, "invalid server configuration");
    if (!c.memory_budget) c.memory_budget = 4ull << 30;
    if (!c.max_active) c.max_active = 256;
    if (!c.quantum_steps) c.quantum_steps = 50;
    if (!c.max_queue) c.max_queue = 65536;
    gmapp_server *s = new (std::nothrow) gmapp_server();
    if (!s) return fail(ctx, GMAPP_ENOMEM, "out of host memory");
    s->ctx = ctx;
    s->cfg = c;
    auto bail = [&](gmapp_status e) {
        gmapp_server_destroy(s);
        return e;
    };
    void *p = nullptr;
    if (hipMalloc(&p, c.memory_budget) != hipSuccess)
        return bail(fail(ctx, GMAPP_ENOMEM, "server memory budget of %llu B", (unsigned long long)c.memory_budget));
    s->arena = static_cast<char *>(p);
    if (hipStreamCreateWithFlags(&s->comp, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->uploaded, hipEventDisableTiming) != hipSuccess)
        return bail(fail(ctx, GMAPP_EDEVICE, "stream or event creation"));
    if ((st = gmapp_batch_create(ctx, c.max_active, &s->batch))) return bail(st);
    void *hw = nullptr, *dw = nullptr;
    if (hipHostMalloc(&hw, sizeof(unsigned) * (size_t)c.max_active, hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
        return bail(fail(ctx, GMAPP_ENOMEM, "pinned cancel words"));
    s->cancel_host = static_cast<unsigned *>(hw);
    std::memset(hw, 0, sizeof(unsigned) * (size_t)c.max_active);
    if (hipHostGetDevicePointer(&dw, hw, 0) != hipSuccess)
        return bail(fail(ctx, GMAPP_EDEVICE, "device address of the cancel words"));
    s->cancel_dev = static_cast<unsigned *>(dw);
    for (int w = c.max_active - 1; w >= 0; --w) s->free_words.push_back(w);
    s->core.reset(new sched::Core(c.memory_budget, c.max_active, c.quantum_steps, c.max_queue));
    s->t0 = std::chrono::steady_clock::now();
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return GMAPP_OK;
}

gmapp_status gmapp_server_submit(gmapp_server *s, const gmapp_request *req, int64_t *id)
{
    if (!s) return GMAPP_EINVAL;
    std::unique_ptr<Item> it(new (std::nothrow) Item());
    if (!it) return GMAPP_ENOMEM;
    {
        std::lock_guard<std::mutex> g(s->m_ctx);
        gmapp_status st = check_request(s->ctx, req);
        if (st) return st;
    }
    it->in = *req;
    it->lay = layout_of(*req);
    it->req.bytes = it->lay.total;
    it->req.n_steps = req->params.n_steps;
    it->req.work = (double)req->n_agents * req->params.n_steps * (double)req->n_points;
    it->req.user = it.get();
    std::lock_guard<std::mutex> lk(s->m);
    const double t = s->now();
    it->req.id = s->next_id;
    it->req.deadline = req->deadline_s > 0 ? t + req->deadline_s : 0;
    const int r = s->core->submit(&it->req, t);
    if (r == -1) {
        std::lock_guard<std::mutex> g(s->m_ctx);
        return fail(s->ctx, GMAPP_EINVAL, "request needs %zu device bytes, the budget is %llu", it->req.bytes,
                    (unsigned long long)s->cfg.memory_budget);
    }
    if (r != 0) {
        std::lock_guard<std::mutex> g(s->m_ctx);
        return fail(s->ctx, GMAPP_ECAPACITY, "request queue is full");
    }
    if (id) *id = s->next_id;
    s->items[s->next_id++] = std::move(it);
    s->cv_work.notify_one();
    return GMAPP_OK;
}

int32_t gmapp_server_poll(gmapp_server *s, gmapp_completion *out, int32_t max, int32_t wait_ms)
{
    if (!s || !out || max < 1) return 0;
    std::unique_lock<std::mutex> lk(s->m);
    if (s->done.empty() && wait_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->done.empty(); });
    int32_t n = 0;
    while (n < max && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    return n;
}

gmapp_status gmapp_server_cancel(gmapp_server *s, int64_t id)
{
    if (!s) return GMAPP_EINVAL;
    std::lock_guard<std::mutex> lk(s->m);
    if (!s->core->cancel(id)) return GMAPP_EINVAL;
    auto f = s->items.find(id);
    if (f != s->items.end() && f->second->word >= 0)   // on the device: stop its work in the running cycle
        __atomic_store_n(s->cancel_host + f->second->word, 1u, __ATOMIC_SEQ_CST);
    s->cv_work.notify_one();
    return GMAPP_OK;
}

gmapp_status gmapp_server_drain(gmapp_server *s, int32_t timeout_ms)
{
    if (!s) return GMAPP_EINVAL;
    std::unique_lock<std::mutex> lk(s->m);
    auto idle = [&] { return s->core->idle(); };
    if (timeout_ms < 0) {
        s->cv_done.wait(lk, idle);
        return GMAPP_OK;
    }
    return s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), idle) ? GMAPP_OK : GMAPP_ETIMEOUT;
}

gmapp_status gmapp_server_get_stats(gmapp_server *s, gmapp_server_stats *out)
{
    if (!s || !out) return GMAPP_EINVAL;
    std::lock_guard<std::mutex> lk(s->m);
    const sched::Stats st = s->core->stats();
    out->submitted = st.submitted;
    out->completed = st.completed;
    out->rejected = st.rejected;
    out->expired = st.expired;
    out->cancelled = st.cancelled;
    out->cycles = st.cycles;
    out->p50_s = st.p50_s;
    out->p99_s = st.p99_s;
    out->max_s = st.max_s;
    out->mean_s = st.mean_s;
    out->busy_s = st.busy_s;
    out->interactions_per_s = st.busy_s > 0 ? st.work_done / st.busy_s : 0;
    out->cycle_mean_s = st.cycle_mean_s;
    out->max_active_seen = st.max_active_seen;
    out->peak_bytes = st.peak_bytes;
    return s->fault;
}

void gmapp_server_destroy(gmapp_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->ctx->device);
    if (s->comp) (void)hipStreamSynchronize(s->comp);
    if (s->copy) (void)hipStreamSynchronize(s->copy);
    if (s->batch) gmapp_batch_destroy(s->batch);
    if (s->uploaded) (void)hipEventDestroy(s->uploaded);
    if (s->comp) (void)hipStreamDestroy(s->comp);
    if (s->copy) (void)hipStreamDestroy(s->copy);
    if (s->arena) (void)hipFree(s->arena);
    if (s->cancel_host) (void)hipHostFree(s->cancel_host);
    delete s;
}

}  // extern "C"
