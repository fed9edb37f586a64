// Host side of the batched launch: job validation, item planning (shape per job,
// longest items first), the job table, the graph of one control cycle, and the
// autotuners of the rollout tiling and of the batched kernel.
#include "gmapp_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

using namespace gm;

namespace {

constexpr int kDefaultTile = 4096;
constexpr int kDefaultBalance = 2;
constexpr int kRunsCap = 2 * kBatchMaxSegments + 2;

struct Tune {
    int tile, wg_per_cu, balance, shape;
};

Tune effective_tuning(const gmapp_ctx *ctx)
{
    Tune t{kDefaultTile, 0, kDefaultBalance, 0};
    auto apply = [&](const gmapp_batch_tuning &f) {
        if (f.tile_points > 0) t.tile = f.tile_points;
        if (f.wg_per_cu > 0) t.wg_per_cu = f.wg_per_cu;
        if (f.balance > 0) t.balance = f.balance;
        if (f.item_shape > 0) t.shape = f.item_shape;
    };
    if (ctx->batch_tuned) apply(ctx->batch_tuned_tuning);
    if (ctx->batch_forced) apply(ctx->batch_forced_tuning);
    return t;
}

gmapp_status check_tuning(gmapp_ctx *ctx, const gmapp_batch_tuning &t)
{
    if (t.tile_points < 0 || (t.tile_points > 0 && (t.tile_points < 64 || t.tile_points > 12288)))
        return fail(ctx, GMAPP_EINVAL, "tile_points must be 0 or in [64, 12288]");
    if (t.wg_per_cu < 0 || t.wg_per_cu > 4) return fail(ctx, GMAPP_EINVAL, "wg_per_cu must be in [0, 4]");
    if (t.balance < 0 || t.balance > 64) return fail(ctx, GMAPP_EINVAL, "balance must be in [0, 64]");
    if (t.item_shape < 0 || t.item_shape > 8) return fail(ctx, GMAPP_EINVAL, "item_shape must be in [0, 8]");
    return GMAPP_OK;
}

gmapp_status check_job(gmapp_ctx *ctx, const gmapp_job &j, int idx)
{
    gmapp_status st;
    if ((st = check_scene(ctx, &j.scene)) || (st = check_agents(ctx, &j.agents)) ||
        (st = check_params(ctx, &j.params, true)) || (st = check_query(ctx, &j.query))) {
        ctx->err = "job " + std::to_string(idx) + ": " + ctx->err;
        return st;
    }
    if (j.agents.heuristic)
        return fail(ctx, GMAPP_EINVAL, "job %d: batched launches run the rotation-vector circular field only "
                                       "(heuristic = NULL)", idx);
    if (j.scene.n_seg > kBatchMaxSegments)
        return fail(ctx, GMAPP_ECAPACITY, "job %d: %d segments (a batched launch takes at most %d)", idx,
                    j.scene.n_seg, kBatchMaxSegments);
    if (j.k_begin < 1 || j.k_begin > j.params.n_steps || j.k_end <= j.k_begin || j.k_end > j.params.n_steps + 1)
        return fail(ctx, GMAPP_EINVAL, "job %d: step range [%d, %d) outside 1..N_k+1 = %d", idx, j.k_begin, j.k_end,
                    j.params.n_steps + 1);
    const bool whole = j.k_begin == 1 && j.k_end == j.params.n_steps + 1;
    if (!whole && j.agents.n_agents > 0 && !j.state)
        return fail(ctx, GMAPP_EINVAL, "job %d: a partial step range needs a state buffer", idx);
    if (!j.out.best) return fail(ctx, GMAPP_EINVAL, "job %d: outputs.best is NULL", idx);
    if (j.agents.n_agents > 0 && !j.out.cost) return fail(ctx, GMAPP_EINVAL, "job %d: outputs.cost is NULL", idx);
    return GMAPP_OK;
}

// item shapes from the coarsest to the finest: (workgroup items?, agents per group)
struct Shape {
    int wg, aw;
};
constexpr Shape kLadder[] = {{0, 8}, {0, 4}, {0, 2}, {0, 1}, {1, 4}, {1, 2}, {1, 1}};

Shape shape_code(int code)
{
    static const Shape s[] = {{0, 1}, {0, 2}, {0, 4}, {0, 8}, {1, 1}, {1, 2}, {1, 4}, {1, 8}};
    return s[code - 1];
}

int agents_per_item(const Shape &s) { return s.wg ? s.aw : kBatchWaves * s.aw; }

// item duration in lane-interactions: every lane of the item handles aw / lanes-per-agent of the world per step
double item_length(const Shape &s, double steps, double n_pts)
{
    return steps * std::max(n_pts, 1.0) * s.aw / (s.wg ? 64.0 * kBatchWaves : 64.0);
}

// Plan the items of n jobs into `tab` (host memory of batch_table_bytes(n)).
gmapp_status plan(gmapp_ctx *ctx, const gmapp_job *jobs, int n, const Tune &tu, unsigned grid, BatchTable *tab)
{
    std::vector<double> len(n);
    std::vector<Shape> shp(n);
    double total = 0;
    for (int i = 0; i < n; ++i)
        total += (double)(jobs[i].k_end - jobs[i].k_begin) * (double)std::max<int64_t>(jobs[i].scene.n_points, 1) *
                 jobs[i].agents.n_agents;
    const double share = total / ((double)grid * 64.0 * kBatchWaves);   // balanced lane-interactions per workgroup
    const double bound = share / tu.balance;
    for (int i = 0; i < n; ++i) {
        const double steps = jobs[i].k_end - jobs[i].k_begin;
        const double np = (double)jobs[i].scene.n_points;
        const int na = std::max(jobs[i].agents.n_agents, 1);
        int p2 = 1;
        while (p2 < na) p2 <<= 1;
        if (tu.shape > 0) {
            shp[i] = shape_code(tu.shape);
        } else {
            shp[i] = kLadder[sizeof kLadder / sizeof kLadder[0] - 1];
            for (const Shape &s : kLadder)
                if (agents_per_item(s) <= p2 && item_length(s, steps, np) <= bound) {
                    shp[i] = s;
                    break;
                }
        }
        len[i] = item_length(shp[i], steps, np);
    }
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return len[a] > len[b]; });
    long long items = 0;
    tab->n_jobs = n;
    for (int q = 0; q < n; ++q) {
        const gmapp_job &j = jobs[order[q]];
        BatchJob &b = tab->jobs[q];
        b.sc = dev_scene(&j.scene);
        b.ag = dev_agents(&j.agents);
        b.pr = dev_params(&j.params, &j.query);
        b.out = Out{j.out.traj, j.out.cost, j.out.min_clear, j.out.best};
        b.state = j.state;
        b.k_begin = j.k_begin;
        b.k_end = j.k_end;
        b.cancel = reinterpret_cast<const unsigned *>(j.cancel);
        b.wg_items = shp[order[q]].wg;
        b.aw = shp[order[q]].aw;
        const int per = agents_per_item(shp[order[q]]);
        b.n_items = std::max(1, (j.agents.n_agents + per - 1) / per);
        b.item_base = (int)items;
        items += b.n_items;
        if (items > (long long)INT32_MAX / 2) return fail(ctx, GMAPP_ECAPACITY, "too many work items (%lld)", items);
    }
    tab->n_items = (int)items;
    return GMAPP_OK;
}

gmapp_status ensure_staging(gmapp_ctx *ctx, size_t bytes)
{
    if (!ctx->tab_copied) GM_HIP(ctx, hipEventCreateWithFlags(&ctx->tab_copied, hipEventDisableTiming));
    GM_HIP(ctx, hipEventSynchronize(ctx->tab_copied));        // the previous copy has read the staging buffer
    if (ctx->tab_host_bytes < bytes) {
        if (ctx->tab_host) GM_HIP(ctx, hipHostFree(ctx->tab_host));
        ctx->tab_host = nullptr;
        ctx->tab_host_bytes = 0;
        void *p = nullptr;
        const size_t want = std::max(bytes, batch_table_bytes(256));
        GM_HIP(ctx, hipHostMalloc(&p, want, hipHostMallocDefault));
        ctx->tab_host = p;
        ctx->tab_host_bytes = want;
    }
    return GMAPP_OK;
}

gmapp_status batch_direct(gmapp_ctx *ctx, const gmapp_job *jobs, int n, const Tune &tu, hipStream_t stream)
{
    BatchLaunch l;
    gmapp_status st = batch_launch_shape(ctx, BatchLay{tu.tile, kRunsCap}, tu.wg_per_cu, l);
    if (st) return st;
    const size_t bytes = batch_table_bytes(n);
    if (bytes > ctx->scratch_bytes) return fail(ctx, GMAPP_ENOMEM, "job table of %zu B exceeds the workspace", bytes);
    if ((st = ensure_staging(ctx, bytes))) return st;
    BatchTable *h = static_cast<BatchTable *>(ctx->tab_host);
    if ((st = plan(ctx, jobs, n, tu, l.grid, h))) return st;
    BatchTable *d = reinterpret_cast<BatchTable *>(ctx->scratch);
    GM_HIP(ctx, hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, stream));
    GM_HIP(ctx, hipEventRecord(ctx->tab_copied, stream));
    return launch_batch(ctx, d, l, stream);
}

gmapp_status check_jobs(gmapp_ctx *ctx, const gmapp_job *jobs, int n)
{
    if (n < 1 || n > kMaxBatchJobs) return fail(ctx, GMAPP_EINVAL, "n_jobs must be in [1, %d]", kMaxBatchJobs);
    if (!jobs) return fail(ctx, GMAPP_EINVAL, "jobs is NULL");
    for (int i = 0; i < n; ++i) {
        gmapp_status st = check_job(ctx, jobs[i], i);
        if (st) return st;
    }
    return GMAPP_OK;
}

}  // namespace

struct gmapp_batch {
    gmapp_ctx *ctx = nullptr;
    int max_jobs = 0;
    Tune tune{};
    BatchLaunch launch{};
    BatchTable *host = nullptr;   // pinned
    BatchTable *dev = nullptr;
    size_t bytes = 0;             // bytes the copy node moves
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t copy = nullptr, kernel = nullptr;
    hipEvent_t replayed = nullptr;
    bool ready = false;           // jobs set
    void *kargs[5]{};
    const BatchTable *arg_tab = nullptr;
};

extern "C" {

gmapp_status gmapp_set_batch_tuning(gmapp_ctx *ctx, const gmapp_batch_tuning *t)
{
    if (!ctx) return GMAPP_EINVAL;
    if (!t) { ctx->batch_forced = false; return GMAPP_OK; }
    gmapp_status st = check_tuning(ctx, *t);
    if (st) return st;
    ctx->batch_forced = true;
    ctx->batch_forced_tuning = *t;
    return GMAPP_OK;
}

gmapp_status gmapp_get_batch_tuning(gmapp_ctx *ctx, gmapp_batch_tuning *out)
{
    if (!ctx || !out) return GMAPP_EINVAL;
    const Tune t = effective_tuning(ctx);
    *out = gmapp_batch_tuning{t.tile, t.wg_per_cu, t.balance, t.shape};
    return GMAPP_OK;
}

gmapp_status gmapp_rollout_batch(gmapp_ctx *ctx, const gmapp_job *jobs, int32_t n_jobs, void *stream)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if ((st = check_jobs(ctx, jobs, n_jobs))) return st;
    return batch_direct(ctx, jobs, n_jobs, effective_tuning(ctx), static_cast<hipStream_t>(stream));
}

gmapp_status gmapp_batch_create(gmapp_ctx *ctx, int32_t max_jobs, gmapp_batch **out)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if (!out) return fail(ctx, GMAPP_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_jobs < 1 || max_jobs > kMaxBatchJobs)
        return fail(ctx, GMAPP_EINVAL, "max_jobs must be in [1, %d]", kMaxBatchJobs);
    gmapp_batch *b = new (std::nothrow) gmapp_batch();
    if (!b) return fail(ctx, GMAPP_ENOMEM, "out of host memory");
    b->ctx = ctx;
    b->max_jobs = max_jobs;
    b->tune = effective_tuning(ctx);
    auto bail = [&](gmapp_status s) {
        gmapp_batch_destroy(b);
        return s;
    };
    if ((st = batch_launch_shape(ctx, BatchLay{b->tune.tile, kRunsCap}, b->tune.wg_per_cu, b->launch)))
        return bail(st);
    const size_t cap = batch_table_bytes(max_jobs);
    void *p = nullptr;
    if (hipHostMalloc(&p, cap, hipHostMallocDefault) != hipSuccess)
        return bail(fail(ctx, GMAPP_ENOMEM, "pinned job table of %zu B", cap));
    b->host = static_cast<BatchTable *>(p);
    std::memset(b->host, 0, cap);
    if (hipMalloc(&p, cap) != hipSuccess) return bail(fail(ctx, GMAPP_ENOMEM, "device job table of %zu B", cap));
    b->dev = static_cast<BatchTable *>(p);
    if (hipEventCreateWithFlags(&b->replayed, hipEventDisableTiming) != hipSuccess)
        return bail(fail(ctx, GMAPP_EDEVICE, "hipEventCreate"));
    b->bytes = batch_table_bytes(1);
    hipError_t e = hipGraphCreate(&b->graph, 0);
    if (e == hipSuccess) e = hipGraphAddMemcpyNode1D(&b->copy, b->graph, nullptr, 0, b->dev, b->host, b->bytes,
                                                     hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        b->arg_tab = b->dev;
        b->kargs[0] = &b->arg_tab;
        b->kargs[1] = &b->launch.queue;
        b->kargs[2] = &b->launch.done;
        b->kargs[3] = &b->launch.lay;
        b->kargs[4] = &b->launch.abort;
        hipKernelNodeParams kp{};
        kp.func = const_cast<void *>(b->launch.fn);
        kp.gridDim = dim3(b->launch.grid);
        kp.blockDim = dim3(b->launch.block);
        kp.sharedMemBytes = (unsigned)b->launch.shm;
        kp.kernelParams = b->kargs;
        kp.extra = nullptr;
        e = hipGraphAddKernelNode(&b->kernel, b->graph, &b->copy, 1, &kp);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "building the control-cycle graph"));
    *out = b;
    return GMAPP_OK;
}

gmapp_status gmapp_batch_set_jobs(gmapp_batch *b, const gmapp_job *jobs, int32_t n_jobs)
{
    if (!b) return GMAPP_EINVAL;
    gmapp_ctx *ctx = b->ctx;
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if (n_jobs > b->max_jobs) return fail(ctx, GMAPP_ECAPACITY, "%d jobs exceed the batch's %d", n_jobs, b->max_jobs);
    if ((st = check_jobs(ctx, jobs, n_jobs))) return st;
    GM_HIP(ctx, hipEventSynchronize(b->replayed));     // the last replay has copied the pinned table
    if ((st = plan(ctx, jobs, n_jobs, b->tune, b->launch.grid, b->host))) {
        b->ready = false;
        return st;
    }
    const size_t bytes = batch_table_bytes(n_jobs);
    if (bytes != b->bytes) {
        GM_HIP(ctx, hipGraphExecMemcpyNodeSetParams1D(b->exec, b->copy, b->dev, b->host, bytes,
                                                      hipMemcpyHostToDevice));
        b->bytes = bytes;
    }
    b->ready = true;
    return GMAPP_OK;
}

gmapp_status gmapp_batch_launch(gmapp_batch *b, void *stream)
{
    if (!b) return GMAPP_EINVAL;
    gmapp_ctx *ctx = b->ctx;
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if (!b->ready) return fail(ctx, GMAPP_EINVAL, "no jobs set on this batch");
    GM_HIP(ctx, hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
    GM_HIP(ctx, hipEventRecord(b->replayed, static_cast<hipStream_t>(stream)));
    return GMAPP_OK;
}

void gmapp_batch_destroy(gmapp_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->ctx->device);
    if (b->replayed) (void)hipEventSynchronize(b->replayed);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->replayed) (void)hipEventDestroy(b->replayed);
    if (b->dev) (void)hipFree(b->dev);
    if (b->host) (void)hipHostFree(b->host);
    delete b;
}

// ---------------------------------------------------------------- autotuners

gmapp_status gmapp_autotune_rollout(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                                    const gmapp_query *query, const gmapp_params *params, int32_t proxy_steps,
                                    gmapp_tiling *best, float *best_ms, void *stream_)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if ((st = check_scene(ctx, scene)) || (st = check_agents(ctx, agents)) || (st = check_params(ctx, params, true)) ||
        (st = check_query(ctx, query)))
        return st;
    if (proxy_steps < 1) return fail(ctx, GMAPP_EINVAL, "proxy_steps must be >= 1");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const int na = agents->n_agents;
    const size_t need = (size_t)std::max(na, 1) * 5 * sizeof(float) + 256;
    if (need > ctx->scratch_bytes) return fail(ctx, GMAPP_ENOMEM, "workspace too small for the proxy outputs");
    gmapp_params pp = *params;
    pp.n_steps = std::min(proxy_steps, params->n_steps);
    Out o{nullptr, reinterpret_cast<float *>(ctx->scratch), nullptr,
          reinterpret_cast<int *>(ctx->scratch + (need - 256))};
    const Prm prm = dev_params(&pp, query);
    const Scn sc = dev_scene(scene);
    const Agt ag = dev_agents(agents);
    // candidates: agent groups per wavefront or per workgroup, waves, shards
    std::vector<Tiling> cand;
    for (int wg = 0; wg <= 1; ++wg)
        for (int A : {1, 2, 4, 8, 16, 32, 64})
            for (int W : {4, 8, 16})
                for (int S : {1, 2, 4, 8, 16, 32}) {
                    if (wg && A > 8) continue;
                    Tiling t{A, W, S, 2048, 0, wg};
                    const long long groups = wg ? (na + A - 1) / A : (na + A * W - 1) / (A * W);
                    if (groups * S > 4ll * ctx->n_cu || (groups * S < ctx->n_cu / 4 && S < 32)) continue;
                    if (check_tiling(ctx, t, scene->n_points, scene->n_seg, params->cutoff) != GMAPP_OK) continue;
                    cand.push_back(t);
                }
    hipEvent_t e0, e1;
    GM_HIP(ctx, hipEventCreate(&e0));
    GM_HIP(ctx, hipEventCreate(&e1));
    float best_t = INFINITY;
    Tiling bt{};
    for (const Tiling &t : cand) {
        if (launch_rollout(ctx, sc, ag, prm, o, nullptr, t, stream) != GMAPP_OK) continue;   // does not fit: skip
        float ms = INFINITY;
        for (int r = 0; r < 3; ++r) {
            (void)hipEventRecord(e0, stream);
            if (launch_rollout(ctx, sc, ag, prm, o, nullptr, t, stream) != GMAPP_OK) break;
            (void)hipEventRecord(e1, stream);
            if (hipEventSynchronize(e1) != hipSuccess) break;
            float m = 0;
            (void)hipEventElapsedTime(&m, e0, e1);
            ms = std::min(ms, m);
        }
        if (ms < best_t) {
            best_t = ms;
            bt = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->err.clear();
    if (!(best_t < INFINITY)) return fail(ctx, GMAPP_ECAPACITY, "no candidate tiling ran");
    const gmapp_tiling g{bt.A, bt.W, bt.S, bt.tile, bt.layout, bt.wg ? 2 : 1};
    ctx->tuned[tune_key(scene->n_points, na, params->n_steps, scene->n_seg, params->cutoff)] = g;
    if (best) *best = g;
    if (best_ms) *best_ms = best_t;
    return GMAPP_OK;
}

gmapp_status gmapp_autotune_batch(gmapp_ctx *ctx, const gmapp_job *jobs, int32_t n_jobs, int32_t proxy_steps,
                                  gmapp_batch_tuning *best, float *best_ms, void *stream_)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if ((st = check_jobs(ctx, jobs, n_jobs))) return st;
    if (proxy_steps < 1) return fail(ctx, GMAPP_EINVAL, "proxy_steps must be >= 1");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    // proxy jobs: whole horizons shortened in proportion, outputs into the workspace
    int max_k = 1;
    size_t out_floats = 0;
    for (int i = 0; i < n_jobs; ++i) {
        max_k = std::max(max_k, jobs[i].k_end - jobs[i].k_begin);
        out_floats += (size_t)jobs[i].agents.n_agents * 5 + 64;
    }
    const size_t tab_bytes = (batch_table_bytes(n_jobs) + 255) / 256 * 256;
    if (tab_bytes + out_floats * 4 > ctx->scratch_bytes)
        return fail(ctx, GMAPP_ENOMEM, "workspace too small for %d proxy jobs", n_jobs);
    std::vector<gmapp_job> px(jobs, jobs + n_jobs);
    float *o = reinterpret_cast<float *>(ctx->scratch + tab_bytes);
    for (int i = 0; i < n_jobs; ++i) {
        gmapp_job &j = px[i];
        const int steps = j.k_end - j.k_begin;
        j.params.n_steps = std::max(1, (int)std::lround((double)steps * proxy_steps / max_k));
        j.k_begin = 1;
        j.k_end = j.params.n_steps + 1;
        j.state = nullptr;
        j.out.traj = nullptr;
        j.out.min_clear = nullptr;
        j.out.cost = o;
        o += (size_t)j.agents.n_agents * 5;
        j.out.best = reinterpret_cast<int32_t *>(o);
        o += 64;
    }
    const Tune base = effective_tuning(ctx);
    std::vector<Tune> cand;
    for (int tile : {2048, 4096, 8192, 12288})
        for (int wpc : {1, 2, 3})
            for (int bal : {1, 2, 4, 8}) {
                Tune t{tile, wpc, bal, base.shape};
                if (batch_lds_bytes(BatchLay{tile, kRunsCap}) * wpc > (size_t)ctx->lds_per_cu) continue;
                cand.push_back(t);
            }
    hipEvent_t e0, e1;
    GM_HIP(ctx, hipEventCreate(&e0));
    GM_HIP(ctx, hipEventCreate(&e1));
    float best_t = INFINITY;
    Tune bt = base;
    for (const Tune &t : cand) {
        if (batch_direct(ctx, px.data(), n_jobs, t, stream) != GMAPP_OK) continue;
        float ms = INFINITY;
        for (int r = 0; r < 2; ++r) {
            (void)hipEventRecord(e0, stream);
            if (batch_direct(ctx, px.data(), n_jobs, t, stream) != GMAPP_OK) break;
            (void)hipEventRecord(e1, stream);
            if (hipEventSynchronize(e1) != hipSuccess) break;
            float m = 0;
            (void)hipEventElapsedTime(&m, e0, e1);
            ms = std::min(ms, m);
        }
        if (ms < best_t) {
            best_t = ms;
            bt = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->err.clear();
    if (!(best_t < INFINITY)) return fail(ctx, GMAPP_ECAPACITY, "no batch tuning ran");
    ctx->batch_tuned = true;
    ctx->batch_tuned_tuning = gmapp_batch_tuning{bt.tile, bt.wg_per_cu, bt.balance, 0};
    if (best) *best = gmapp_batch_tuning{bt.tile, bt.wg_per_cu, bt.balance, bt.shape};
    if (best_ms) *best_ms = best_t;
    return GMAPP_OK;
}

}  // extern "C"
