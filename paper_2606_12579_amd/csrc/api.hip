// C ABI entry points: context lifetime, argument validation and dispatch.
// Every check runs on the host before anything is enqueued.
#include "gmapp_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>

using gm::fail;

namespace {

__global__ void k_fill_u32(unsigned *p, size_t n, unsigned v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

bool finite(float x) { return std::isfinite(x); }

}  // namespace

namespace gm {

gmapp_status check_ctx(gmapp_ctx *ctx)
{
    if (!ctx) return GMAPP_EINVAL;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return gm::hip_fail(ctx, e, "hipSetDevice");
    return GMAPP_OK;
}

gmapp_status check_scene(gmapp_ctx *ctx, const gmapp_scene *sc)
{
    if (!sc) return fail(ctx, GMAPP_EINVAL, "scene is NULL");
    if (sc->n_points < 0) return fail(ctx, GMAPP_EINVAL, "n_points must be >= 0");
    if (sc->n_points > (int64_t)INT32_MAX) return fail(ctx, GMAPP_ECAPACITY, "n_points exceeds 2^31 - 1");
    if (sc->n_points > 0 && (!sc->x || !sc->y || !sc->z)) return fail(ctx, GMAPP_EINVAL, "scene x/y/z is NULL");
    if (!finite(sc->r_obs) || sc->r_obs < 0) return fail(ctx, GMAPP_EINVAL, "r_obs must be finite and >= 0");
    if (sc->n_seg < 0) return fail(ctx, GMAPP_EINVAL, "n_seg must be >= 0");
    if (sc->n_seg > 0 && (!sc->seg_begin || !sc->seg_vel))
        return fail(ctx, GMAPP_EINVAL, "seg_begin/seg_vel is NULL with n_seg > 0");
    if (sc->n_seg > 0 && sc->n_points_dev)
        return fail(ctx, GMAPP_EINVAL, "a device-resident point count needs a static scene (n_seg = 0)");
    return GMAPP_OK;
}

gmapp_status check_agents(gmapp_ctx *ctx, const gmapp_agents *ag)
{
    if (!ag) return fail(ctx, GMAPP_EINVAL, "agents is NULL");
    if (ag->n_agents < 0) return fail(ctx, GMAPP_EINVAL, "n_agents must be >= 0");
    if (ag->n_agents > (1 << 24)) return fail(ctx, GMAPP_ECAPACITY, "n_agents exceeds 2^24");
    if (ag->n_agents > 0 && (!ag->k_a || !ag->d_a || !ag->k_f || !ag->r_d || !ag->r_a || !ag->omega))
        return fail(ctx, GMAPP_EINVAL, "an agent parameter array is NULL");
    return GMAPP_OK;
}

gmapp_status check_params(gmapp_ctx *ctx, const gmapp_params *p, bool need_steps)
{
    if (!p) return fail(ctx, GMAPP_EINVAL, "params is NULL");
    if (need_steps && p->n_steps < 1) return fail(ctx, GMAPP_EINVAL, "n_steps must be >= 1");
    if (p->n_steps > (1 << 24)) return fail(ctx, GMAPP_ECAPACITY, "n_steps exceeds 2^24");
    if (!finite(p->dt) || p->dt <= 0) return fail(ctx, GMAPP_EINVAL, "dt must be finite and > 0");
    if (!finite(p->inv_mass)) return fail(ctx, GMAPP_EINVAL, "inv_mass must be finite");
    if (!finite(p->eps) || p->eps <= 0) return fail(ctx, GMAPP_EINVAL, "eps must be finite and > 0");
    if (!finite(p->r_cost) || p->r_cost <= 0) return fail(ctx, GMAPP_EINVAL, "r_cost must be finite and > 0");
    if (!finite(p->a_max) || p->a_max <= 0) return fail(ctx, GMAPP_EINVAL, "a_max must be finite and > 0");
    if (!finite(p->w_goal) || !finite(p->w_obs) || !finite(p->w_path) || !finite(p->w_smooth) || !finite(p->alpha))
        return fail(ctx, GMAPP_EINVAL, "cost weights and alpha must be finite");
    if (p->cutoff != 0 && p->cutoff != 1) return fail(ctx, GMAPP_EINVAL, "cutoff must be 0 (hard) or 1 (taper)");
    if (p->cutoff == 1 && (!finite(p->taper_band) || p->taper_band <= 0 || p->taper_band > 1))
        return fail(ctx, GMAPP_EINVAL, "taper_band must be in (0, 1]");
    return GMAPP_OK;
}

gmapp_status check_query(gmapp_ctx *ctx, const gmapp_query *query)
{
    if (!query) return fail(ctx, GMAPP_EINVAL, "query is NULL");
    for (int a = 0; a < 3; ++a)
        if (!finite(query->p0[a]) || !finite(query->v0[a]) || !finite(query->goal[a]))
            return fail(ctx, GMAPP_EINVAL, "query start/velocity/goal must be finite");
    if (!finite(query->t0)) return fail(ctx, GMAPP_EINVAL, "query t0 must be finite");
    return GMAPP_OK;
}

gm::Scn dev_scene(const gmapp_scene *sc)
{
    gm::Scn s;
    s.x = sc->x; s.y = sc->y; s.z = sc->z;
    s.n_cap = sc->n_points;
    s.n_dev = reinterpret_cast<const long long *>(sc->n_points_dev);
    s.r_obs = sc->r_obs;
    s.n_seg = sc->n_seg;
    s.seg_begin = sc->seg_begin;
    s.seg_vel = sc->seg_vel;
    return s;
}

gm::Agt dev_agents(const gmapp_agents *ag)
{
    return gm::Agt{ag->k_a, ag->d_a, ag->k_f, ag->r_d, ag->r_a, ag->omega, ag->n_agents, ag->heuristic};
}

gm::Prm dev_params(const gmapp_params *p, const gmapp_query *q)
{
    gm::Prm r;
    r.dt = p->dt; r.inv_mass = p->inv_mass; r.eps = p->eps; r.r_cost = p->r_cost;
    r.w0 = p->w_goal; r.w1 = p->w_obs; r.w2 = p->w_path; r.w3 = p->w_smooth;
    r.a_max = p->a_max; r.alpha = p->alpha; r.band = p->cutoff == 1 ? p->taper_band : 1.0f;
    r.n_steps = p->n_steps; r.cutoff = p->cutoff;
    for (int a = 0; a < 3; ++a) {
        r.p0[a] = q ? q->p0[a] : 0.f;
        r.v0[a] = q ? q->v0[a] : 0.f;
        r.goal[a] = q ? q->goal[a] : 0.f;
    }
    r.incumbent = q ? q->incumbent : -1;
    r.t0 = q ? q->t0 : 0.f;
    return r;
}

}  // namespace gm

using namespace gm;

namespace {

gm::Tiling tiling_for(gmapp_ctx *ctx, long long n_points, int n_agents, int n_steps, int n_seg, int cutoff)
{
    gm::Tiling t = gm::choose_tiling(ctx, n_points, n_agents, n_steps, n_seg, cutoff);
    const gmapp_tiling *use = nullptr;
    if (ctx->forced) {
        use = &ctx->forced_tiling;
    } else {
        auto it = ctx->tuned.find(gm::tune_key(n_points, n_agents, n_steps, n_seg, cutoff));
        if (it != ctx->tuned.end()) use = &it->second;
    }
    if (use) {
        const gmapp_tiling &f = *use;
        if (f.group > 0) t.wg = f.group == 2 ? 1 : 0;
        if (f.agents > 0) t.A = f.agents;
        if (f.waves > 0) t.W = f.waves;
        if (f.shards > 0) t.S = f.shards;
        if (f.tile_points > 0) t.tile = f.tile_points;
        t.layout = f.layout;
    }
    return t;
}

// the exchange waits' limit and the device address of the abort word, in the words after
// the status word (a synchronous copy: launches enqueued afterwards see them)
gmapp_status write_wait_settings(gmapp_ctx *ctx)
{
    unsigned long long v[2] = {ctx->watchdog_ticks, (unsigned long long)reinterpret_cast<uintptr_t>(ctx->abort_word)};
    unsigned *dst = ctx->sync + gm::kCounterWords + 16 + gm::kWaitLimitWord;
    const hipError_t e = hipMemcpy(dst, v, sizeof v, hipMemcpyHostToDevice);
    if (e != hipSuccess) return gm::hip_fail(ctx, e, "hipMemcpy(wait settings)");
    return GMAPP_OK;
}

// lattice and self-filter arguments of the voxel pass
gmapp_status voxel_grid(gmapp_ctx *ctx, float voxel, const float lo[3], const int32_t dims[3], int32_t min_count,
                        const float *robot_spheres, int32_t n_spheres, gm::VoxGrid &g)
{
    if (!lo || !dims) return fail(ctx, GMAPP_EINVAL, "lo and dims must be non-NULL");
    if (!finite(voxel) || voxel <= 0.f) return fail(ctx, GMAPP_EINVAL, "voxel must be finite and > 0");
    if (min_count < 1) return fail(ctx, GMAPP_EINVAL, "min_count must be >= 1");
    if (n_spheres < 0 || (n_spheres > 0 && !robot_spheres))
        return fail(ctx, GMAPP_EINVAL, "n_spheres must be >= 0, with robot_spheres non-NULL when > 0");
    g.voxel = voxel;
    g.excl = n_spheres > 0 ? robot_spheres : nullptr;
    g.n_excl = n_spheres;
    long long cells = 1;
    for (int a = 0; a < 3; ++a) {
        if (!finite(lo[a])) return fail(ctx, GMAPP_EINVAL, "lo must be finite");
        if (dims[a] < 1) return fail(ctx, GMAPP_EINVAL, "dims must be >= 1");
        // k + 1/2 exact in FP32, so that each centre lo + (k + 1/2) voxel is one rounding (a fused multiply-add)
        if (dims[a] > (1 << 23)) return fail(ctx, GMAPP_ECAPACITY, "dims must be <= 2^23 per axis");
        g.lo[a] = lo[a];
        g.dims[a] = dims[a];
        cells *= dims[a];
        if (cells > (1ll << 31)) return fail(ctx, GMAPP_ECAPACITY, "voxel grid exceeds 2^31 cells");
    }
    return GMAPP_OK;
}

}  // namespace

extern "C" {

const char *gmapp_version(void) { return "gmapp 0.1 gfx950"; }

gmapp_status gmapp_create(int32_t device, size_t workspace_bytes, gmapp_ctx **out)
{
    if (!out) return GMAPP_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return GMAPP_EDEVICE;
    if (device < 0 || device >= n) return GMAPP_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return GMAPP_EDEVICE;
    gmapp_ctx *ctx = new (std::nothrow) gmapp_ctx();
    if (!ctx) return GMAPP_ENOMEM;
    ctx->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete ctx; return GMAPP_EDEVICE; }
    ctx->n_cu = prop.multiProcessorCount;
    ctx->lds_per_cu = (int)prop.maxSharedMemoryPerMultiProcessor;
    if (workspace_bytes == 0) workspace_bytes = (size_t)256 << 20;
    const size_t sync_bytes = (gm::kSyncWords * sizeof(unsigned) + 4095) / 4096 * 4096;
    const size_t fixed = sync_bytes + gm::kXchgBytes;
    if (workspace_bytes < fixed + (1 << 20)) workspace_bytes = fixed + (1 << 20);
    void *p = nullptr;
    if (hipMalloc(&p, workspace_bytes) != hipSuccess) { delete ctx; return GMAPP_ENOMEM; }
    ctx->arena = static_cast<char *>(p);
    ctx->arena_bytes = workspace_bytes;
    ctx->sync = reinterpret_cast<unsigned *>(ctx->arena);
    ctx->xchg = reinterpret_cast<unsigned long long *>(ctx->arena + sync_bytes);
    ctx->scratch = ctx->arena + fixed;
    ctx->scratch_bytes = workspace_bytes - fixed;
    // the host's abort word: pinned, coherent and mapped, so that a running kernel's waits see a
    // host store without any copy
    void *hw = nullptr;
    if (hipHostMalloc(&hw, 64, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        (void)hipFree(p);
        delete ctx;
        return GMAPP_ENOMEM;
    }
    *static_cast<volatile unsigned *>(hw) = 0u;
    ctx->abort_host = static_cast<unsigned *>(hw);
    void *dw = nullptr;
    if (hipHostGetDevicePointer(&dw, hw, 0) != hipSuccess) {
        (void)hipHostFree(hw);
        (void)hipFree(p);
        delete ctx;
        return GMAPP_EDEVICE;
    }
    ctx->abort_word = static_cast<unsigned *>(dw);
    hipLaunchKernelGGL(k_fill_u32, dim3(256), dim3(256), 0, nullptr, ctx->sync, fixed / sizeof(unsigned), 0u);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess || write_wait_settings(ctx) ||
        gm::static_scratch_init(ctx) != GMAPP_OK) {
        (void)hipHostFree(hw);
        (void)hipFree(p);
        delete ctx;
        return GMAPP_EDEVICE;
    }
    *out = ctx;
    return GMAPP_OK;
}

void gmapp_destroy(gmapp_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->arena) (void)hipFree(ctx->arena);
    if (ctx->vgrid) (void)hipFree(ctx->vgrid);
    if (ctx->vbsum) (void)hipFree(ctx->vbsum);
    if (ctx->tab_host) (void)hipHostFree(ctx->tab_host);
    if (ctx->abort_host) (void)hipHostFree(ctx->abort_host);
    if (ctx->tab_copied) (void)hipEventDestroy(ctx->tab_copied);
    delete ctx;
}

const char *gmapp_last_error(const gmapp_ctx *ctx)
{
    if (!ctx) return "no context";
    return ctx->err.c_str();
}

gmapp_status gmapp_set_watchdog(gmapp_ctx *ctx, double seconds)
{
    if (!ctx) return GMAPP_EINVAL;
    if (seconds == 0.0) seconds = 4.0;
    if (!std::isfinite(seconds) || seconds < 0.0 || seconds > 3600.0)
        return fail(ctx, GMAPP_EINVAL, "watchdog limit must be in (0, 3600] s (0 = the default 4 s)");
    ctx->watchdog_ticks = std::max<unsigned long long>(1ull, (unsigned long long)(seconds * 1e8));
    return write_wait_settings(ctx);
}

gmapp_status gmapp_abort(gmapp_ctx *ctx, int32_t raise)
{
    if (!ctx || !ctx->abort_host) return GMAPP_EINVAL;
    __atomic_store_n(ctx->abort_host, raise ? 1u : 0u, __ATOMIC_SEQ_CST);
    return GMAPP_OK;
}

gmapp_status gmapp_wait(gmapp_ctx *ctx, void *stream_, double timeout_s)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if (!(timeout_s >= 0.0)) return fail(ctx, GMAPP_EINVAL, "timeout must be >= 0");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const auto t0 = std::chrono::steady_clock::now();
    while (true) {
        const hipError_t e = hipStreamQuery(stream);
        if (e == hipSuccess) return GMAPP_OK;
        if (e != hipErrorNotReady) return gm::hip_fail(ctx, e, "hipStreamQuery");
        if (std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > timeout_s) break;
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    // out of time: raise the abort word so that every exchange wait ends, drain, lower it
    __atomic_store_n(ctx->abort_host, 1u, __ATOMIC_SEQ_CST);
    const hipError_t e = hipStreamSynchronize(stream);
    __atomic_store_n(ctx->abort_host, 0u, __ATOMIC_SEQ_CST);
    if (e != hipSuccess) return gm::hip_fail(ctx, e, "hipStreamSynchronize");
    return fail(ctx, GMAPP_ETIMEOUT, "stream work did not finish within %.3f s; its launches were aborted", timeout_s);
}

gmapp_status gmapp_set_tiling(gmapp_ctx *ctx, const gmapp_tiling *t)
{
    if (!ctx) return GMAPP_EINVAL;
    if (!t) { ctx->forced = false; return GMAPP_OK; }
    if (t->agents < 0 || t->waves < 0 || t->shards < 0 || t->tile_points < 0 || t->layout < 0 || t->group < 0 ||
        t->group > 2)
        return fail(ctx, GMAPP_EINVAL, "tiling fields must be >= 0");
    ctx->forced = true;
    ctx->forced_tiling = *t;
    return GMAPP_OK;
}

gmapp_status gmapp_get_tiling(gmapp_ctx *ctx, int64_t n_points, int32_t n_agents, int32_t n_steps, int32_t n_seg,
                              int32_t cutoff, gmapp_tiling *out)
{
    if (!ctx || !out) return GMAPP_EINVAL;
    gm::Tiling t = tiling_for(ctx, n_points, n_agents, n_steps, n_seg, cutoff);
    *out = gmapp_tiling{t.A, t.W, t.S, t.tile, t.layout, t.wg ? 2 : 1};
    return GMAPP_OK;
}

gmapp_status gmapp_rollout(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                           const gmapp_query *query, const gmapp_params *params, const gmapp_outputs *out,
                           void *stream)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if ((st = check_scene(ctx, scene)) || (st = check_agents(ctx, agents)) || (st = check_params(ctx, params, true)))
        return st;
    if ((st = check_query(ctx, query))) return st;
    if (!out || !out->best) return fail(ctx, GMAPP_EINVAL, "outputs.best is NULL");
    if (agents->n_agents > 0 && !out->cost) return fail(ctx, GMAPP_EINVAL, "outputs.cost is NULL");
    gm::Tiling t = tiling_for(ctx, scene->n_points, agents->n_agents, params->n_steps, scene->n_seg, params->cutoff);
    gm::Out o{out->traj, out->cost, out->min_clear, out->best};
    return gm::launch_rollout(ctx, dev_scene(scene), dev_agents(agents), dev_params(params, query), o, nullptr, t,
                              static_cast<hipStream_t>(stream));
}

gmapp_status gmapp_force_probe(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents, const float *p,
                               const float *v, float t, const gmapp_params *params, float *f_r, float *rho_min,
                               void *stream)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if ((st = check_scene(ctx, scene)) || (st = check_agents(ctx, agents)) || (st = check_params(ctx, params, false)))
        return st;
    if (agents->n_agents > 0 && (!p || !v || !f_r)) return fail(ctx, GMAPP_EINVAL, "p, v and f_r must be non-NULL");
    if (!finite(t)) return fail(ctx, GMAPP_EINVAL, "t must be finite");
    gm::Tiling tl = tiling_for(ctx, scene->n_points, agents->n_agents, 1, scene->n_seg, params->cutoff);
    gm::Probe pb{p, v, t, f_r, rho_min};
    gm::Out o{nullptr, nullptr, nullptr, nullptr};
    return gm::launch_rollout(ctx, dev_scene(scene), dev_agents(agents), dev_params(params, nullptr), o, &pb, tl,
                              static_cast<hipStream_t>(stream));
}

namespace {

// shared by the pose and arm entry points: validation and launch of the 6-D rollout
gmapp_status rollout_6d(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                        const gmapp_pose_agents *pose, const gmapp_arm *arm, const gmapp_query *query,
                        const gmapp_pose_query *pose_query, const gmapp_params *params, const gmapp_outputs *out,
                        float *rot, float *joints, void *stream);

}  // namespace

gmapp_status gmapp_rollout_pose(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                                const gmapp_pose_agents *pose, const gmapp_query *query,
                                const gmapp_pose_query *pose_query, const gmapp_params *params,
                                const gmapp_outputs *out, float *rot, void *stream)
{
    return rollout_6d(ctx, scene, agents, pose, nullptr, query, pose_query, params, out, rot, nullptr, stream);
}

gmapp_status gmapp_rollout_arm(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                               const gmapp_pose_agents *pose, const gmapp_arm *arm, const gmapp_query *query,
                               const gmapp_pose_query *pose_query, const gmapp_params *params,
                               const gmapp_outputs *out, float *rot, float *joints, void *stream)
{
    if (ctx && !arm) return fail(ctx, GMAPP_EINVAL, "arm is NULL");
    return rollout_6d(ctx, scene, agents, pose, arm, query, pose_query, params, out, rot, joints, stream);
}

namespace {

gmapp_status rollout_6d(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                        const gmapp_pose_agents *pose, const gmapp_arm *arm, const gmapp_query *query,
                        const gmapp_pose_query *pose_query, const gmapp_params *params, const gmapp_outputs *out,
                        float *rot, float *joints, void *stream)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if ((st = check_scene(ctx, scene)) || (st = check_agents(ctx, agents)) || (st = check_params(ctx, params, true)))
        return st;
    if ((st = check_query(ctx, query))) return st;
    if (!pose || !pose_query) return fail(ctx, GMAPP_EINVAL, "pose agents and pose query must be non-NULL");
    if (agents->n_agents > 0 && (!pose->k_r || !pose->d_r || !pose->inv_inertia_r))
        return fail(ctx, GMAPP_EINVAL, "pose gains k_r, d_r and inv_inertia_r must be non-NULL");
    auto rotor_ok = [](const float *q) {
        const float n = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
        return finite(q[0]) && finite(q[1]) && finite(q[2]) && finite(q[3]) && finite(n) && n > 0.0f;
    };
    if ((!arm && !rotor_ok(pose_query->q0)) || !rotor_ok(pose_query->qg))
        return fail(ctx, GMAPP_EINVAL, "q0 and qg must be finite rotors with a non-zero norm");
    if (arm) {
        if (arm->n_joints < 1 || arm->n_joints > gm::kMaxArmJoints)
            return fail(ctx, GMAPP_EINVAL, "n_joints must be in [1, %d]", gm::kMaxArmJoints);
        if (!arm->links || !arm->q0) return fail(ctx, GMAPP_EINVAL, "arm links and q0 must be non-NULL");
        if (!finite(arm->damping) || arm->damping < 0.0f)
            return fail(ctx, GMAPP_EINVAL, "damping must be finite and >= 0");
        if (arm->damping == 0.0f && arm->n_joints < 6)   // J_b J_b^T (6 x 6) has rank <= n_joints
            return fail(ctx, GMAPP_EINVAL, "damping 0 needs at least 6 joints (J_b J_b^T is singular)");
    }
    if (!finite(pose_query->w0[0]) || !finite(pose_query->w0[1]) || !finite(pose_query->w0[2]))
        return fail(ctx, GMAPP_EINVAL, "w0 must be finite");
    if (!out || !out->best) return fail(ctx, GMAPP_EINVAL, "outputs.best is NULL");
    if (agents->n_agents > 0 && !out->cost) return fail(ctx, GMAPP_EINVAL, "outputs.cost is NULL");
    gm::Tiling t = tiling_for(ctx, scene->n_points, agents->n_agents, params->n_steps, scene->n_seg, params->cutoff);
    // arm agents hold a lane per joint in a wave: a chosen or tuned tiling is capped
    if (arm && !ctx->forced && t.A > gm::kMaxArmAgentsPerGroup) t.A = gm::kMaxArmAgentsPerGroup;
    gm::Agt ag = dev_agents(agents);
    if (agents->n_agents > 0) {
        ag.k_r = pose->k_r;
        ag.d_r = pose->d_r;
        ag.i_r = pose->inv_inertia_r;
    }
    gm::Prm pr = dev_params(params, query);
    for (int a = 0; a < 4; ++a) {
        pr.q0[a] = pose_query->q0[a];
        pr.qg[a] = pose_query->qg[a];
    }
    for (int a = 0; a < 3; ++a) pr.om0[a] = pose_query->w0[a];
    if (arm) {
        pr.arm_links = arm->links;
        pr.arm_q0 = arm->q0;
        pr.arm_n = arm->n_joints;
        pr.arm_lam2 = arm->damping * arm->damping;
    }
    const gm::Scn sc = dev_scene(scene);
    // the pose kernels hold more registers: a chosen tiling may need fewer shards to stay co-resident
    if (!ctx->forced && (st = gm::fit_coresident(ctx, t, sc, ag, pr))) return st;
    gm::Out o{out->traj, out->cost, out->min_clear, out->best, rot, arm ? joints : nullptr};
    return gm::launch_rollout(ctx, sc, ag, pr, o, nullptr, t, static_cast<hipStream_t>(stream));
}

}  // namespace

gmapp_status gmapp_plan_loop(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                             const gmapp_query *query, const gmapp_params *params, const gmapp_loop_config *cfg,
                             const gmapp_loop_outputs *out, void *stream)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if ((st = check_scene(ctx, scene)) || (st = check_agents(ctx, agents)) || (st = check_params(ctx, params, true)))
        return st;
    if ((st = check_query(ctx, query))) return st;
    if (!cfg) return fail(ctx, GMAPP_EINVAL, "loop config is NULL");
    if (cfg->n_cycles < 1) return fail(ctx, GMAPP_EINVAL, "n_cycles must be >= 1");
    if (cfg->ctrl_steps < 1) return fail(ctx, GMAPP_EINVAL, "ctrl_steps must be >= 1");
    if (!finite(cfg->ctrl_dt) || !(cfg->ctrl_dt > 0.0f)) return fail(ctx, GMAPP_EINVAL, "ctrl_dt must be finite and > 0");
    if (agents->n_agents < 1) return fail(ctx, GMAPP_EINVAL, "the planning loop needs at least one agent");
    if (scene->n_seg > gm::kMaxControlSegments)
        return fail(ctx, GMAPP_ECAPACITY, "the control steps take at most %d segments", gm::kMaxControlSegments);
    if (!out || !out->robot || !out->best || !out->cost || !out->n_switches)
        return fail(ctx, GMAPP_EINVAL, "loop outputs robot, best, cost and n_switches must be non-NULL");
    if ((long long)cfg->n_cycles * cfg->ctrl_steps > (long long)INT32_MAX)
        return fail(ctx, GMAPP_ECAPACITY, "n_cycles x ctrl_steps exceeds 2^31 - 1");
    gm::Tiling t = tiling_for(ctx, scene->n_points, agents->n_agents, params->n_steps, scene->n_seg, params->cutoff);
    return gm::launch_plan_loop(ctx, dev_scene(scene), dev_agents(agents), dev_params(params, query), t, *cfg, *out,
                                static_cast<hipStream_t>(stream));
}

gmapp_status gmapp_control_force(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                                 const int32_t *agent, const float *state, float t, const gmapp_params *params,
                                 float *f_r, float *rho_min, void *stream)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if ((st = check_scene(ctx, scene)) || (st = check_agents(ctx, agents)) || (st = check_params(ctx, params, false)))
        return st;
    if (!agent || !state || !f_r) return fail(ctx, GMAPP_EINVAL, "agent, state and f_r must be non-NULL");
    if (scene->n_seg > gm::kMaxControlSegments)
        return fail(ctx, GMAPP_ECAPACITY, "the control query takes at most %d segments", gm::kMaxControlSegments);
    if (!finite(t)) return fail(ctx, GMAPP_EINVAL, "t must be finite");
    return gm::launch_control_force(ctx, dev_scene(scene), dev_agents(agents), dev_params(params, nullptr), agent,
                                    state, t, f_r, rho_min, static_cast<hipStream_t>(stream));
}

gmapp_status gmapp_depth_to_points(gmapp_ctx *ctx, const float *depth, int32_t w, int32_t h, const float K[4],
                                   const float T_wc[12], float *x, float *y, float *z, void *stream)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if (w < 0 || h < 0) return fail(ctx, GMAPP_EINVAL, "image size must be >= 0");
    if ((long long)w * h > (long long)INT32_MAX) return fail(ctx, GMAPP_ECAPACITY, "image exceeds 2^31 - 1 pixels");
    if (!K || !T_wc) return fail(ctx, GMAPP_EINVAL, "K and T_wc must be non-NULL");
    for (int i = 0; i < 4; ++i)
        if (!finite(K[i])) return fail(ctx, GMAPP_EINVAL, "intrinsics must be finite");
    if (K[0] == 0.f || K[1] == 0.f) return fail(ctx, GMAPP_EINVAL, "focal lengths must be non-zero");
    gm::Mat34 T;
    for (int i = 0; i < 12; ++i) {
        if (!finite(T_wc[i])) return fail(ctx, GMAPP_EINVAL, "T_wc must be finite");
        T.r[i] = T_wc[i];
    }
    if ((long long)w * h > 0 && (!depth || !x || !y || !z))
        return fail(ctx, GMAPP_EINVAL, "depth and output pointers must be non-NULL");
    return gm::launch_depth_to_points(ctx, depth, w, h, K, T, x, y, z, static_cast<hipStream_t>(stream));
}

gmapp_status gmapp_depth_to_points_batch(gmapp_ctx *ctx, const float *depth, int32_t n_frames, int32_t w, int32_t h,
                                         const float K[4], const float *T_wc, float *x, float *y, float *z,
                                         void *stream)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if (w < 0 || h < 0 || n_frames < 0) return fail(ctx, GMAPP_EINVAL, "image size and frame count must be >= 0");
    if ((long long)w * h * n_frames > (1ll << 40)) return fail(ctx, GMAPP_ECAPACITY, "more than 2^40 pixels");
    if ((long long)w * h > (long long)INT32_MAX) return fail(ctx, GMAPP_ECAPACITY, "image exceeds 2^31 - 1 pixels");
    if (!K) return fail(ctx, GMAPP_EINVAL, "K must be non-NULL");
    for (int i = 0; i < 4; ++i)
        if (!finite(K[i])) return fail(ctx, GMAPP_EINVAL, "intrinsics must be finite");
    if (K[0] == 0.f || K[1] == 0.f) return fail(ctx, GMAPP_EINVAL, "focal lengths must be non-zero");
    if ((long long)w * h * n_frames > 0 && (!depth || !T_wc || !x || !y || !z))
        return fail(ctx, GMAPP_EINVAL, "depth, poses and output pointers must be non-NULL");
    return gm::launch_depth_to_points_batch(ctx, depth, n_frames, w, h, K, T_wc, x, y, z,
                                            static_cast<hipStream_t>(stream));
}

gmapp_status gmapp_voxel_downsample(gmapp_ctx *ctx, const float *x, const float *y, const float *z, int64_t n,
                                    float voxel, const float lo[3], const int32_t dims[3], int32_t min_count,
                                    float *ox, float *oy, float *oz, int64_t capacity, int64_t *n_out_dev,
                                    void *stream)
{
    return gmapp_voxel_downsample_filtered(ctx, x, y, z, n, voxel, lo, dims, min_count, nullptr, 0, ox, oy, oz,
                                           capacity, n_out_dev, stream);
}

gmapp_status gmapp_voxel_downsample_filtered(gmapp_ctx *ctx, const float *x, const float *y, const float *z,
                                             int64_t n, float voxel, const float lo[3], const int32_t dims[3],
                                             int32_t min_count, const float *robot_spheres, int32_t n_spheres,
                                             float *ox, float *oy, float *oz, int64_t capacity, int64_t *n_out_dev,
                                             void *stream)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if (n < 0 || capacity < 0) return fail(ctx, GMAPP_EINVAL, "n and capacity must be >= 0");
    if (n > 0 && (!x || !y || !z)) return fail(ctx, GMAPP_EINVAL, "input points must be non-NULL");
    if (capacity > 0 && (!ox || !oy || !oz)) return fail(ctx, GMAPP_EINVAL, "output arrays must be non-NULL");
    if (!n_out_dev) return fail(ctx, GMAPP_EINVAL, "n_out_dev must be non-NULL");
    gm::VoxGrid g;
    if ((st = voxel_grid(ctx, voxel, lo, dims, min_count, robot_spheres, n_spheres, g))) return st;
    return gm::launch_voxel_downsample(ctx, x, y, z, n, nullptr, g, (unsigned)min_count, ox, oy, oz, capacity,
                                       reinterpret_cast<long long *>(n_out_dev), static_cast<hipStream_t>(stream));
}

gmapp_status gmapp_voxel_downsample_noalloc(gmapp_ctx *ctx, const float *x, const float *y, const float *z,
                                            int64_t n, float voxel, const float lo[3], const int32_t dims[3],
                                            int32_t min_count, float *ox, float *oy, float *oz, int64_t capacity,
                                            int64_t *n_out_dev, void *stream)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if (n < 0 || capacity < 0) return fail(ctx, GMAPP_EINVAL, "n and capacity must be >= 0");
    if (n > 0 && (!x || !y || !z)) return fail(ctx, GMAPP_EINVAL, "input points must be non-NULL");
    if (capacity > 0 && (!ox || !oy || !oz)) return fail(ctx, GMAPP_EINVAL, "output arrays must be non-NULL");
    if (!n_out_dev) return fail(ctx, GMAPP_EINVAL, "n_out_dev must be non-NULL");
    gm::VoxGrid g;
    if ((st = voxel_grid(ctx, voxel, lo, dims, min_count, nullptr, 0, g))) return st;
    return gm::launch_voxel_downsample_static(ctx, x, y, z, n, g, (unsigned)min_count, ox, oy, oz, capacity,
                                              reinterpret_cast<long long *>(n_out_dev),
                                              static_cast<hipStream_t>(stream));
}

gmapp_status gmapp_depth_to_voxels(gmapp_ctx *ctx, const float *depth, int32_t n_frames, int32_t w, int32_t h,
                                   const float K[4], const float *T_wc, float voxel, const float lo[3],
                                   const int32_t dims[3], int32_t min_count, const float *robot_spheres,
                                   int32_t n_spheres, float *ox, float *oy, float *oz, int64_t capacity,
                                   int64_t *n_out_dev, void *stream)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if (w < 0 || h < 0 || n_frames < 0) return fail(ctx, GMAPP_EINVAL, "image size and frame count must be >= 0");
    if ((long long)w * h * n_frames > (1ll << 40)) return fail(ctx, GMAPP_ECAPACITY, "more than 2^40 pixels");
    if ((long long)w * h > (long long)INT32_MAX) return fail(ctx, GMAPP_ECAPACITY, "image exceeds 2^31 - 1 pixels");
    if (!K) return fail(ctx, GMAPP_EINVAL, "K must be non-NULL");
    for (int i = 0; i < 4; ++i)
        if (!finite(K[i])) return fail(ctx, GMAPP_EINVAL, "intrinsics must be finite");
    if (K[0] == 0.f || K[1] == 0.f) return fail(ctx, GMAPP_EINVAL, "focal lengths must be non-zero");
    const long long n = (long long)w * h * n_frames;
    if (n > 0 && (!depth || !T_wc)) return fail(ctx, GMAPP_EINVAL, "depth and poses must be non-NULL");
    if (capacity < 0) return fail(ctx, GMAPP_EINVAL, "capacity must be >= 0");
    if (capacity > 0 && (!ox || !oy || !oz)) return fail(ctx, GMAPP_EINVAL, "output arrays must be non-NULL");
    if (!n_out_dev) return fail(ctx, GMAPP_EINVAL, "n_out_dev must be non-NULL");
    gm::VoxGrid g;
    if ((st = voxel_grid(ctx, voxel, lo, dims, min_count, robot_spheres, n_spheres, g))) return st;
    gm::Cam cam{K[0], K[1], K[2], K[3], w, h, n_frames, T_wc};
    return gm::launch_voxel_downsample(ctx, depth, nullptr, nullptr, n, &cam, g, (unsigned)min_count, ox, oy, oz,
                                       capacity, reinterpret_cast<long long *>(n_out_dev),
                                       static_cast<hipStream_t>(stream));
}

gmapp_status gmapp_rollout_backward(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                                    const gmapp_query *query, const gmapp_params *params, const float *grad_total,
                                    int32_t ckpt_every, float *g_k_a, float *g_d_a, float *g_k_f, float *g_omega,
                                    void *stream)
{
    gmapp_status st = check_ctx(ctx);
    if (st) return st;
    if ((st = check_scene(ctx, scene)) || (st = check_agents(ctx, agents)) || (st = check_params(ctx, params, true)))
        return st;
    if ((st = check_query(ctx, query))) return st;
    if (ckpt_every < 1 || ckpt_every > 1024) return fail(ctx, GMAPP_EINVAL, "ckpt_every must be in [1, 1024]");
    if (scene->n_seg > gm::kMaxSegments)
        return fail(ctx, GMAPP_ECAPACITY, "at most %d segments are supported", gm::kMaxSegments);
    if (agents->heuristic)
        return fail(ctx, GMAPP_EINVAL, "the adjoint covers the rotation-vector circular field only (heuristic = NULL)");
    if (agents->n_agents > 0 && (!grad_total || !g_k_a || !g_d_a || !g_k_f || !g_omega))
        return fail(ctx, GMAPP_EINVAL, "grad_total and the gradient outputs must be non-NULL");
    return gm::launch_adjoint(ctx, dev_scene(scene), dev_agents(agents), dev_params(params, query), grad_total,
                              ckpt_every, g_k_a, g_d_a, g_k_f, g_omega, static_cast<hipStream_t>(stream));
}

}  // extern "C"

