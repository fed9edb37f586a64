// Host side of the forward rollout: tiling checks, LDS layout, launch and the
// homogeneous-field kernel instantiations.  The kernel itself, its work
// decomposition and arithmetic are in rollout_kernel.h.
#include "rollout_kernel.h"

#include <algorithm>
#include <cmath>

namespace gm {

using namespace dev;

namespace {

// agent kind of a launch: 0 point masses, 1 pose agents, 2 arm agents
int kind_of(const Agt &ag, const Prm &pr)
{
    return ag.k_r == nullptr ? 0 : (pr.arm_links != nullptr ? 2 : 1);
}

KFn pick_kernel(int AW, int W, bool wg, int cut, bool probe, bool het, int kind)
{
    if (kind == 2) return probe ? nullptr : pick_kernel_arm(AW, W, wg, cut);
    if (kind == 1) return probe ? nullptr : pick_kernel_pose(AW, W, wg, cut);
    return het ? pick_kernel_het(AW, W, wg, cut, probe) : pick_kernel_t<false, 0>(AW, W, wg, cut, probe);
}

}  // namespace

__global__ void k_write_best(int *best, int v)
{
    best[0] = v;
}

// ---------------------------------------------------------------- host side
namespace {

constexpr size_t kLdsBudget = 160 * 1024;

}  // namespace

// Layout for a tiling: the whole shard resident in LDS when it fits (or when
// forced), else streamed tiles of t.tile points.
Lay make_layout(const Tiling &t, long long n_points, int n_seg)
{
    Lay l;
    l.runs_cap = 2 * n_seg + 2;
    const long long per = (n_points + t.S - 1) / t.S;     // largest shard
    l.resident = t.layout == 2 ? 0 : 1;
    l.cap = (int)std::min<long long>(std::max<long long>(per, 1), 1 << 24);
    if (t.layout == 0 && lds_plan(l, t.W, t.wg ? t.W : 1, t.A, t.S).total > kLdsBudget) l.resident = 0;
    if (!l.resident) l.cap = t.tile > 0 ? t.tile : 4096;
    return l;
}

size_t rollout_lds_bytes(const Tiling &t, long long n_points, int n_seg)
{
    Lay l = make_layout(t, n_points, n_seg);
    return lds_plan(l, t.W, t.wg ? t.W : 1, t.A, t.S).total;
}

gmapp_status check_tiling(gmapp_ctx *ctx, const Tiling &t, long long n_points, int n_seg, int cutoff)
{
    if (!pick_kernel(t.A, t.W, t.wg != 0, cutoff, false, false, 0))
        return fail(ctx, GMAPP_EINVAL, "unsupported tiling: %d agents per %s with %d waves", t.A,
                    t.wg ? "workgroup" : "wave", t.W);
    if (t.S < 1 || t.S > kMaxShards) return fail(ctx, GMAPP_EINVAL, "shards must be in [1, %d]", kMaxShards);
    if (t.S > 1 && t.S * t.A > kMaxGather)
        return fail(ctx, GMAPP_EINVAL, "shards x agents per group must be <= %d", kMaxGather);
    if (t.tile != 0 && t.tile < 64) return fail(ctx, GMAPP_EINVAL, "tile_points must be >= 64");
    if (t.layout < 0 || t.layout > 2) return fail(ctx, GMAPP_EINVAL, "layout must be 0, 1 or 2");
    if (n_seg > kMaxSegments) return fail(ctx, GMAPP_ECAPACITY, "at most %d segments are supported", kMaxSegments);
    if (rollout_lds_bytes(t, n_points, n_seg) > kLdsBudget)
        return fail(ctx, GMAPP_ECAPACITY, "tiling does not fit in LDS (%s layout)",
                    make_layout(t, n_points, n_seg).resident ? "resident" : "streamed");
    return GMAPP_OK;
}

Tiling choose_tiling(const gmapp_ctx *ctx, long long n_points, int n_agents, int n_steps, int n_seg, int cutoff)
{
    (void)n_steps; (void)cutoff;
    const int cus = ctx && ctx->n_cu > 0 ? ctx->n_cu : 256;
    // shard count: the smallest power of two that covers the chip with an
    // LDS-resident shard, within the co-residency a cooperative launch needs
    auto shard = [&](Tiling t) {
        const int per_wg = t.wg ? t.A : t.A * t.W;
        const long long G = std::max(1, (n_agents + per_wg - 1) / per_wg);
        int best = 1;
        for (int S = 1; S <= kMaxShards && S * t.A <= kMaxGather; S *= 2) {
            if (S > 1 && n_points / S < 64) break;
            Tiling u = t;
            u.S = S;
            const Lay l = make_layout(u, n_points, n_seg);
            const size_t lds = lds_plan(l, t.W, t.wg ? t.W : 1, t.A, S).total;
            const long long per_cu = std::min<long long>(kLdsBudget / std::max<size_t>(lds, 1), 16 / t.W);
            if (S > 1 && G * S > per_cu * cus) break;
            best = S;
            if (G * S >= cus && l.resident) break;
        }
        t.S = best;
        return t;
    };
    // many agents: every wave is its own group (no barriers in the step loop);
    // few agents: workgroup-wide groups keep the shard count, hence the exchange, small
    if ((long long)n_agents >= (long long)cus * 4) {
        Tiling t{1, 4, 1, 4096, 0, 0};
        while (t.A < 8 && (long long)n_agents >= (long long)cus * t.W * t.A * 2) t.A *= 2;
        return shard(t);
    }
    Tiling t{1, 8, 1, 4096, 0, 1};
    while (t.A < 8 && (long long)n_agents > (long long)cus * t.A / 4) t.A *= 2;
    return shard(t);
}

// Halve the shard count of a chosen (not forced) tiling until the kernel that
// will run, with its own register and LDS needs, fits the cooperative launch.
gmapp_status fit_coresident(gmapp_ctx *ctx, Tiling &t, const Scn &sc, const Agt &ag, const Prm &pr)
{
    if (ag.n == 0) return GMAPP_OK;
    KFn fn = pick_kernel(t.A, t.W, t.wg != 0, pr.cutoff, false, ag.heur != nullptr, kind_of(ag, pr));
    if (!fn) return GMAPP_OK;
    const int per_wg = t.wg ? t.A : t.A * t.W;
    const long long G = (ag.n + per_wg - 1) / per_wg;
    while (t.S > 1) {
        const Lay lay = make_layout(t, sc.n_cap, sc.n_seg);
        const size_t shm = lds_plan(lay, t.W, t.wg ? t.W : 1, t.A, t.S).total;
        int per_cu = 0;
        GM_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
        GM_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(fn),
                                                                 64 * t.W, shm));
        if ((long long)per_cu * ctx->n_cu >= (G * t.S + 7) / 8 * 8) break;
        t.S /= 2;
    }
    return GMAPP_OK;
}

gmapp_status launch_rollout(gmapp_ctx *ctx, const Scn &sc, const Agt &ag, const Prm &pr, const Out &out,
                            const Probe *probe, const Tiling &t, hipStream_t stream)
{
    gmapp_status st = check_tiling(ctx, t, sc.n_cap, sc.n_seg, pr.cutoff);
    if (st) return st;
    const bool is_probe = probe != nullptr;
    if (ag.n == 0) {
        if (!is_probe) hipLaunchKernelGGL(k_write_best, dim3(1), dim3(1), 0, stream, out.best, -1);
        GM_HIP(ctx, hipGetLastError());
        return GMAPP_OK;
    }
    KFn fn = pick_kernel(t.A, t.W, t.wg != 0, pr.cutoff, is_probe, ag.heur != nullptr, kind_of(ag, pr));
    if (!fn) {
        if (is_probe) return fail(ctx, GMAPP_EINVAL, "6-D pose agents have no teacher-forced form");
        return fail(ctx, GMAPP_EINVAL, "arm agents take at most %d agents per group (tiling has %d)",
                    kMaxArmAgentsPerGroup, t.A);
    }
    const int per_wg = t.wg ? t.A : t.A * t.W;
    const int gpw = t.wg ? 1 : t.W;
    const int G = (ag.n + per_wg - 1) / per_wg;
    const long long nwg_real = (long long)G * t.S;
    long long nwg = nwg_real;
    if (t.S > 1) nwg = (nwg + 7) / 8 * 8;
    if (nwg > kMaxWorkgroups)
        return fail(ctx, GMAPP_ECAPACITY, "%lld workgroups exceed the limit %d", nwg, kMaxWorkgroups);
    const size_t need_partial = (size_t)2 * G * gpw * t.S * t.A * kSlotWords * sizeof(unsigned long long);
    if (t.S > 1 && need_partial > kXchgBytes)
        return fail(ctx, GMAPP_ECAPACITY, "exchange area needs %zu bytes, the context holds %zu", need_partial,
                    kXchgBytes);
    Xch xc = make_xch(ctx, t.S, G);
    Probe pb{};
    if (probe) pb = *probe;
    Lay lay = make_layout(t, sc.n_cap, sc.n_seg);
    const size_t shm = lds_plan(lay, t.W, t.wg ? t.W : 1, t.A, t.S).total;
    void *args[] = {(void *)&sc, (void *)&ag, (void *)&pr, (void *)&out, (void *)&pb, (void *)&xc, (void *)&lay};
    GM_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)shm));
    if (t.S > 1) {
        int per_cu = 0;
        GM_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(fn),
                                                                 64 * t.W, shm));
        if ((long long)per_cu * ctx->n_cu < nwg)
            return fail(ctx, GMAPP_ECAPACITY,
                        "sharded rollout needs %lld co-resident workgroups, the device holds %d x %d", nwg, per_cu,
                        ctx->n_cu);
        GM_HIP(ctx, hipLaunchCooperativeKernel(reinterpret_cast<const void *>(fn), dim3((unsigned)nwg),
                                               dim3(64 * t.W), args, (unsigned)shm, stream));
    } else {
        GM_HIP(ctx, hipLaunchKernel(reinterpret_cast<const void *>(fn), dim3((unsigned)nwg), dim3(64 * t.W), args,
                                    shm, stream));
    }
    return GMAPP_OK;
}

}  // namespace gm
