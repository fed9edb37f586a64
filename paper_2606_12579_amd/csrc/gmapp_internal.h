// Internal declarations shared by the library's translation units (kernels,
// context, perception, adjoint).  Not installed; the public ABI is include/gmapp.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/gmapp.h"

namespace gm {

// ---------------------------------------------------------------- device views
struct Scn {
    const float *x, *y, *z;
    long long n_cap;          // N_O (or capacity when n_dev != nullptr)
    const long long *n_dev;   // device-resident N_O or nullptr
    float r_obs;
    int n_seg;
    const int *seg_begin;
    const float *seg_vel;
};

struct Agt {
    const float *k_a, *d_a, *k_f, *r_d, *r_a, *omega;
    int n;
};

struct Prm {
    float dt, inv_mass, eps, r_cost;
    float w0, w1, w2, w3;
    float a_max, alpha, band;
    int n_steps, cutoff;
    float p0[3], v0[3], goal[3];
    int incumbent;
    float t0;
};

struct Out {
    float *traj, *cost, *min_clear;
    int *best;
};

// teacher-forced single-step mode (force probe)
struct Probe {
    const float *p, *v;
    float t;
    float *f_r, *rho_min;
};

// cross-workgroup exchange area (part of the context arena)
struct Xch {
    unsigned long long *partial;  // [2][wave groups][S][AW][4] words: Fx, Fy, Fz, min r2, each | step tag << 32
    unsigned *flags;     // spare counters (zero between launches)
    unsigned *done;      // [1]       finished-workgroup counter, zero between launches
    unsigned *status;    // [1]       watchdog flag, zero between launches
    int S, G;
};

// camera-to-world transform, row-major 3x4 [R | t]
struct Mat34 {
    float r[12];
};

// voxel lattice over the workspace box: cells of size `voxel` from `lo`
struct VoxGrid {
    float lo[3];
    float voxel;
    int dims[3];
};

struct Tiling {
    int A, W, S;      // agents per group, waves per workgroup, shards
    int tile;         // points per tile (streamed layout)
    int layout;       // 0 auto, 1 resident, 2 streamed tiles
    int wg;           // 0: every wave is a group; 1: the workgroup is one group
};

// ---------------------------------------------------------------- sizes
constexpr int kMaxShards = 64;
constexpr int kMaxGather = 256;                       // shards x agents per wave (LDS gather)
constexpr int kMaxSegments = 1024;                    // moving segments per scene
constexpr int kMaxGroups = 4096;                      // agent groups per launch
constexpr int kMaxWorkgroups = 65536;
constexpr size_t kCounterWords = (size_t)kMaxGroups * 16;
constexpr size_t kSyncWords = kCounterWords + 64;     // counters + done + status (+ pad)
constexpr size_t kXchgBytes = (size_t)16 << 20;       // rollout exchange area

}  // namespace gm

// ---------------------------------------------------------------- context
struct gmapp_ctx {
    int device = 0;
    int n_cu = 0;
    int lds_per_cu = 0;
    char *arena = nullptr;        // device arena
    size_t arena_bytes = 0;
    unsigned *sync = nullptr;     // kSyncWords, kept zero between launches
    unsigned long long *xchg = nullptr;  // rollout exchange words (kXchgBytes), kept zero between launches
    char *scratch = nullptr;      // remainder of the arena (voxel grids, checkpoints, work tables)
    size_t scratch_bytes = 0;
    bool forced = false;
    gmapp_tiling forced_tiling{0, 0, 0, 0, 0, 0};
    std::string err;
};

namespace gm {

inline gmapp_status fail(gmapp_ctx *ctx, gmapp_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return st;
}

inline gmapp_status hip_fail(gmapp_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, GMAPP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define GM_HIP(ctx, call)                                   \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return gm::hip_fail(ctx, e_, #call); \
    } while (0)

// rollout launcher (rollout.hip)
gmapp_status launch_rollout(gmapp_ctx *ctx, const Scn &sc, const Agt &ag, const Prm &pr, const Out &out,
                            const Probe *probe, const Tiling &t, hipStream_t stream);
Tiling choose_tiling(const gmapp_ctx *ctx, long long n_points, int n_agents, int n_steps, int n_seg, int cutoff);

// adjoint (adjoint.hip)
gmapp_status launch_adjoint(gmapp_ctx *ctx, const Scn &sc, const Agt &ag, const Prm &pr, const float *grad_total,
                            int ckpt_every, float *g_ka, float *g_da, float *g_kf, float *g_om, hipStream_t stream);

// perception (perception.hip)
gmapp_status launch_depth_to_points(gmapp_ctx *ctx, const float *depth, int w, int h, const float K[4],
                                    const Mat34 &T, float *x, float *y, float *z, hipStream_t stream);
size_t voxel_workspace_bytes(long long cells);
gmapp_status launch_voxel_downsample(gmapp_ctx *ctx, const float *x, const float *y, const float *z, long long n,
                                     const VoxGrid &g, unsigned min_count, float *ox, float *oy, float *oz,
                                     long long capacity, long long *n_out_dev, hipStream_t stream);
gmapp_status check_tiling(gmapp_ctx *ctx, const Tiling &t, long long n_points, int n_seg, int cutoff);
size_t rollout_lds_bytes(const Tiling &t, long long n_points, int n_seg);

}  // namespace gm
