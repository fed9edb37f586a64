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
    float4 *partial;     // [2][G][S][A]
    unsigned *flags;     // [G * S]   step counters, zero between launches
    unsigned *done;      // [1]       finished-workgroup counter, zero between launches
    unsigned *status;    // [1]       watchdog flag, zero between launches
    int S, G;
};

struct Tiling {
    int A, W, S, tile;
};

// ---------------------------------------------------------------- sizes
constexpr int kMaxShards = 64;
constexpr int kMaxWorkgroups = 65536;
constexpr size_t kSyncWords = kMaxWorkgroups + 64;   // flags + done + status (+ pad)

}  // namespace gm

// ---------------------------------------------------------------- context
struct gmapp_ctx {
    int device = 0;
    int n_cu = 0;
    int lds_per_cu = 0;
    char *arena = nullptr;        // device arena
    size_t arena_bytes = 0;
    unsigned *sync = nullptr;     // kSyncWords, kept zero between launches
    char *scratch = nullptr;      // remainder of the arena (partials, voxel grids, checkpoints)
    size_t scratch_bytes = 0;
    bool forced = false;
    gmapp_tiling forced_tiling{0, 0, 0, 0};
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
gmapp_status check_tiling(gmapp_ctx *ctx, const Tiling &t, int n_agents, int cutoff);

}  // namespace gm
