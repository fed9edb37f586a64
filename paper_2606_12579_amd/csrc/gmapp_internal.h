// Internal declarations shared by the library's translation units (kernels,
// context, perception, adjoint).  Not installed; the public ABI is include/gmapp.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstddef>
#include <cstdio>
#include <map>
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
    const int *heur;          // per-agent heuristic or nullptr (all rotation-vector field)
    const float *k_r = nullptr, *d_r = nullptr, *i_r = nullptr;   // 6-D pose agents: rotational gains
};

struct Prm {
    float dt, inv_mass, eps, r_cost;
    float w0, w1, w2, w3;
    float a_max, alpha, band;
    int n_steps, cutoff;
    float p0[3], v0[3], goal[3];
    int incumbent;
    float t0;
    float q0[4] = {1.f, 0.f, 0.f, 0.f};   // 6-D pose agents: start rotor (w, x, y, z)
    float om0[3] = {0.f, 0.f, 0.f};       // start angular velocity (body frame)
    float qg[4] = {1.f, 0.f, 0.f, 0.f};   // goal rotor
    const float *arm_links = nullptr;   // arm agents: device [arm_n + 1][7] link transforms
    const float *arm_q0 = nullptr;      // device [arm_n] start joint angles
    int arm_n = 0;
    float arm_lam2 = 0.f;               // damping lambda^2 of the pseudo-inverse
    const float *start = nullptr;   // device [6] p0, v0 in place of p0, v0 (closed loop) or nullptr
    const int *inc_dev = nullptr;   // device incumbent in place of `incumbent` (closed loop) or nullptr
};

struct Out {
    float *traj, *cost, *min_clear;
    int *best;
    float *rot = nullptr;     // 6-D pose agents: [N_a][N_k + 1][4] rotors, or nullptr
    float *joints = nullptr;  // arm agents: [N_a][N_k + 1][n_joints] joint angles, or nullptr
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
    unsigned *status;    // [1]       0 ok, 1 a wait ran out of time, 2 aborted by the host; zero between launches;
                         //           followed by the wait settings (kWaitLimitWord, kAbortAddrWord)
    int S, G;
    int fine;            // 1: check the wait limit from a wait's first failed poll (limits below 1 ms)
};
// wait settings after the status word, set by the host: the longest wait without progress
// (u64, 100 MHz real-time ticks) and the device address of the host's abort word (u64)
constexpr int kWaitLimitWord = 8;
constexpr int kAbortAddrWord = 10;

// camera-to-world transform, row-major 3x4 [R | t]
struct Mat34 {
    float r[12];
};

// voxel lattice over the workspace box: cells of size `voxel` from `lo`
struct VoxGrid {
    float lo[3];
    float voxel;
    int dims[3];
    const float *excl = nullptr;  // robot self-filter: [n_excl][4] sphere centres and radii, or nullptr
    int n_excl = 0;
    double lod[3] = {0, 0, 0};    // lo, voxel and 1 / voxel in FP64, and 1 / voxel in FP32 (set by the launcher)
    double sd = 0, inv_s = 0;
    float inv_s32 = 0;
};

// pinhole intrinsics and the frames of a fused depth -> voxel pass
struct Cam {
    float fx, fy, cx, cy;
    int w, h, n_frames;
    const float *T;               // device [n_frames][12] camera-to-world poses
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
// sync words [0, kCounterWords): per-job completion counters of the batched launch;
// kCounterWords: rollout done counter; +16: watchdog status; +24..27: wait settings; +32, +33: batch queue
constexpr size_t kBatchQueueWord = kCounterWords + 32;
constexpr int kMaxBatchJobs = 16384;
constexpr int kBatchWaves = 8;                        // waves per workgroup of the batched kernel
constexpr int kBatchMaxSegments = 64;                 // moving segments per scene in a batched launch
constexpr int kStateFloats = 28;                      // resumable agent state, floats per agent

// one job of a batched launch (device copy in the job table)
struct BatchJob {
    Scn sc;
    Agt ag;
    Prm pr;
    Out out;
    float *state;       // [N_a][kStateFloats]
    int k_begin, k_end; // steps [k_begin, k_end) of 1..N_k run in this launch
    int item_base;      // first work item of the job
    int n_items;
    int wg_items;       // 0: every wave is an agent group of aw agents; 1: the workgroup holds aw agents
    int aw;             // agents per group: 1, 2, 4, 8
    const unsigned *cancel;   // device-readable word (mapped host memory) or null: nonzero cancels the job
};

struct BatchTable {
    int n_jobs, n_items, pad[2];
    BatchJob jobs[1];   // n_jobs entries (the table is allocated for its capacity)
};
constexpr size_t batch_table_bytes(int n_jobs)
{
    return offsetof(BatchTable, jobs) + (size_t)(n_jobs > 0 ? n_jobs : 1) * sizeof(BatchJob);
}

struct BatchLay {
    int cap;            // LDS points (tile size; worlds up to cap points stay resident)
    int runs_cap;       // segment runs
};

struct BatchLaunch {
    const void *fn;
    unsigned grid;
    int block;
    size_t shm;
    BatchLay lay;
    unsigned *queue, *done;
    const unsigned *abort;   // the context's abort word (device address of pinned host memory)
};

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
    std::map<unsigned long long, gmapp_tiling> tuned;   // autotuned rollout tilings by shape class
    bool batch_forced = false;
    gmapp_batch_tuning batch_forced_tuning{0, 0, 0, 0};
    bool batch_tuned = false;
    gmapp_batch_tuning batch_tuned_tuning{0, 0, 0, 0};
    unsigned *vgrid = nullptr;    // voxel grid (occupancy bytes or counts), all zero between calls
    size_t vgrid_words = 0;
    unsigned *vbsum = nullptr;    // voxel pass: per-block occupied-cell counts, then per-block dirty bytes
    size_t vbsum_blocks = 0;      // blocks the table holds (the dirty bytes start after that many counts)
    unsigned *static_grid = nullptr;  // device address of the static voxel grid on this device
    unsigned long long watchdog_ticks = 400000000ull;   // per-wait limit of the exchanges (4 s)
    unsigned *abort_host = nullptr;   // pinned, coherent host word: nonzero ends every exchange wait
    unsigned *abort_word = nullptr;   // its device address
    void *tab_host = nullptr;     // pinned staging of the batched job table
    size_t tab_host_bytes = 0;
    hipEvent_t tab_copied = nullptr;   // recorded after the last table copy
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

// the context's exchange area and status word for a sharded launch
inline Xch make_xch(gmapp_ctx *ctx, int S, int G)
{
    Xch xc;
    xc.partial = ctx->xchg;
    xc.flags = ctx->sync;
    xc.done = ctx->sync + kCounterWords;
    xc.status = ctx->sync + kCounterWords + 16;
    xc.S = S;
    xc.G = G;
    xc.fine = ctx->watchdog_ticks < 100000ull ? 1 : 0;
    return xc;
}

// rollout launcher (rollout.hip)
gmapp_status launch_rollout(gmapp_ctx *ctx, const Scn &sc, const Agt &ag, const Prm &pr, const Out &out,
                            const Probe *probe, const Tiling &t, hipStream_t stream);
Tiling choose_tiling(const gmapp_ctx *ctx, long long n_points, int n_agents, int n_steps, int n_seg, int cutoff);
gmapp_status fit_coresident(gmapp_ctx *ctx, Tiling &t, const Scn &sc, const Agt &ag, const Prm &pr);

constexpr int kMaxArmJoints = 7;                      // serial chains of arm agents
constexpr int kMaxArmAgentsPerGroup = 8;              // arm agents hold a lane per joint in a wave

// closed planning loop and the control query (control.hip)
constexpr int kMaxControlSegments = 128;
gmapp_status launch_plan_loop(gmapp_ctx *ctx, const Scn &sc, const Agt &ag, const Prm &pr0, const Tiling &t,
                              const gmapp_loop_config &cfg, const gmapp_loop_outputs &o, hipStream_t stream);
gmapp_status launch_control_force(gmapp_ctx *ctx, const Scn &sc, const Agt &ag, const Prm &pr, const int *agent,
                                  const float *state, float t, float *f_r, float *rho_min, hipStream_t stream);

// adjoint (adjoint.hip)
gmapp_status launch_adjoint(gmapp_ctx *ctx, const Scn &sc, const Agt &ag, const Prm &pr, const float *grad_total,
                            int ckpt_every, float *g_ka, float *g_da, float *g_kf, float *g_om, hipStream_t stream);

// perception (perception.hip)
gmapp_status launch_depth_to_points(gmapp_ctx *ctx, const float *depth, int w, int h, const float K[4],
                                    const Mat34 &T, float *x, float *y, float *z, hipStream_t stream);
gmapp_status launch_depth_to_points_batch(gmapp_ctx *ctx, const float *depth, int n_frames, int w, int h,
                                          const float K[4], const float *T_dev, float *x, float *y, float *z,
                                          hipStream_t stream);
// the voxel pass over points (x, y, z) or, with cam != nullptr, over the back-projected
// pixels of cam's depth frames (x = depth)
gmapp_status launch_voxel_downsample(gmapp_ctx *ctx, const float *x, const float *y, const float *z, long long n,
                                     const Cam *cam, const VoxGrid &g, unsigned min_count, float *ox, float *oy,
                                     float *oz, long long capacity, long long *n_out_dev, hipStream_t stream);
// the same pass on the statically sized grid (no allocation): grids of at most kStaticCells cells
constexpr long long kStaticCells = 1ll << 21;
gmapp_status static_scratch_init(gmapp_ctx *ctx);
gmapp_status launch_voxel_downsample_static(gmapp_ctx *ctx, const float *x, const float *y, const float *z,
                                            long long n, const VoxGrid &g, unsigned min_count, float *ox,
                                            float *oy, float *oz, long long capacity, long long *n_out_dev,
                                            hipStream_t stream);
gmapp_status check_tiling(gmapp_ctx *ctx, const Tiling &t, long long n_points, int n_seg, int cutoff);
size_t rollout_lds_bytes(const Tiling &t, long long n_points, int n_seg);

// shape class of the rollout autotuner's cache: N_O and N_k rounded up to powers of two
inline unsigned long long tune_key(long long n_points, int n_agents, int n_steps, int n_seg, int cutoff)
{
    auto lg = [](long long v) {
        unsigned long long b = 0;
        while ((1ll << b) < v && b < 62) ++b;
        return b;
    };
    return (lg(n_points) << 56) | (lg(n_steps) << 48) | ((unsigned long long)(n_seg > 0) << 47) |
           ((unsigned long long)(cutoff & 1) << 46) | (unsigned long long)(unsigned)n_agents;
}

// batched launch (batch.hip)
size_t batch_lds_bytes(const BatchLay &lay);
gmapp_status batch_launch_shape(gmapp_ctx *ctx, const BatchLay &lay, int wg_per_cu, BatchLaunch &out);
gmapp_status launch_batch(gmapp_ctx *ctx, const BatchTable *tab_dev, const BatchLaunch &l, hipStream_t stream);

// argument checks and device views shared by the entry points (api.hip)
gmapp_status check_ctx(gmapp_ctx *ctx);
gmapp_status check_scene(gmapp_ctx *ctx, const gmapp_scene *sc);
gmapp_status check_agents(gmapp_ctx *ctx, const gmapp_agents *ag);
gmapp_status check_params(gmapp_ctx *ctx, const gmapp_params *p, bool need_steps);
gmapp_status check_query(gmapp_ctx *ctx, const gmapp_query *q);
Scn dev_scene(const gmapp_scene *sc);
Agt dev_agents(const gmapp_agents *ag);
Prm dev_params(const gmapp_params *p, const gmapp_query *q);

}  // namespace gm
