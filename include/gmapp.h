/*
 * gmapp.h -- C ABI of the MI355X (gfx950) multi-agent circular-field rollout
 * library: the data-parallel hot path of G-MAPP (Bishnoi et al., "G-MAPP:
 * GPU-accelerated Multi-Agent Planning and Perception for Reactive Motion
 * Generation").
 *
 * The calls follow the paper's problem statement (Sec. II): a sphere-world point
 * cloud S_W (Eq. 5), start and goal poses, N_a planning agents with their
 * parameters and a horizon of N_k steps go in; per-agent trajectories (Eq. 15),
 * costs (Eqs. 16-20) and the selected agent come out.
 *
 * Conventions for every entry point
 *  - Return value: GMAPP_OK (0) or a negative gmapp_status.  Argument checks
 *    happen on the host, before anything is enqueued; on error nothing is
 *    enqueued and gmapp_last_error() describes the problem.
 *  - Array arguments marked "device" are device pointers (hipMalloc or torch
 *    allocations on the context's device) owned by the caller; the library never
 *    frees or retains them past the call.  Arrays marked "host" are read during
 *    the call only.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and is
 *    complete once that stream is synchronised.  Calls on one context must be
 *    ordered (one stream at a time): the context's workspace is shared by them.
 *  - Layouts are C order, FP32 unless stated: points SoA x[N_O], y[N_O], z[N_O];
 *    per-agent scalars [N_a]; vectors [N_a][3].
 *  - A context is used by one host thread at a time; a server is thread-safe.
 */
#ifndef GMAPP_H
#define GMAPP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gmapp_status;
#define GMAPP_OK 0
#define GMAPP_EINVAL (-1)     /* invalid argument (nothing enqueued) */
#define GMAPP_ENOMEM (-2)     /* workspace or device memory exhausted */
#define GMAPP_EDEVICE (-3)    /* no usable device, or a HIP runtime error */
#define GMAPP_ECAPACITY (-4)  /* request exceeds a fixed capacity (grid residency, output capacity) */
#define GMAPP_ETIMEOUT (-5)   /* deadline passed, or an exchange wait stalled past the watchdog */
#define GMAPP_ECANCELLED (-6) /* request cancelled */

typedef struct gmapp_ctx gmapp_ctx;

/* Create a context on HIP device `device`.  `workspace_bytes` sizes the device
 * arena used for cross-workgroup exchange, voxel grids and adjoint checkpoints
 * (0 = 256 MiB).  The arena is allocated once here and freed by gmapp_destroy. */
gmapp_status gmapp_create(int32_t device, size_t workspace_bytes, gmapp_ctx **out);
void gmapp_destroy(gmapp_ctx *ctx);
/* Message for the last failing call on this context (never NULL). */
const char *gmapp_last_error(const gmapp_ctx *ctx);
/* Library version string, e.g. "gmapp 0.1 gfx950". */
const char *gmapp_version(void);

/* Sphere world S_W of Eq. (5): N_O sphere centres with one radius r_O.
 * Optional moving obstacles: the points are grouped into n_seg contiguous
 * segments (objects), seg_begin[s] .. seg_begin[s+1]-1, each translating with the
 * constant velocity seg_vel[s] over the horizon (sphere j sits at
 * p_j + t_k v_seg(j), t_k = t0 + (k-1) dt, see gmapp_query).  Points outside every
 * segment are static.
 * seg_begin must be non-decreasing with seg_begin[0] = 0 and
 * seg_begin[n_seg] = N_O; other tables give unspecified (but memory-safe) results. */
typedef struct {
    const float *x, *y, *z;       /* device [N_O] each */
    int64_t n_points;             /* N_O; with n_points_dev: the capacity of x, y, z */
    const int64_t *n_points_dev;  /* device [1] or NULL: actual N_O (<= n_points), e.g. from
                                     gmapp_voxel_downsample, read on the device (no host sync) */
    float r_obs;                  /* r_O >= 0 */
    int32_t n_seg;                /* 0 = static scene */
    const int32_t *seg_begin;     /* device [n_seg + 1] */
    const float *seg_vel;         /* device [n_seg][3], m/s */
} gmapp_scene;

/* Per-agent parameters (Alg. 1 inputs and the attractor of Eq. 7): circular-field
 * gain k_f, detection radius r_d, agent radius r_a, stiffness K = k_a I, damping
 * D = d_a I, and the rotation vector omega that parameterises the current vector
 * of Eq. (3): c = omega - n (n . omega).
 * heuristic (Sec. III-A; NULL = every agent GMAPP_H_CF_OMEGA) selects each agent's
 * repulsive field: GMAPP_H_CF_OMEGA the circular field above; GMAPP_H_MFI_VEL the
 * same field with the current of Eq. (3) taken from the relative velocity w,
 * c = w - n (n . w) (omega unused); GMAPP_H_APF the artificial potential field of
 * Eq. (1), f = k_f (1/rho - 1/r_d) (1/rho^2) d/|d| with the surface distance rho.
 * Heterogeneous agents run in gmapp_rollout, gmapp_rollout_pose, gmapp_rollout_arm,
 * gmapp_plan_loop, gmapp_control_force and gmapp_force_probe; the batched, adjoint
 * and served entry points require heuristic = NULL (EINVAL otherwise). */
#define GMAPP_H_CF_OMEGA 0
#define GMAPP_H_MFI_VEL 1
#define GMAPP_H_APF 2
typedef struct {
    const float *k_a, *d_a, *k_f, *r_d, *r_a; /* device [N_a] each */
    const float *omega;                       /* device [N_a][3] */
    int32_t n_agents;                         /* N_a >= 0 */
    const int32_t *heuristic;                 /* device [N_a] or NULL; values 0, 1, 2 (others read as 0) */
} gmapp_agents;

/* Planning query (host values): start position p^(1), start velocity v^(0),
 * goal p_g; `incumbent` is the agent selected in the previous cycle (-1 = none),
 * whose cost plays C_best in the selection rule; t0 is the time of step 1 on the
 * clock of the moving segments (step k is at t_k = t0 + (k-1) dt), so a resident
 * scene can be replanned cycle after cycle without moving its points. */
typedef struct {
    float p0[3], v0[3], goal[3];
    int32_t incumbent;
    float t0;
} gmapp_query;

/* Integrator, cost and selection parameters (host values).
 *   v^(k) = v^(k-1) + (dt/2) inv_mass F^(k)            Eqs. (9), (10)
 *   p^(k+1) = p^(k) + dt v^(k)                          Eq. (11), point mass
 *   rho = max(|p - p_O| - (r_O + r_a), eps)             Alg. 1
 *   cutoff 0: force kept iff rho <= r_d (Alg. 1); 1: C1 smoothstep taper over
 *   [r_d (1 - taper_band), r_d].  Costs use the radius r_cost (Eqs. 17-18), the
 *   weights w_* (Eq. 16) and a_max (Eq. 20); alpha tightens the selection rule. */
typedef struct {
    float dt, inv_mass, eps, r_cost;
    float w_goal, w_obs, w_path, w_smooth;
    float a_max, alpha, taper_band;
    int32_t n_steps; /* N_k >= 1 */
    int32_t cutoff;  /* 0 hard, 1 taper */
} gmapp_params;

/* Outputs (device).  traj[i][k] = p^(k+1) for k = 0..N_k (N_k + 1 poses);
 * cost[i] = {C_goal, C_obs, C_path, C_smooth, C_total}; min_clear[i][k] =
 * rho_min^(k+1), the smallest clamped surface distance at step k+1 (+inf when the
 * scene is empty); best[0] = i*, or -1 when N_a = 0, or GMAPP_ETIMEOUT when an
 * exchange wait of a sharded launch stalled past the watchdog limit
 * (gmapp_set_watchdog), or GMAPP_ECANCELLED when the host's abort word ended a
 * wait (gmapp_abort, gmapp_wait); the other outputs of such a launch are undefined.
 * traj and min_clear may be NULL. */
typedef struct {
    float *traj;      /* device [N_a][N_k + 1][3] or NULL */
    float *cost;      /* device [N_a][5] */
    float *min_clear; /* device [N_a][N_k] or NULL */
    int32_t *best;    /* device [1] */
} gmapp_outputs;

/* Forward rollout of one planning cycle (Sec. IV-A, Eqs. 6-11 and 15-20, Alg. 1 at
 * every step, selection rule of Sec. IV-A): all N_a agents over N_k steps in one
 * persistent launch; the repulsive force of each agent at each step is the sum of
 * Eq. (2) over all N_O spheres.  Selection: i* = argmin{C_i : C_i < alpha C_best},
 * ties to the lowest index; no incumbent gives the plain argmin. */
gmapp_status gmapp_rollout(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                           const gmapp_query *query, const gmapp_params *params, const gmapp_outputs *out,
                           void *stream);

/* Teacher-forced response of Alg. 1: for each agent i, the repulsive force
 * f_r[i] = sum_j Eq. (2) at position p[i], velocity v[i] and time t, and rho_min[i].
 * Same device code as one step of gmapp_rollout.  p, v, f_r: device [N_a][3];
 * rho_min: device [N_a] (may be NULL). */
gmapp_status gmapp_force_probe(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                               const float *p, const float *v, float t, const gmapp_params *params, float *f_r,
                               float *rho_min, void *stream);

/* 6-D pose agents (Sec. II, Sec. IV-A Eqs. 6-11 on Spin(3) x| R^3, the planner of
 * Sec. V-B).  An agent's pose is a unit rotor q (w, x, y, z) and a position p; its
 * twist (omega, u) is in the body frame.  Per step:
 *   e = log(M^-1 M_g)  (the Lie-group logarithm of SE(3): rotation vector of
 *       q^-1 q_g and J(phi)^-1 R^T (p_g - p), J the left Jacobian of SO(3)),
 *   F = K e - D v + (0, R^T f_r),  K = diag(k_r I, k_a I), D = diag(d_r I, d_a I),
 *   v += (dt/2) diag(i_r I, m^-1 I) F,   M <- M exp(dt v),
 * with f_r the agent's field (any heuristic) at p and at the world velocity
 * R(q) u of the body origin.  Costs (Eqs. 16-20) are taken on the positions, the
 * jerk literally from the position increments.
 * k_r, d_r, inv_inertia_r: device [N_a] each.  The query's p0 and goal give the
 * start and goal positions and v0 the start world linear velocity. */
typedef struct {
    const float *k_r;            /* rotational stiffness */
    const float *d_r;            /* rotational damping */
    const float *inv_inertia_r;  /* inverse rotational inertia */
} gmapp_pose_agents;

typedef struct {
    float q0[4];    /* start rotor (w, x, y, z), normalised on use */
    float w0[3];    /* start angular velocity, body frame [rad/s] */
    float qg[4];    /* goal rotor */
} gmapp_pose_query;

/* Forward rollout of 6-D pose agents: as gmapp_rollout (costs, selection, traj
 * and min_clear outputs), plus rot: device [N_a][N_k + 1][4] rotors or NULL.
 * EINVAL for a NULL pose or pose_query, NULL gain arrays with N_a > 0, or rotors
 * that are not finite with a non-zero norm. */
gmapp_status gmapp_rollout_pose(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                                const gmapp_pose_agents *pose, const gmapp_query *query,
                                const gmapp_pose_query *pose_query, const gmapp_params *params,
                                const gmapp_outputs *out, float *rot, void *stream);

/* Arm agents (Sec. IV-A Eqs. 12-14): each agent drives a serial chain of n revolute
 * joints about their local z axes, M(q) = L_0 Rz(q_1) L_1 ... Rz(q_n) L_n.  Per
 * step the wrench and twist are those of gmapp_rollout_pose (Eqs. 6-10) at the
 * end-effector pose M(q); then qdot = J_b^T (J_b J_b^T + damping^2 I)^-1 v with
 * J_b the body Jacobian of M, q += dt qdot, and M = M(q).  Costs are taken on the
 * end-effector positions.  The start pose is M(q0): the query's p0 and the pose
 * query's q0 are not used; v0 (world, linear) and w0 (body, angular) give the
 * start twist, goal and qg the goal pose. */
typedef struct {
    int32_t n_joints;      /* 1..7 */
    const float *links;    /* device [n_joints + 1][7]: L_i as rotor (w, x, y, z) and offset (x, y, z) */
    const float *q0;       /* device [n_joints]: start joint angles [rad] */
    float damping;         /* lambda >= 0 of the damped pseudo-inverse (0: J_b^T (J_b J_b^T)^-1, which needs
                              n_joints >= 6 and gives non-finite joint rates at a singular configuration) */
} gmapp_arm;

/* Forward rollout of arm agents: outputs as gmapp_rollout_pose, plus joints:
 * device [N_a][N_k + 1][n_joints] joint angles (q0 + the sum of dt qdot, not wrapped)
 * or NULL.  EINVAL for a NULL arm, n_joints outside 1..7, NULL links or q0, a damping
 * that is not finite and >= 0, damping 0 with fewer than 6 joints (J_b J_b^T, 6 x 6, is
 * then singular), or a forced tiling (gmapp_set_tiling) with more than 8 agents per
 * group (each agent holds one lane per joint in a wave). */
gmapp_status gmapp_rollout_arm(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                               const gmapp_pose_agents *pose, const gmapp_arm *arm, const gmapp_query *query,
                               const gmapp_pose_query *pose_query, const gmapp_params *params,
                               const gmapp_outputs *out, float *rot, float *joints, void *stream);

/* Closed planning loop (Sec. V-B, planner architecture; selection rule of Sec. IV-A
 * across cycles).  The robot is a point mass like the agents.  Cycle c = 0 ..
 * n_cycles - 1 runs, in stream order and with no host round trip:
 *  1. the rollout of gmapp_rollout from the robot's state (row c * ctrl_steps of
 *     out->robot) at t0_c = query->t0 + c * ctrl_steps * ctrl_dt (computed in double,
 *     rounded to float), its incumbent being i* of cycle c - 1 (query->incumbent for
 *     c = 0), so that C_best is the incumbent's cost in this cycle;
 *  2. ctrl_steps control steps of the robot under the selected agent i*_c: at each,
 *     the repulsive force of i*_c's field at the robot's state and time
 *     t0_c + j ctrl_dt (the control thread's query), the attractor with i*_c's
 *     k_a, d_a, and the integration of gmapp_rollout with dt = ctrl_dt.
 * N_sw counts the cycles whose i* differs from a valid previous i*.  If a cycle's
 * i* is negative (an error status) the robot keeps its state for that cycle.
 * Heterogeneous agents are allowed.  All outputs are device memory:
 *   robot       [n_cycles * ctrl_steps + 1][6]  p, v of the robot; row 0 = query p0, v0
 *   robot_clear [n_cycles * ctrl_steps] or NULL  rho_min at each control step
 *   best        [n_cycles]                       i* of each cycle
 *   cost        [n_cycles][N_a][5]               each cycle's costs (as gmapp_outputs.cost)
 *   n_switches  [1]                              N_sw
 * EINVAL for n_cycles < 1, ctrl_steps < 1, ctrl_dt not finite and > 0, N_a = 0 or
 * a NULL required output; ECAPACITY for a scene of more than 128 segments. */
typedef struct {
    int32_t n_cycles;     /* planning cycles, >= 1 */
    int32_t ctrl_steps;   /* control steps of the robot per cycle, >= 1 */
    float ctrl_dt;        /* control period [s] (0.01 = 100 Hz) */
} gmapp_loop_config;

typedef struct {
    float *robot;
    float *robot_clear;
    int32_t *best;
    float *cost;
    int32_t *n_switches;
} gmapp_loop_outputs;

gmapp_status gmapp_plan_loop(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                             const gmapp_query *query, const gmapp_params *params, const gmapp_loop_config *cfg,
                             const gmapp_loop_outputs *out, void *stream);

/* The control thread's query (Sec. V-B): the repulsive force f_r (Alg. 1, the
 * agent's own field) of the agent whose index is read from agent (device int32
 * [1]) at the state (device [6]: p, v) and time t, and rho_min.  f_r: device [3];
 * rho_min: device [1] or NULL.  An index outside [0, N_a) gives NaN outputs.
 * ECAPACITY for a scene of more than 128 segments. */
gmapp_status gmapp_control_force(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                                 const int32_t *agent, const float *state, float t, const gmapp_params *params,
                                 float *f_r, float *rho_min, void *stream);

/* Tiling of the rollout kernel.  An agent group is `agents` agents (power of two)
 * sharing the lanes of one wavefront (group = 1: agents 1..64) or of the whole
 * workgroup (group = 2: agents 1..8, 4/8/16 waves); a workgroup has `waves`
 * wavefronts (1, 2, 4, 8, 16) and one of `shards` point shards (>= 1; > 1 uses a
 * cooperative launch with one cross-workgroup exchange per step).  The shard sits
 * in LDS for the whole rollout (layout 1) or is streamed through tiles of
 * tile_points points every step (layout 2); layout 0 picks resident whenever it
 * fits.  Zero fields mean "choose". */
typedef struct {
    int32_t agents, waves, shards;
    int32_t tile_points, layout;
    int32_t group; /* 0 choose, 1 wavefront, 2 workgroup */
} gmapp_tiling;
/* Failure handling of the persistent launches (no passage of the paper: the one
 * failure rule it has is the perception buffer's frame time-out, Sec. V-A).  A
 * sharded rollout, adjoint or control launch exchanges partial sums between
 * workgroups every step, and every exchange wait is bounded.  A wait that finds its
 * words missing checks, every 64th poll (every poll with a limit below 1 ms), whether
 * another wave already ended a wait, whether the host raised the abort word, and
 * whether it has made no progress for longer than the watchdog limit; if so it ends,
 * and so do all later waits of the launch, which then runs its remaining steps
 * without waiting and reports best = GMAPP_ETIMEOUT (limit) or GMAPP_ECANCELLED
 * (abort), or NaN gradients.  Waits that are answered promptly are never
 * interrupted, so a launch that makes progress runs to its end.
 *  - gmapp_set_watchdog: the limit in seconds (0 = the default 4 s; EINVAL outside
 *    (0, 3600]) for launches enqueued afterwards.  The clock restarts with every
 *    wait, so a long launch is never cut short while it makes progress.
 *  - gmapp_abort(raise = 1): raises the context's abort word, a pinned host word the
 *    waits read, for the running and later launches on this context, until
 *    gmapp_abort(raise = 0).  May be called from any host thread while a launch runs.
 *  - gmapp_wait: waits up to timeout_s seconds for `stream`; past that it raises the
 *    abort word, so that no wait of the stream's launches can hang, waits for them
 *    to drain, lowers it again and returns GMAPP_ETIMEOUT. */
gmapp_status gmapp_set_watchdog(gmapp_ctx *ctx, double seconds);
gmapp_status gmapp_abort(gmapp_ctx *ctx, int32_t raise);
gmapp_status gmapp_wait(gmapp_ctx *ctx, void *stream, double timeout_s);

/* Force a tiling for later rollouts on this context (NULL restores the automatic choice). */
gmapp_status gmapp_set_tiling(gmapp_ctx *ctx, const gmapp_tiling *tiling);
/* The tiling gmapp_rollout would use for this problem shape. */
gmapp_status gmapp_get_tiling(gmapp_ctx *ctx, int64_t n_points, int32_t n_agents, int32_t n_steps, int32_t n_seg,
                              int32_t cutoff, gmapp_tiling *out);

/* ------------------------------------------------------------------------
 * Many planning problems per launch.  Each job is one planning cycle of its own
 * scene, agents, query and parameters (the rollout, costs and selection rule of
 * gmapp_rollout), optionally restricted to the step range [k_begin, k_end) so
 * that a long horizon can be advanced a quantum of steps per launch: the agents'
 * integration state (position, velocity and their compensation terms, the last
 * two net forces, the running cost sums) is kept in `state` between launches.
 * Costs, min_clear and the selection are written when a launch reaches the end
 * of the horizon (k_end = N_k + 1); trajectory rows k_begin..k_end-1 (and row 0
 * when k_begin = 1) are written by every launch.  Results do not depend on the
 * other jobs of the launch, on the step ranges or on the tuning, except through
 * FP32 summation order (tuning changes which lanes sum which points).
 */
#define GMAPP_STATE_FLOATS 28
#define GMAPP_BATCH_MAX_JOBS 16384
#define GMAPP_BATCH_MAX_SEGMENTS 64 /* moving segments per scene in a batched launch */

typedef struct {
    gmapp_scene scene;
    gmapp_agents agents;
    gmapp_query query;
    gmapp_params params;
    gmapp_outputs out;
    float *state;    /* device [N_a][GMAPP_STATE_FLOATS]; required unless k_begin = 1 and k_end = N_k + 1 */
    int32_t k_begin; /* first step of this launch, 1 <= k_begin <= N_k */
    int32_t k_end;   /* one past the last step, k_begin < k_end <= N_k + 1 */
    const uint32_t *cancel; /* NULL, or a word the device can read while the launch runs (the device
                               address of mapped, coherent host memory): nonzero cancels the job --
                               its work items not yet started are skipped, running ones stop within
                               64 steps, and best[0] reads GMAPP_ECANCELLED; its other outputs (and
                               state) are then undefined.  Keep the word raised until the launch ends. */
} gmapp_job;

/* Tuning of the batched kernel.  Zero fields mean "choose" (the autotuned values
 * when gmapp_autotune_batch has run on this context, else built-in defaults).
 *   tile_points: points per LDS tile; worlds of at most this many points stay
 *                resident in LDS for a whole item (64 .. 12288);
 *   wg_per_cu:   persistent workgroups per CU (1..4, capped by what fits);
 *   balance:     an item may take at most 1/balance of the launch's balanced
 *                per-workgroup share of work (1..64);
 *   item_shape:  1..4: every wave runs 1, 2, 4 or 8 agents (8 waves per item);
 *                5..8: the workgroup's 512 lanes run 1, 2, 4 or 8 agents. */
typedef struct {
    int32_t tile_points, wg_per_cu, balance, item_shape;
} gmapp_batch_tuning;

/* One persistent launch over n_jobs jobs (1..GMAPP_BATCH_MAX_JOBS, at most
 * GMAPP_BATCH_MAX_SEGMENTS segments per scene).  Workgroups pull (job, agent
 * block) items from a device queue, longest items first.  The job table is staged
 * through pinned host memory owned by the context.  A job's cancel word (see
 * gmapp_job) and the context's abort word (gmapp_abort, gmapp_wait) are read at the
 * start of every item and every 64 steps within one: a raised word ends that job's
 * (or, for the abort word, every job's) work early, with best[0] = GMAPP_ECANCELLED. */
gmapp_status gmapp_rollout_batch(gmapp_ctx *ctx, const gmapp_job *jobs, int32_t n_jobs, void *stream);
/* Force a batch tuning on this context (NULL restores the automatic choice). */
gmapp_status gmapp_set_batch_tuning(gmapp_ctx *ctx, const gmapp_batch_tuning *t);
/* The tuning batched launches on this context use (zero item_shape = per job). */
gmapp_status gmapp_get_batch_tuning(gmapp_ctx *ctx, gmapp_batch_tuning *out);

/* A control cycle as an instantiated HIP graph: a copy of the job table from
 * pinned host memory, then the batched kernel; each launch replays it.  The
 * batch owns its pinned and device tables (max_jobs entries) and fixes the
 * kernel tuning at creation.  gmapp_batch_set_jobs waits for the previous replay
 * to finish reading the pinned table, plans the items and updates the copy node;
 * gmapp_batch_launch enqueues one replay on `stream`.  A batch belongs to one
 * context and shares its workspace (calls ordered on one stream). */
typedef struct gmapp_batch gmapp_batch;
gmapp_status gmapp_batch_create(gmapp_ctx *ctx, int32_t max_jobs, gmapp_batch **out);
gmapp_status gmapp_batch_set_jobs(gmapp_batch *b, const gmapp_job *jobs, int32_t n_jobs);
gmapp_status gmapp_batch_launch(gmapp_batch *b, void *stream);
void gmapp_batch_destroy(gmapp_batch *b);

/* Autotuner.  gmapp_autotune_rollout times the valid tilings of gmapp_rollout on
 * a proxy of the problem (its first min(proxy_steps, N_k) steps, outputs into the
 * context workspace) and caches the fastest for the problem's shape class
 * (N_O rounded up to a power of two, N_a, N_k rounded up to a power of two,
 * static or moving, cut-off mode); later rollouts of that class use it unless a
 * tiling is forced.  gmapp_autotune_batch times tile size, workgroups per CU and
 * balance for the given jobs, each shortened in proportion to its step count
 * (the longest to proxy_steps), and keeps the fastest for later batched launches
 * and batches created afterwards.  best / best_ms (host, may be NULL) receive the
 * choice and its proxy time.  Both synchronise the stream. */
gmapp_status gmapp_autotune_rollout(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                                    const gmapp_query *query, const gmapp_params *params, int32_t proxy_steps,
                                    gmapp_tiling *best, float *best_ms, void *stream);
gmapp_status gmapp_autotune_batch(gmapp_ctx *ctx, const gmapp_job *jobs, int32_t n_jobs, int32_t proxy_steps,
                                  gmapp_batch_tuning *best, float *best_ms, void *stream);

/* ------------------------------------------------------------------------
 * Replanning server: a request loop on its own host thread that admits requests
 * while device memory (a budget allocated once at creation) and slots allow,
 * uploads their worlds and agents once, and runs control cycles in which every
 * active request advances by `quantum_steps` steps (gmapp_batch graph replays;
 * agent state stays on the device between cycles).  Requests that arrive while
 * others run join at the next cycle (continuous batching); a request's result
 * is the rollout and selection of gmapp_rollout for its problem.  Uploads of
 * newly admitted requests overlap the running cycle.  The server owns its
 * context while it exists: make no other calls on that context meanwhile.
 */
typedef struct gmapp_server gmapp_server;

typedef struct {
    uint64_t memory_budget; /* device bytes for admitted requests (0 = 4 GiB) */
    int32_t max_active;     /* requests on the device at once, 1..GMAPP_BATCH_MAX_JOBS (0 = 256) */
    int32_t quantum_steps;  /* steps per request per cycle (0 = 50) */
    int32_t max_queue;      /* waiting requests before submit refuses with ECAPACITY (0 = 65536) */
} gmapp_server_config;

/* A replanning request.  All arrays are host memory owned by the caller and must
 * stay valid until the request's completion has been polled (inputs are copied
 * to the device at admission, outputs written before completion).  Device bytes used while
 * active: 12 N_O + 16 n_seg + 4 + 32 N_a (agents) + 20 N_a + 4 (costs, choice)
 * + 112 N_a (state) + 12 N_a (N_k + 1) if traj is requested, each piece rounded
 * up to 256 B. */
typedef struct {
    const float *x, *y, *z;     /* [N_O] */
    int64_t n_points;
    float r_obs;
    int32_t n_seg;              /* <= GMAPP_BATCH_MAX_SEGMENTS */
    const int32_t *seg_begin;   /* [n_seg + 1] */
    const float *seg_vel;       /* [n_seg][3] */
    const float *k_a, *d_a, *k_f, *r_d, *r_a; /* [N_a] */
    const float *omega;         /* [N_a][3] */
    int32_t n_agents;
    gmapp_query query;
    gmapp_params params;
    double deadline_s;          /* finish within this many seconds of submission, else ETIMEOUT (0 = none) */
    float *cost;                /* out [N_a][5] or NULL */
    float *traj;                /* out [N_a][N_k + 1][3] or NULL (then no device trajectory either) */
} gmapp_request;

typedef struct {
    int64_t id;
    gmapp_status status;        /* OK, ETIMEOUT (deadline passed) or ECANCELLED */
    int32_t best;               /* i*, -1 for N_a = 0 or when status != OK */
    double queue_s;             /* submission to admission (-1 if never admitted) */
    double latency_s;           /* submission to completion */
} gmapp_completion;

typedef struct {
    int64_t submitted, completed, rejected, expired, cancelled, cycles;
    double p50_s, p99_s, max_s, mean_s; /* latency of completed requests */
    double busy_s;                      /* time spent in cycles */
    double interactions_per_s;          /* N_a N_k N_O of completed requests / busy_s */
    double cycle_mean_s;
    int32_t max_active_seen;
    uint64_t peak_bytes;
} gmapp_server_stats;

gmapp_status gmapp_server_create(gmapp_ctx *ctx, const gmapp_server_config *cfg, gmapp_server **out);
/* Queue a request; *id receives its id.  EINVAL for a malformed request or one
 * that can never fit the budget, ECAPACITY when the queue is full. */
gmapp_status gmapp_server_submit(gmapp_server *s, const gmapp_request *req, int64_t *id);
/* Up to max completions, waiting up to wait_ms for the first; returns the count (>= 0). */
int32_t gmapp_server_poll(gmapp_server *s, gmapp_completion *out, int32_t max, int32_t wait_ms);
/* Cancel a waiting or active request (it completes with ECANCELLED); EINVAL if unknown or finished.
 * An active request's work in the running cycle is skipped or stopped on the device (its job's
 * cancel word, see gmapp_job), so it completes without waiting for its quantum to finish. */
gmapp_status gmapp_server_cancel(gmapp_server *s, int64_t id);
/* Wait until no request is waiting or active (ETIMEOUT after timeout_ms; < 0 = no limit). */
gmapp_status gmapp_server_drain(gmapp_server *s, int32_t timeout_ms);
/* Counters and latency percentiles so far; returns the first device error the
 * loop met (its requests completed with that status), else GMAPP_OK. */
gmapp_status gmapp_server_get_stats(gmapp_server *s, gmapp_server_stats *out);
/* Stops the loop after the running cycle; requests not finished are dropped. */
void gmapp_server_destroy(gmapp_server *s);

/* Adjoint rollout: gradients of sum_i grad_total[i] C_i, with C_i agent i's total
 * cost (Eq. 16) after the rollout of gmapp_rollout, with respect to each agent's
 * k_a, d_a, k_f (Eqs. 2, 7) and rotation vector omega (Eq. 3).  One launch runs
 * the forward rollout storing the agent state every ckpt_every steps, then, for
 * each segment from last to first, recomputes the segment and sweeps it
 * backwards (reverse mode, FP32).  The hard cut-off (cutoff 0) is differentiated
 * almost everywhere; use the C1 taper (cutoff 1) for gradients that match finite
 * differences.  grad_total: device [N_a]; g_k_a, g_d_a, g_k_f: device [N_a];
 * g_omega: device [N_a][3].  Checkpoints and per-step records live in LDS:
 * (N_k / ckpt_every) checkpoints of 80 bytes and ckpt_every records of 48 bytes
 * per agent of a workgroup; ECAPACITY if they do not fit. */
gmapp_status gmapp_rollout_backward(gmapp_ctx *ctx, const gmapp_scene *scene, const gmapp_agents *agents,
                                    const gmapp_query *query, const gmapp_params *params, const float *grad_total,
                                    int32_t ckpt_every, float *g_k_a, float *g_d_a, float *g_k_f, float *g_omega,
                                    void *stream);

/* Back-projection of a z-depth image into world points (Sec. IV-B / V-A: the
 * perception pipeline's coordinate transform).  Pixel (u, v) = column, row with
 * depth z = depth[v * w + u] (metres) maps to the camera point
 * ((u - c_x) z / f_x, (v - c_y) z / f_y, z) and then to R X_c + t with
 * T_wc = [R | t] (host, row-major 3 x 4).  K = {f_x, f_y, c_x, c_y} (host).
 * Pixels with z <= 0 or non-finite z give NaN points (dropped by the voxel pass).
 * depth: device [h][w]; x, y, z: device [w * h] SoA outputs. */
gmapp_status gmapp_depth_to_points(gmapp_ctx *ctx, const float *depth, int32_t w, int32_t h, const float K[4],
                                   const float T_wc[12], float *x, float *y, float *z, void *stream);

/* The same back-projection for n_frames images of one camera (intrinsics K,
 * host) taken from n_frames poses (multi-view fusion into one world cloud):
 * depth: device [n_frames][h][w]; T_wc: device [n_frames][12], row-major [R | t]
 * per frame (poses are not checked for finiteness); frame f's pixel (u, v) goes
 * to x, y, z [f w h + v w + u] (device).  Feeding the n_frames w h points to
 * gmapp_voxel_downsample gives the fused voxel-centre cloud. */
gmapp_status gmapp_depth_to_points_batch(gmapp_ctx *ctx, const float *depth, int32_t n_frames, int32_t w, int32_t h,
                                         const float K[4], const float *T_wc, float *x, float *y, float *z,
                                         void *stream);

/* Uniform voxel lattice of the sphere world (Sec. IV-B; voxel size 2 r_O in
 * Sec. V-A, voxel-centre clouds): the cell of a point is the exact lattice
 * coordinate floor((p - lo) / voxel) per axis of the real values of the FP32
 * inputs p, lo and voxel (no rounding of the quotient decides it); points outside
 * the box lo + [0, dims * voxel) or non-finite are dropped (the workspace
 * bounding-box filter).  Every cell holding at least min_count points (>= 1;
 * larger values filter sensing artifacts) contributes its centre
 * lo + (k + 1/2) voxel, rounded once to FP32 (dims: 1 .. 2^23 per axis, at most 2^31
 * cells, else ECAPACITY).  Centres are written to ox, oy, oz
 * (device [capacity]) in increasing linear cell index (x fastest, then y, then z);
 * the number of occupied cells goes to n_out_dev (device int64 [1]), even when it
 * exceeds capacity (then only the first `capacity` centres are written).
 * The context keeps a grid over the box (1 byte per cell for min_count = 1,
 * 4 bytes per cell otherwise) and a table of about 133 bytes per 1024 cells, both
 * allocated by the first call that needs larger ones (a device allocation, ENOMEM if
 * it fails) and freed by gmapp_destroy.
 * x, y, z: device [n]. */
gmapp_status gmapp_voxel_downsample(gmapp_ctx *ctx, const float *x, const float *y, const float *z, int64_t n,
                                    float voxel, const float lo[3], const int32_t dims[3], int32_t min_count,
                                    float *ox, float *oy, float *oz, int64_t capacity, int64_t *n_out_dev,
                                    void *stream);

/* The voxel pass with the robot self-filter of Sec. V-A: before voxelisation,
 * points within any of the robot's bounding spheres are removed (the caller
 * places the spheres by forward kinematics).  robot_spheres: device [n_spheres][4]
 * (centre x, y, z, radius); a point p is removed when |p - c|^2 <= r^2, evaluated
 * in FP64 as ((dx dx + dy dy) + dz dz) with each operation rounded (no fused
 * multiply-add).  n_spheres = 0 is gmapp_voxel_downsample.  EINVAL for
 * n_spheres < 0 or a NULL robot_spheres with n_spheres > 0; otherwise as
 * gmapp_voxel_downsample. */
gmapp_status gmapp_voxel_downsample_filtered(gmapp_ctx *ctx, const float *x, const float *y, const float *z,
                                             int64_t n, float voxel, const float lo[3], const int32_t dims[3],
                                             int32_t min_count, const float *robot_spheres, int32_t n_spheres,
                                             float *ox, float *oy, float *oz, int64_t capacity, int64_t *n_out_dev,
                                             void *stream);

/* For callers that cannot allocate device memory during the call (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the voxel
 * pass of gmapp_voxel_downsample (no robot self-filter) on a statically sized grid
 * that the library holds per device for the life of the process (8.3 MiB, set up by
 * gmapp_create), so this call allocates nothing.  Grids of more than 2^21 cells give
 * ECAPACITY; otherwise arguments, outputs and errors are those of
 * gmapp_voxel_downsample.  Every call on one device shares that device's grid: calls
 * whose work overlaps on one device (other streams, other contexts or threads) race
 * and must be ordered by the caller. */
gmapp_status gmapp_voxel_downsample_noalloc(gmapp_ctx *ctx, const float *x, const float *y, const float *z,
                                            int64_t n, float voxel, const float lo[3], const int32_t dims[3],
                                            int32_t min_count, float *ox, float *oy, float *oz, int64_t capacity,
                                            int64_t *n_out_dev, void *stream);

/* Depth frames straight to the voxel-centre cloud (Sec. IV-B / V-A: coordinate
 * transform, robot self-filter and voxel lattice in one pass): every pixel is
 * back-projected exactly as gmapp_depth_to_points_batch does it (the same FP32
 * operations, so the same point) and its cell marked without writing the point
 * to memory.  The result equals gmapp_depth_to_points_batch followed by
 * gmapp_voxel_downsample_filtered on its n_frames w h points, bit for bit.
 * depth: device [n_frames][h][w]; K = {f_x, f_y, c_x, c_y} (host); T_wc: device
 * [n_frames][12]; lattice, self-filter, outputs and errors as
 * gmapp_voxel_downsample_filtered (robot_spheres may be NULL with n_spheres 0). */
gmapp_status gmapp_depth_to_voxels(gmapp_ctx *ctx, const float *depth, int32_t n_frames, int32_t w, int32_t h,
                                   const float K[4], const float *T_wc, float voxel, const float lo[3],
                                   const int32_t dims[3], int32_t min_count, const float *robot_spheres,
                                   int32_t n_spheres, float *ox, float *oy, float *oz, int64_t capacity,
                                   int64_t *n_out_dev, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GMAPP_H */
