#pragma once
// Forward rollout of N_a circular-field agents over N_k steps (G-MAPP, Sec. IV-A
// and Alg. 1), one persistent launch per planning cycle, for gfx950 (CDNA4).
//
// Work decomposition
//   An agent group is either one wavefront (WS = 1) or the whole workgroup of W
//   waves (WS = W).  Its lanes are (agent, slice) pairs, lane = agent + AW * slice,
//   so each of its AW agents spreads the shard's points over L = 64 WS / AW lanes.
//   A workgroup holds W / WS groups and one shard of the sphere world (a contiguous
//   range of the N_O points) in LDS, read by all its waves; S workgroups (shards)
//   cover the points.  Points of one segment (object) are dealt round-robin to the
//   lanes of the run, so every point read is broadcast to the AW agents of its slice
//   and a run wastes at most one interaction per lane.  With wave groups no
//   workgroup barrier sits in the step loop when the shard is LDS-resident; a
//   workgroup-wide group reduces its waves' partials through LDS (two barriers per
//   step).  Shards too large for LDS are streamed through tiles.
//
//   After each step the S shards of a group exchange partial sums through the
//   context arena.  Each 64-bit word carries one float and the step number, so a
//   reader knows a word is current without any fence or counter: the device-scope
//   (sc1) stores and loads are single-copy atomic.  Every shard adds the S
//   partials in shard order, so all shards hold bit-identical agent states.
//   Shards of a group are placed on one XCD (dispatch is round-robin over 8 XCDs).
//   Each group's lead wave (the group's only wave for wave groups) publishes and
//   polls; wave groups of one CU overlap one another's exchange latency.
//   Every wait is bounded (slow_check): a wait that stalls past the context's limit,
//   or sees the host's abort word, ends, and so do the launch's later waits; the
//   rollout then runs its remaining steps without waiting and reports the status.
//
// Per interaction (agent i, sphere j) the lane evaluates the factored form of
// Eq. (2) with the current vector c = omega - n (n . omega):
//   f_j = g_j k_f |w| P_w (omega - n_j (n_j . omega)),  g_j = [rho_j <= r_d] / rho_j,
// where P_w projects out w (the relative velocity, uniform over a segment) so
//   sum_j f_j = k_f |w| P_w (omega G - S),  G = sum g_j,  S = sum g_j (d_j . omega) d_j / |d_j|^2.
// The lane accumulates G, S (4 floats) and min |d|^2 over its points with about
// 21.5 VALU ops and 2 transcendentals (rsq, rcp) per interaction, plus about 2 of
// loop bookkeeping (LDS addresses, the per-lane trip count) in the 4-point unrolled loop.
// rho_min^(k) = max(sqrt(min |d|^2) - (r_O + r_a), eps).
//
// Heterogeneous ensembles (HET) take each agent's field from its heuristic code:
// the same factored sum with omega replaced by w (velocity current, Eq. 3), or the
// APF of Eq. (1) on the surface distance, sum_j [rho_j <= r_d] (1/rho_j - 1/r_d)
// d_j / (rho_j^2 |d_j|), scaled by k_f (about as many VALU ops per interaction).
//
// Integration (Eqs. 6, 7, 9-11; explicit: forces use v^(k-1)) and the running
// costs (Eqs. 17-20) are O(1) per agent per step; positions, velocities and
// cost sums carry Kahan compensation.  The jerk of Eq. (20) uses the identity
// p^(k) - 3p^(k-1) + 3p^(k-2) - p^(k-3) = (dt^2 / 2m) (F^(k-1) - F^(k-2)).
// The last workgroup to finish applies the selection rule and clears the
// exchange area for the next launch.
#include "gmapp_internal.h"
#include "pairs.h"
#include "pose.h"
#include "arm.h"

#include <algorithm>
#include <cmath>

namespace gm {

using namespace dev;

// Words per (shard, agent) exchange slot: Fx, Fy, Fz, min r2 (the rest pads the slot
// to its own 128-byte line).
constexpr int kSlotWords = 4;
static_assert(kSlotWords == 4, "the one-instruction exchange maps lane l to word l of a slot row");

// Launch-time layout of the shard in LDS.
struct Lay {
    int resident;   // 1 = the whole shard is loaded once, 0 = streamed tiles
    int cap;        // points held in LDS (shard capacity or tile size)
    int runs_cap;   // segment runs per shard
};

// Dynamic LDS layout of k_rollout, in bytes (16-byte aligned pieces):
//   points [cap][3] (x, y, z interleaved)  ·  red float4 [2][W][AW]  ·  tot float4 [groups][AW][2]
//   ·  xt float4 [groups][S*AW]
//   ·  runs int4 [runs_cap]  ·  rvel float4 [runs_cap]  ·  sel (float, int) [NT]
struct LdsPlan {
    size_t cx, cy, cz, red, tot, xt, runs, rvel, sel, total;
};
__host__ __device__ inline LdsPlan lds_plan(const Lay &l, int W, int WS, int AW, int S)
{
    LdsPlan p;
    const size_t plane = ((size_t)l.cap * 4 + 15) / 16 * 16;
    const int groups = W / WS;                    // agent groups per workgroup
    p.cx = 0; p.cy = plane; p.cz = 2 * plane;   // [cx, cx + 3 plane): the points, interleaved x, y, z
    p.red = 3 * plane;                            // [2][W][AW] wave partials (WS > 1)
    p.tot = p.red + (WS > 1 ? (size_t)2 * W * AW * 16 : 0);   // [groups][AW] group totals (WS > 1)
    p.xt = p.tot + (WS > 1 ? (size_t)groups * AW * 32 : 0);   // tot: new (p, v) per agent, 2 float4
    p.runs = p.xt + (S > 1 ? (size_t)groups * S * AW * 16 : 0);
    p.rvel = p.runs + (size_t)l.runs_cap * 16;
    p.sel = p.rvel + (size_t)l.runs_cap * 16;
    p.total = p.sel + (size_t)64 * W * 8;
    return p;
}

// An agent group is WS waves (1 or W) sharing AW agents; a workgroup holds W / WS
// groups.  PROBE: one teacher-forced step at the given states (no integration, no costs).
// HET: each agent takes its field from ag.heur (rotation-vector circular field,
// velocity-current field or APF); without it every agent runs the rotation-vector field.
// KIND 1: 6-D pose agents (rotor and translation, body twist; Eqs. 6-11 on
// Spin(3) x| R^3); KIND 2: arm agents (the same wrench and twist, the pose moved
// through the joints, Eqs. 12-14).  The pairwise pass sees their end-effector
// position and world velocity.
template <int AW, int W, int WS, int CUT, bool PROBE, bool HET, int KIND>
__global__ __launch_bounds__(64 * W) void k_rollout(Scn sc, Agt ag, Prm pr, Out out, Probe pb, Xch xc, Lay lay)
{
    constexpr int NT = 64 * W;
    constexpr int GPW = W / WS;                   // agent groups per workgroup
    constexpr int L = 64 * WS / AW;               // slices per agent
    static_assert(AW >= 1 && AW <= 64 && 64 % AW == 0, "agents per group");
    static_assert(WS == 1 || WS == W, "a group is one wave or the whole workgroup");
    extern __shared__ float4 lds4[];
    const int S = xc.S, G = xc.G;                // G: workgroups per shard
    const LdsPlan lp = lds_plan(lay, W, WS, AW, S);
    char *lds = reinterpret_cast<char *>(lds4);
    float *lpt = reinterpret_cast<float *>(lds + lp.cx);          // points interleaved: x, y, z per point
    int4 *runs = reinterpret_cast<int4 *>(lds + lp.runs);      // [runs_cap]: begin, end, first slice, slices
    float4 *rvel = reinterpret_cast<float4 *>(lds + lp.rvel);  // [runs_cap]
    __shared__ int s_last, s_nruns, s_split;

    constexpr bool POSE = KIND >= 1;
    constexpr bool ARM = KIND == 2;
    static_assert(!ARM || AW <= kMaxArmAgentsPerGroup, "arm agents hold a lane per joint in a wave");
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int gi = wave / WS;                     // group within the workgroup
    const int a_w = lane % AW;
    const int slice = ((wave % WS) * 64 + lane) / AW;
    const bool lead = (wave % WS) == 0;           // the group's wave that exchanges with other shards
    float4 *red = reinterpret_cast<float4 *>(lds + lp.red);
    float4 *tot = reinterpret_cast<float4 *>(lds + lp.tot) + (size_t)gi * AW * 2;
    float4 *xtw = reinterpret_cast<float4 *>(lds + lp.xt) + (size_t)gi * S * AW;  // this group's gather

    // workgroup -> (group g, shard s); for S > 1 the S shards of a group share an
    // XCD (dispatch is round-robin over 8 XCDs)
    int g, s;
    if (S > 1) {
        const int nwg = gridDim.x;                // multiple of 8
        const int lin = (blockIdx.x & 7) * (nwg >> 3) + (blockIdx.x >> 3);
        g = lin / S;
        s = lin % S;
    } else {
        g = blockIdx.x;
        s = 0;
    }
    if (g >= G) return;                           // padding workgroup (not counted in `done`)

    const int GW = G * GPW;                       // agent groups in the launch
    const int gw = g * GPW + gi;                  // this lane's group
    const int agent = gw * AW + a_w;
    const bool valid = agent < ag.n;
    const int ai = valid ? agent : 0;
    Agent P;
    P.ka = ag.k_a[ai];
    P.da = ag.d_a[ai];
    P.kf = ag.k_f[ai];
    P.rd = ag.r_d[ai];
    P.R = sc.r_obs + ag.r_a[ai];
    P.wx = ag.omega[3 * ai];
    P.wy = ag.omega[3 * ai + 1];
    P.wz = ag.omega[3 * ai + 2];
    P.tb_a = 1.0f / (pr.band * P.rd);             // taper: s = (r_d - rho) / (band r_d)
    P.tb_b = P.rd * P.tb_a;
    if constexpr (POSE) {
        P.kr = ag.k_r[ai];
        P.dr = ag.d_r[ai];
        P.ir = ag.i_r[ai];
    }
    if constexpr (HET) {
        P.hz = ag.heur ? ag.heur[ai] : 0;           // pose kernels run HET with or without codes
        if (P.hz != 1 && P.hz != 2) P.hz = 0;
        P.ird = 1.0f / P.rd;
    }

    long long n_pts = sc.n_cap;
    if (sc.n_dev) n_pts = min(max(*sc.n_dev, 0ll), sc.n_cap);
    const long long sb = n_pts * s / S, se = n_pts * (s + 1) / S;
    const long long n_shard = se - sb;

    // segment runs of this shard, and the split of every agent's slices over them
    if (tid == 0) {
        int split = 0;
        s_nruns = build_runs(sc, n_pts, sb, se, runs, rvel, lay.runs_cap, L, split);
        s_split = split;
    }
    const bool resident = lay.resident && n_shard <= (long long)lay.cap;
    if (resident)
        for (int i = tid; i < (int)n_shard; i += NT) {
            lpt[3 * i] = sc.x[sb + i]; lpt[3 * i + 1] = sc.y[sb + i]; lpt[3 * i + 2] = sc.z[sb + i];
        }
    __syncthreads();
    const int n_runs = s_nruns;
    // this lane's run when the slices are split over the runs (resident layout)
    const bool split = resident && s_split;
    int my_j0 = 0, my_n = 0, my_stride = 1;
    float4 my_v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (split) lane_run(runs, rvel, n_runs, slice, my_j0, my_n, my_stride, my_v);

    // agent state
    float px, py, pz, vx, vy, vz, t_fixed = 0.0f;
    if constexpr (PROBE) {
        px = pb.p[3 * ai]; py = pb.p[3 * ai + 1]; pz = pb.p[3 * ai + 2];
        vx = pb.v[3 * ai]; vy = pb.v[3 * ai + 1]; vz = pb.v[3 * ai + 2];
        t_fixed = pb.t;
    } else if (pr.start) {
        px = pr.start[0]; py = pr.start[1]; pz = pr.start[2];
        vx = pr.start[3]; vy = pr.start[4]; vz = pr.start[5];
    } else {
        px = pr.p0[0]; py = pr.p0[1]; pz = pr.p0[2];
        vx = pr.v0[0]; vy = pr.v0[1]; vz = pr.v0[2];
    }
    float cpx = 0, cpy = 0, cpz = 0, cvx = 0, cvy = 0, cvz = 0;     // Kahan terms
    float F1x = 0, F1y = 0, F1z = 0, F2x = 0, F2y = 0, F2z = 0;     // F^(k-1), F^(k-2)
    // 6-D pose agents: rotor, body twist (omega, u), and the last three position increments
    // p^(k) - p^(k-1), ... (the point-mass jerk identity does not hold for them)
    pose::Q qr{1.f, 0.f, 0.f, 0.f};
    float ox = 0, oy = 0, oz = 0, ux = 0, uy = 0, uz = 0, cux = 0, cuy = 0, cuz = 0;
    float D1x = 0, D1y = 0, D1z = 0, D2x = 0, D2y = 0, D2z = 0, D3x = 0, D3y = 0, D3z = 0;
    // arm agents: lane a_w + AW j of each wave owns joint j (j = lane / AW): its half-angle
    // rotor and its angle; every lane holds the FP64 end-effector position and the start position
    const int my_j = lane / AW;
    double jc_own = 1.0, js_own = 0.0, q_own = 0.0;
    float colj[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};     // this lane's column of J at the current joints
    double pdx = 0, pdy = 0, pdz = 0;
    float a0x = 0, a0y = 0, a0z = 0;
    if constexpr (ARM && !PROBE) {
        if (my_j < pr.arm_n) {
            q_own = (double)pr.arm_q0[my_j];
            sincos(0.5 * q_own, &js_own, &jc_own);
        }
        arm::QD r;
        arm::fk_scan<AW>(pr.arm_links, pr.arm_n, a_w, my_j, jc_own, js_own, r, pdx, pdy, pdz, colj);
        qr = pose::Q{(float)r.w, (float)r.x, (float)r.y, (float)r.z};
        px = (float)pdx; py = (float)pdy; pz = (float)pdz;
        a0x = px; a0y = py; a0z = pz;
    }
    if constexpr (POSE && !PROBE) {
        if constexpr (!ARM) qr = pose::qnormalize(pose::Q{pr.q0[0], pr.q0[1], pr.q0[2], pr.q0[3]});
        ox = pr.om0[0]; oy = pr.om0[1]; oz = pr.om0[2];
        pose::qrot(qr, -1.0f, vx, vy, vz, ux, uy, uz);              // body linear velocity
    }
    float sg = 0, cg = 0, so = 0, co = 0, sp = 0, cp = 0, sj = 0, cj = 0;  // cost sums
    const float gx = pr.goal[0], gy = pr.goal[1], gz = pr.goal[2];
    const float h = 0.5f * pr.dt * pr.inv_mass;
    const float hj = h * pr.dt;                                     // dt^2 / 2m
    const float inv_rc = 1.0f / pr.r_cost;
    const bool writer = valid && s == 0 && slice == 0 && !PROBE;
    const int n_steps = PROBE ? 1 : pr.n_steps;
    const size_t traj_row = (size_t)(pr.n_steps + 1) * 3;
    if (writer && out.traj) {
        float *tr = out.traj + (size_t)agent * traj_row;
        tr[0] = px; tr[1] = py; tr[2] = pz;
    }
    if constexpr (POSE) {
        if (writer && out.rot) {
            float *ro = out.rot + (size_t)agent * (pr.n_steps + 1) * 4;
            ro[0] = qr.w; ro[1] = qr.x; ro[2] = qr.y; ro[3] = qr.z;
        }
    }
    // joint angles are written by their owner lanes of the lead wave of shard 0
    const bool jwriter = ARM && valid && s == 0 && lead && !PROBE && my_j < pr.arm_n;
    if constexpr (ARM) {
        if (jwriter && out.joints) out.joints[(size_t)agent * (pr.n_steps + 1) * pr.arm_n + my_j] = pr.arm_q0[my_j];
    }

    for (int k = 1; k <= n_steps; ++k) {
        const float t = PROBE ? t_fixed : fmaf((float)(k - 1), pr.dt, pr.t0);
        float Fx = 0, Fy = 0, Fz = 0, m2 = INFINITY;

        // ---- pairwise pass over this shard (hot loop)
        if (split) {
            const float psx = fmaf(-t, my_v.x, px), psy = fmaf(-t, my_v.y, py), psz = fmaf(-t, my_v.z, pz);
            const float *q = lpt + 3 * my_j0;
            const int step3 = 3 * my_stride;
            if (HET && P.hz == 2) {                 // artificial potential field
                float Ax = 0, Ay = 0, Az = 0;
#pragma unroll 4
                for (int i = 0; i < my_n; ++i, q += step3)
                    interact_apf<CUT>(q[0], q[1], q[2], psx, psy, psz, P.R, pr.eps, P.rd, P.ird, P.tb_a, P.tb_b, Ax,
                                      Ay, Az, m2);
                Fx = fmaf(P.kf, Ax, Fx); Fy = fmaf(P.kf, Ay, Fy); Fz = fmaf(P.kf, Az, Fz);
            } else {                                // circular field; current from omega or from w
                const float ux = vx - my_v.x, uy = vy - my_v.y, uz = vz - my_v.z;
                const bool cur = HET && P.hz == 1;
                const float cwx = cur ? ux : P.wx, cwy = cur ? uy : P.wy, cwz = cur ? uz : P.wz;
                float Gs = 0, Sx = 0, Sy = 0, Sz = 0;
#pragma unroll 4
                for (int i = 0; i < my_n; ++i, q += step3)
                    interact<CUT>(q[0], q[1], q[2], psx, psy, psz, cwx, cwy, cwz, P.R, pr.eps, P.rd, P.tb_a, P.tb_b,
                                  Gs, Sx, Sy, Sz, m2);
                // velocity current: the G w part of the summed current lies along w, and the
                // projection across w removes it exactly; dropping it leaves no FP32 residue
                project_add(ux, uy, uz, P.kf, cwx, cwy, cwz, cur ? 0.0f : Gs, Sx, Sy, Sz, Fx, Fy, Fz);
            }
        }
        const int tile = resident ? (int)max(n_shard, 1ll) : lay.cap;
        for (long long tb = sb; tb < se && !split; tb += tile) {
            const int tn = (int)min((long long)tile, se - tb);
            if (!resident) {
                __syncthreads();
                for (int i = tid; i < tn; i += NT) {
                    lpt[3 * i] = sc.x[tb + i]; lpt[3 * i + 1] = sc.y[tb + i]; lpt[3 * i + 2] = sc.z[tb + i];
                }
                __syncthreads();
            }
            const int t0r = (int)(tb - sb), t1r = t0r + tn;
            for (int r = 0; r < n_runs; ++r) {
                const int4 rr = runs[r];
                const int b = max(rr.x, t0r), e = min(rr.y, t1r);
                if (b >= e) continue;
                const float4 ov = rvel[r];
                // agent position relative to the moving segment
                const float psx = fmaf(-t, ov.x, px), psy = fmaf(-t, ov.y, py), psz = fmaf(-t, ov.z, pz);
                {
                    if (HET && P.hz == 2) {
                        float Ax = 0, Ay = 0, Az = 0;
                        interact_run_apf_aos<L, CUT>(lpt, b - t0r, e - t0r, slice, psx, psy, psz, P.R, pr.eps, P.rd,
                                                     P.ird, P.tb_a, P.tb_b, Ax, Ay, Az, m2);
                        Fx = fmaf(P.kf, Ax, Fx); Fy = fmaf(P.kf, Ay, Fy); Fz = fmaf(P.kf, Az, Fz);
                    } else {
                        const float ux = vx - ov.x, uy = vy - ov.y, uz = vz - ov.z;
                        const bool cur = HET && P.hz == 1;
                        const float cwx = cur ? ux : P.wx, cwy = cur ? uy : P.wy, cwz = cur ? uz : P.wz;
                        float Gs = 0, Sx = 0, Sy = 0, Sz = 0;
                        interact_run_aos<L, CUT>(lpt, b - t0r, e - t0r, slice, psx, psy, psz, cwx, cwy, cwz, P.R,
                                                 pr.eps, P.rd, P.tb_a, P.tb_b, Gs, Sx, Sy, Sz, m2);
                        project_add(ux, uy, uz, P.kf, cwx, cwy, cwz, cur ? 0.0f : Gs, Sx, Sy, Sz, Fx, Fy, Fz);
                    }
                }
            }
        }

        // ---- reduce over the slices of each agent: inside the wave ...
        if constexpr (AW < 64) {
            Fx = agent_allreduce<AW, false>(Fx);
            Fy = agent_allreduce<AW, false>(Fy);
            Fz = agent_allreduce<AW, false>(Fz);
            m2 = agent_allreduce<AW, true>(m2);
        }
        const int par = k & 1;

        // pose agents: the parts of the step that do not depend on f_r, computed while the
        // exchange is in flight -- the attractor's linear wrench, the new angular velocity
        // (f_r is a pure force), its exponential and the coefficients of J(dt omega)
        float aLx = 0, aLy = 0, aLz = 0, jA = 0, jB = 0;
        pose::Q dq{1.f, 0.f, 0.f, 0.f};
        double Af[21];                      // arm agents: factor of J J^T + lambda^2 I
        auto pose_early = [&]() {
            float phx, phy, phz, tx, ty, tz, rx, ry, rz;
            pose::so3_log(pose::qmul(pose::Q{qr.w, -qr.x, -qr.y, -qr.z},
                                     pose::Q{pr.qg[0], pr.qg[1], pr.qg[2], pr.qg[3]}), phx, phy, phz);
            pose::qrot(qr, -1.0f, gx - px, gy - py, gz - pz, tx, ty, tz);
            pose::jac_apply(phx, phy, phz, -1.0f, tx, ty, tz, rx, ry, rz);
            aLx = fmaf(P.ka, rx, -P.da * ux);
            aLy = fmaf(P.ka, ry, -P.da * uy);
            aLz = fmaf(P.ka, rz, -P.da * uz);
            const float hr = 0.5f * pr.dt * P.ir;
            ox = fmaf(hr, fmaf(P.kr, phx, -P.dr * ox), ox);
            oy = fmaf(hr, fmaf(P.kr, phy, -P.dr * oy), oy);
            oz = fmaf(hr, fmaf(P.kr, phz, -P.dr * oz), oz);
            if constexpr (ARM) {
                // the factor of J J^T + lambda^2 I at the current joints (Eq. 12), from the columns
                // the last forward kinematics left on the joint lanes
                arm::factor_cols<AW>(colj, pr.arm_lam2, Af);
            } else {
                const float ax = pr.dt * ox, ay = pr.dt * oy, az = pr.dt * oz;
                dq = pose::so3_exp(ax, ay, az);
                pose::jac_coeffs(ax, ay, az, 1.0f, jA, jB);
            }
        };

        // running costs that do not depend on this step's force (Eqs. 17, 19, 20): p^(k), v^(k-1), F^(k-1), F^(k-2)
        auto costs_early = [&]() {
            if constexpr (POSE) pose_early();
            const float ex = gx - px, ey = gy - py, ez = gz - pz;
            const float dgoal = __builtin_amdgcn_sqrtf(fmaf(ez, ez, fmaf(ey, ey, ex * ex)));
            kahan_add(sg, cg, fminf(dgoal, pr.r_cost) * inv_rc);
            if constexpr (POSE) {
                if (k >= 2) kahan_add(sp, cp, __builtin_amdgcn_sqrtf(fmaf(D1z, D1z, fmaf(D1y, D1y, D1x * D1x))));
                if (k >= 4) {       // p^(k) - 3 p^(k-1) + 3 p^(k-2) - p^(k-3) from the increments
                    const float jx = (D1x - D2x) - (D2x - D3x), jy = (D1y - D2y) - (D2y - D3y);
                    const float jz = (D1z - D2z) - (D2z - D3z);
                    kahan_add(sj, cj, fmaf(jz, jz, fmaf(jy, jy, jx * jx)));
                }
            } else {
                if (k >= 2) kahan_add(sp, cp, pr.dt * __builtin_amdgcn_sqrtf(fmaf(vz, vz, fmaf(vy, vy, vx * vx))));
                if (k >= 4) {
                    const float jx = hj * (F1x - F2x), jy = hj * (F1y - F2y), jz = hj * (F1z - F2z);
                    kahan_add(sj, cj, fmaf(jz, jz, fmaf(jy, jy, jx * jx)));
                }
            }
        };
        // device-scope exchange of the group's shard totals, summed in shard order (run by the lead wave)
        // Cross-shard exchange of the group's partial sums, in two halves so that work
        // independent of the total force runs while the words travel.  When the group's
        // 4 S AW words fit one wave, one store instruction publishes this shard's slot
        // (lane l holds component l & 3 of agent l >> 2) and one load instruction polls
        // every slot of the group; otherwise each lane handles whole slots.
        constexpr bool kVecX = 4 * AW <= 64;
        const unsigned tag = (unsigned)k;
        unsigned long long *const garea = xc.partial + kSlotWords * ((size_t)(par * GW + gw) * S * AW);
        auto publish = [&](float Fx_, float Fy_, float Fz_, float m2_) {
            if (kVecX && 4 * S * AW <= 64) {
                const int pa = lane >> 2, pc = lane & 3;
                float v;
                if constexpr (AW == 1) {
                    v = pc == 0 ? Fx_ : pc == 1 ? Fy_ : pc == 2 ? Fz_ : m2_;
                } else {
                    const int src = (pa < AW ? pa : 0) << 2;      // byte address of agent pa's lane
                    const float x = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(Fx_)));
                    const float y = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(Fy_)));
                    const float z = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(Fz_)));
                    const float m = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(m2_)));
                    v = pc == 0 ? x : pc == 1 ? y : pc == 2 ? z : m;
                }
                if (lane < 4 * AW) st64_agent(garea + (size_t)s * AW * kSlotWords + lane, xword(v, tag));
            } else if (lane < AW) {
                unsigned long long *slot = garea + kSlotWords * ((size_t)s * AW + lane);
                st64_agent(slot, xword(Fx_, tag));
                st64_agent(slot + 1, xword(Fy_, tag));
                st64_agent(slot + 2, xword(Fz_, tag));
                st64_agent(slot + 3, xword(m2_, tag));
            }
        };
        auto collect = [&](float &Fx_, float &Fy_, float &Fz_, float &m2_) {
            unsigned long long t_wait = xc.fine ? __builtin_amdgcn_s_memrealtime() : 0ull;
            if (kVecX && 4 * S * AW <= 64) {
                const bool poller = lane < 4 * S * AW;
                unsigned long long q = 0;
                unsigned spins = 0;
                while (true) {
                    if (poller) q = ld64_agent(garea + lane);
                    if (__all(!poller || xtag(q) == tag)) break;
                    if ((++spins & 63u) == 0 || xc.fine) {
                        if (slow_check(xc, t_wait, spins)) break;
                    }
                }
                if (poller) reinterpret_cast<float *>(xtw)[lane] = xval(q);
            } else {
                // each lane polls the four words of one (shard, agent) slot until all carry this step's tag
                for (int l = lane; l < S * AW; l += 64) {
                    const unsigned long long *slot = garea + kSlotWords * (size_t)l;
                    unsigned long long q0, q1, q2, q3;
                    unsigned spins = 0;
                    while (true) {                   // the four loads are in flight together
                        q0 = ld64_agent(slot); q1 = ld64_agent(slot + 1); q2 = ld64_agent(slot + 2);
                        q3 = ld64_agent(slot + 3);
                        if (xtag(q0) == tag && xtag(q1) == tag && xtag(q2) == tag && xtag(q3) == tag) break;
                        __builtin_amdgcn_s_sleep(2);
                        if ((++spins & 63u) == 0 || xc.fine) {
                            if (slow_check(xc, t_wait, spins)) break;
                        }
                    }
                    xtw[l] = make_float4(xval(q0), xval(q1), xval(q2), xval(q3));
                }
            }
            __builtin_amdgcn_wave_barrier();
            float4 a4 = xtw[a_w];
            for (int r = 1; r < S; ++r) {           // fixed shard order in every shard
                const float4 q = xtw[r * AW + a_w];
                a4.x += q.x; a4.y += q.y; a4.z += q.z; a4.w = fminf(a4.w, q.w);
            }
            __builtin_amdgcn_wave_barrier();        // xtw is rewritten next step
            Fx_ = a4.x; Fy_ = a4.y; Fz_ = a4.z; m2_ = a4.w;
        };
        // net force (Eqs. 6, 7), obstacle cost (Eq. 18), integration (Eqs. 9-11), outputs
        auto finish = [&](float Fx_, float Fy_, float Fz_, float m2_) {
            const float rho_min = (m2_ < INFINITY) ? fmaxf(__builtin_amdgcn_sqrtf(m2_) - P.R, pr.eps) : INFINITY;
            if constexpr (PROBE) {
                if (valid && s == 0 && slice == 0) {
                    pb.f_r[3 * agent] = Fx_; pb.f_r[3 * agent + 1] = Fy_; pb.f_r[3 * agent + 2] = Fz_;
                    if (pb.rho_min) pb.rho_min[agent] = rho_min;
                }
                return;
            }
            if constexpr (POSE) {
                kahan_add(so, co, 1.0f - fminf(rho_min, pr.r_cost) * inv_rc);
                // wrench (Eqs. 6-8): the attractor's part (K e - D v, e = log(M^-1 M_g), K = diag(k_r, k_a),
                // D = diag(d_r, d_a)) came from pose_early; f_r enters as a pure force in the body frame
                float fx, fy, fz;
                pose::qrot(qr, -1.0f, Fx_, Fy_, Fz_, fx, fy, fz);
                // twist (Eqs. 9, 10), inertia diag(i_r, 1/m): omega was advanced in pose_early
                kahan_add(ux, cux, h * (aLx + fx));
                kahan_add(uy, cuy, h * (aLy + fy));
                kahan_add(uz, cuz, h * (aLz + fz));
                float dx, dy, dz;
                if constexpr (ARM) {
                    // joints (Eqs. 12, 13): qdot = J^+ v, q += dt qdot (each on its owner lane);
                    // pose (Eq. 14): M = FK(q)
                    float wa[3], wl[3];
                    pose::qrot(qr, 1.0f, ox, oy, oz, wa[0], wa[1], wa[2]);
                    pose::qrot(qr, 1.0f, ux, uy, uz, wl[0], wl[1], wl[2]);
                    double y[6] = {wa[0], wa[1], wa[2], wl[0], wl[1], wl[2]};
                    arm::solve(Af, y);
                    const float qd = (float)(colj[0] * y[0] + colj[1] * y[1] + colj[2] * y[2] + colj[3] * y[3] +
                                             colj[4] * y[4] + colj[5] * y[5]);
                    if (my_j < pr.arm_n) {
                        arm::advance(jc_own, js_own, 0.5 * (double)pr.dt * (double)qd);
                        q_own += (double)pr.dt * (double)qd;
                    }
                    arm::QD r;
                    double tx, ty, tz;
                    arm::fk_scan<AW>(pr.arm_links, pr.arm_n, a_w, my_j, jc_own, js_own, r, tx, ty, tz, colj);
                    dx = (float)(tx - pdx); dy = (float)(ty - pdy); dz = (float)(tz - pdz);
                    pdx = tx; pdy = ty; pdz = tz;
                    px = (float)tx; py = (float)ty; pz = (float)tz;
                    qr = pose::Q{(float)r.w, (float)r.x, (float)r.y, (float)r.z};
                } else {
                    // pose (Eq. 11): M <- M exp(dt v); the translation moves by R J(dt omega) dt u
                    const float ax = pr.dt * ox, ay = pr.dt * oy, az = pr.dt * oz;
                    float jx, jy, jz;
                    pose::jac_mul(ax, ay, az, jA, jB, pr.dt * ux, pr.dt * uy, pr.dt * uz, jx, jy, jz);
                    pose::qrot(qr, 1.0f, jx, jy, jz, dx, dy, dz);
                    kahan_add(px, cpx, dx);
                    kahan_add(py, cpy, dy);
                    kahan_add(pz, cpz, dz);
                    qr = pose::qnormalize(pose::qmul(qr, dq));
                }
                D3x = D2x; D3y = D2y; D3z = D2z;
                D2x = D1x; D2y = D1y; D2z = D1z;
                D1x = dx; D1y = dy; D1z = dz;
                pose::qrot(qr, 1.0f, ux, uy, uz, vx, vy, vz);        // world velocity of the body origin
                if (writer) {
                    if (out.traj) {
                        float *tr = out.traj + (size_t)agent * traj_row + 3 * (size_t)k;
                        tr[0] = px; tr[1] = py; tr[2] = pz;
                    }
                    if (out.rot) {
                        float *ro = out.rot + ((size_t)agent * (pr.n_steps + 1) + k) * 4;
                        ro[0] = qr.w; ro[1] = qr.x; ro[2] = qr.y; ro[3] = qr.z;
                    }
                    if (out.min_clear) out.min_clear[(size_t)agent * pr.n_steps + (k - 1)] = rho_min;
                }
                if constexpr (ARM) {
                    if (jwriter && out.joints)
                        out.joints[((size_t)agent * (pr.n_steps + 1) + k) * pr.arm_n + my_j] = (float)q_own;
                }
                return;
            }
            const float ex = gx - px, ey = gy - py, ez = gz - pz;
            const float Ftx = fmaf(P.ka, ex, fmaf(-P.da, vx, Fx_));
            const float Fty = fmaf(P.ka, ey, fmaf(-P.da, vy, Fy_));
            const float Ftz = fmaf(P.ka, ez, fmaf(-P.da, vz, Fz_));
            kahan_add(so, co, 1.0f - fminf(rho_min, pr.r_cost) * inv_rc);
            F2x = F1x; F2y = F1y; F2z = F1z;
            F1x = Ftx; F1y = Fty; F1z = Ftz;
            kahan_add(vx, cvx, h * Ftx);
            kahan_add(vy, cvy, h * Fty);
            kahan_add(vz, cvz, h * Ftz);
            kahan_add(px, cpx, pr.dt * vx);
            kahan_add(py, cpy, pr.dt * vy);
            kahan_add(pz, cpz, pr.dt * vz);
            if (writer) {
                if (out.traj) {
                    float *tr = out.traj + (size_t)agent * traj_row + 3 * (size_t)k;
                    tr[0] = px; tr[1] = py; tr[2] = pz;
                }
                if (out.min_clear) out.min_clear[(size_t)agent * pr.n_steps + (k - 1)] = rho_min;
            }
        };

        if constexpr (WS > 1) {
            // across the waves of the workgroup (LDS); the lead wave completes the step for the
            // group and hands the new positions and velocities to the other waves
            if (lane < AW) red[(par * W + wave) * AW + lane] = make_float4(Fx, Fy, Fz, m2);
            __syncthreads();
            if (lead) {
                float4 acc = red[(par * W) * AW + a_w];
#pragma unroll
                for (int r = 1; r < W; ++r) {
                    const float4 q = red[(par * W + r) * AW + a_w];
                    acc.x += q.x; acc.y += q.y; acc.z += q.z; acc.w = fminf(acc.w, q.w);
                }
                Fx = acc.x; Fy = acc.y; Fz = acc.z; m2 = acc.w;
                if (S > 1) publish(Fx, Fy, Fz, m2);
                if constexpr (!PROBE) costs_early();       // overlaps the exchange
                if (S > 1) collect(Fx, Fy, Fz, m2);
                finish(Fx, Fy, Fz, m2);
                if (lane < AW) {
                    tot[2 * lane] = make_float4(px, py, pz, vx);
                    tot[2 * lane + 1] = make_float4(vy, vz, 0.f, 0.f);
                }
            }
            __syncthreads();
            if constexpr (PROBE) break;
            if (!lead) {
                const float4 a = tot[2 * a_w], b = tot[2 * a_w + 1];
                px = a.x; py = a.y; pz = a.z; vx = a.w; vy = b.x; vz = b.y;
            }
        } else {
            if (S > 1) publish(Fx, Fy, Fz, m2);
            if constexpr (!PROBE) costs_early();
            if (S > 1) collect(Fx, Fy, Fz, m2);
            finish(Fx, Fy, Fz, m2);
            if constexpr (PROBE) break;
        }
    }

    // ---- final costs (Eqs. 16-20)
    if (writer) {
        const float N = (float)pr.n_steps;
        const float Cg = sg / N, Co = so / N;
        const float *p0 = pr.start ? pr.start : pr.p0;
        const float s0x = ARM ? a0x : p0[0], s0y = ARM ? a0y : p0[1], s0z = ARM ? a0z : p0[2];
        const float e1x = gx - s0x, e1y = gy - s0y, e1z = gz - s0z;
        const float d1 = sqrtf(fmaf(e1z, e1z, fmaf(e1y, e1y, e1x * e1x)));
        float Cp;
        if (sp >= d1) Cp = (sp > 0.0f) ? 1.0f - d1 / sp : 0.0f;
        else Cp = 1.0f - sp / d1;
        const float dt2 = pr.dt * pr.dt;
        const float Cs = fminf(1.0f, sj / (N * dt2 * dt2 * pr.a_max * pr.a_max));
        const float C = pr.w0 * Cg + pr.w1 * Co + pr.w2 * Cp + pr.w3 * Cs;
        float *co5 = out.cost + 5 * (size_t)agent;
        co5[0] = Cg; co5[1] = Co; co5[2] = Cp; co5[3] = Cs; co5[4] = C;
    }

    // ---- last workgroup: selection rule, then clear the exchange area
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) {
        unsigned prev = __hip_atomic_fetch_add(xc.done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == (unsigned)(G * S - 1)) ? 1 : 0;
    }
    __syncthreads();
    if (!s_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if constexpr (!PROBE) {
        // argmin over C_i (ties -> lowest index, NaN never wins), incumbent rule
        const int inc_in = pr.inc_dev ? pr.inc_dev[0] : pr.incumbent;
        const int inc = (inc_in >= 0 && inc_in < ag.n) ? inc_in : -1;
        const float bound = inc >= 0 ? pr.alpha * out.cost[5 * (size_t)inc + 4] : INFINITY;
        float bv = INFINITY;
        int bi = -1;
        for (int i = tid; i < ag.n; i += NT) {
            float c = out.cost[5 * (size_t)i + 4];
            if (!(c == c)) continue;
            if (inc >= 0 && !(c < bound)) continue;
            if (bi < 0 || c < bv) { bv = c; bi = i; }
        }
        // block reduction of (bv, bi): smaller value, then smaller index
        float *rv = reinterpret_cast<float *>(lds + lp.sel);
        int *ri = reinterpret_cast<int *>(lds + lp.sel) + NT;
        rv[tid] = bv;
        ri[tid] = bi;
        __syncthreads();
        for (int off = NT / 2; off > 0; off >>= 1) {
            if (tid < off) {
                float v2 = rv[tid + off];
                int i2 = ri[tid + off];
                if (i2 >= 0 && (ri[tid] < 0 || v2 < rv[tid] || (v2 == rv[tid] && i2 < ri[tid]))) {
                    rv[tid] = v2;
                    ri[tid] = i2;
                }
            }
            __syncthreads();
        }
        if (tid == 0) {
            int best = ri[0];
            if (best < 0) best = inc;             // no candidate beats the incumbent (or N_a = 0)
            const unsigned stt = ld_agent(xc.status);
            if (stt != 0u) best = stt == 1u ? GMAPP_ETIMEOUT : GMAPP_ECANCELLED;
            out.best[0] = best;
        }
    } else {
        if (tid == 0 && ld_agent(xc.status) != 0u && pb.rho_min) pb.rho_min[0] = NAN;
    }
    if (S > 1) {
        const size_t words = (size_t)2 * GW * S * AW * kSlotWords;
        for (size_t i = tid; i < words; i += NT) st64_agent(xc.partial + i, 0ull);
    }
    if (tid == 0) {
        st_agent(xc.status, 0u);
        st_agent(xc.done, 0u);
    }
}

// ---------------------------------------------------------------- kernel tables
using KFn = void (*)(Scn, Agt, Prm, Out, Probe, Xch, Lay);

template <int AW, int W, int WS, bool HET, int KIND>
KFn pick_cut(int cut, bool probe)
{
    if constexpr (KIND == 2 && AW > kMaxArmAgentsPerGroup) {   // arm agents need a lane per joint in a wave
        (void)cut; (void)probe;
        return nullptr;
    } else if constexpr (KIND != 0) {   // pose and arm agents have no teacher-forced form (the probe takes p, v)
        if (probe) return nullptr;
        return cut ? k_rollout<AW, W, WS, 1, false, HET, KIND> : k_rollout<AW, W, WS, 0, false, HET, KIND>;
    } else {
        if (probe) return cut ? k_rollout<AW, W, WS, 1, true, HET, 0> : k_rollout<AW, W, WS, 0, true, HET, 0>;
        return cut ? k_rollout<AW, W, WS, 1, false, HET, 0> : k_rollout<AW, W, WS, 0, false, HET, 0>;
    }
}

// per-wave groups: every (AW, W); workgroup-wide groups: AW <= 8 with 4, 8 or 16 waves
template <int W, bool HET, int KIND>
KFn pick_a(int AW, bool wg, int cut, bool probe)
{
    if (wg) {
        if constexpr (W >= 4) {
            switch (AW) {
            case 1: return pick_cut<1, W, W, HET, KIND>(cut, probe);
            case 2: return pick_cut<2, W, W, HET, KIND>(cut, probe);
            case 4: return pick_cut<4, W, W, HET, KIND>(cut, probe);
            case 8: return pick_cut<8, W, W, HET, KIND>(cut, probe);
            default: return nullptr;
            }
        }
        return nullptr;
    }
    switch (AW) {
    case 1: return pick_cut<1, W, 1, HET, KIND>(cut, probe);
    case 2: return pick_cut<2, W, 1, HET, KIND>(cut, probe);
    case 4: return pick_cut<4, W, 1, HET, KIND>(cut, probe);
    case 8: return pick_cut<8, W, 1, HET, KIND>(cut, probe);
    case 16: return pick_cut<16, W, 1, HET, KIND>(cut, probe);
    case 32: return pick_cut<32, W, 1, HET, KIND>(cut, probe);
    case 64: return pick_cut<64, W, 1, HET, KIND>(cut, probe);
    default: return nullptr;
    }
}

template <bool HET, int KIND>
KFn pick_kernel_t(int AW, int W, bool wg, int cut, bool probe)
{
    switch (W) {
    case 1: return pick_a<1, HET, KIND>(AW, wg, cut, probe);
    case 2: return pick_a<2, HET, KIND>(AW, wg, cut, probe);
    case 4: return pick_a<4, HET, KIND>(AW, wg, cut, probe);
    case 8: return pick_a<8, HET, KIND>(AW, wg, cut, probe);
    case 16: return pick_a<16, HET, KIND>(AW, wg, cut, probe);
    default: return nullptr;
    }
}

// The kernel for a tiling (nullptr if unsupported); the heterogeneous-field
// instantiations are compiled in their own unit.
KFn pick_kernel_het(int AW, int W, bool wg, int cut, bool probe);
// 6-D pose agents (any heuristic), forward rollouts only; in rollout_pose.hip.
KFn pick_kernel_pose(int AW, int W, bool wg, int cut);
// arm agents (any heuristic), forward rollouts only; in rollout_arm.hip.
KFn pick_kernel_arm(int AW, int W, bool wg, int cut);

}  // namespace gm
