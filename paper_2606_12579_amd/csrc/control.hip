// The closed planning loop of Sec. V-B on the device.
//
// A cycle is one rollout (k_rollout) whose start state and incumbent are read
// from device memory, followed by the robot's control steps under the selected
// agent i* (k_control).  Nothing returns to the host between cycles, so a loop
// of C cycles is 2 C + 1 launches in stream order.
//
// k_control is one workgroup of 1024 lanes.  At every control step each lane
// sums i*'s field (the same pair functions as the rollout: circular field with
// omega or with the velocity current, or the APF) over a strided share of the
// spheres, segment by segment; the partials are reduced in a fixed order (wave
// DPP reduction, then the 16 wave sums in index order), and lane 0 applies the
// attractor (Eq. 7) and the integration of Eqs. 9-11 with the control period,
// with Kahan-compensated velocity and position, and hands the new state to all
// lanes through LDS.  With zero steps the kernel answers the control thread's
// query: f_r and rho_min at a given state.
#include "gmapp_internal.h"
#include "pairs.h"

#include <cmath>

namespace gm {

using namespace dev;

namespace {

constexpr int kCtlThreads = 1024;
constexpr int kCtlWaves = kCtlThreads / 64;

struct Ctl {
    float *state;       // [steps + 1][6]: row 0 is read, rows 1..steps are written
    float *clear;       // [max(steps, 1)] rho_min per step, or nullptr
    const int *best;    // the selected agent (device)
    const int *prev;    // the previous cycle's selection (device), or nullptr
    int prev_host;      // the previous selection when prev is nullptr
    int *n_switch;      // switch counter (device), or nullptr
    float *f_out;       // query mode: f_r [3]
    float t0, dt;       // time of step 0, control period
    int steps;          // 0 = query mode
};

// This lane's share of agent P's repulsive force at (p, v) and time t, and of min |d|^2.
template <int CUT>
__device__ __forceinline__ void control_share(const Scn &sc, long long n_pts, const Agent &P, float eps, float px,
                                              float py, float pz, float vx, float vy, float vz, float t, int tid,
                                              float &Fx, float &Fy, float &Fz, float &m2)
{
    const int nseg = sc.n_seg > 0 ? sc.n_seg : 1;
    for (int g = 0; g < nseg; ++g) {
        long long b = 0, e = n_pts;
        float ox = 0.f, oy = 0.f, oz = 0.f;
        if (sc.n_seg > 0) {
            b = min(max((long long)sc.seg_begin[g], 0ll), n_pts);
            e = min(max((long long)sc.seg_begin[g + 1], b), n_pts);
            ox = sc.seg_vel[3 * g]; oy = sc.seg_vel[3 * g + 1]; oz = sc.seg_vel[3 * g + 2];
        }
        // agent position relative to the moving segment
        const float psx = fmaf(-t, ox, px), psy = fmaf(-t, oy, py), psz = fmaf(-t, oz, pz);
        if (P.hz == 2) {
            float Ax = 0, Ay = 0, Az = 0;
            for (long long j = b + tid; j < e; j += kCtlThreads)
                interact_apf<CUT>(sc.x[j], sc.y[j], sc.z[j], psx, psy, psz, P.R, eps, P.rd, P.ird, P.tb_a, P.tb_b, Ax,
                                  Ay, Az, m2);
            Fx = fmaf(P.kf, Ax, Fx); Fy = fmaf(P.kf, Ay, Fy); Fz = fmaf(P.kf, Az, Fz);
        } else {
            const float ux = vx - ox, uy = vy - oy, uz = vz - oz;
            const bool cur = P.hz == 1;
            const float cwx = cur ? ux : P.wx, cwy = cur ? uy : P.wy, cwz = cur ? uz : P.wz;
            float G = 0, Sx = 0, Sy = 0, Sz = 0;
            for (long long j = b + tid; j < e; j += kCtlThreads)
                interact<CUT>(sc.x[j], sc.y[j], sc.z[j], psx, psy, psz, cwx, cwy, cwz, P.R, eps, P.rd, P.tb_a, P.tb_b,
                              G, Sx, Sy, Sz, m2);
            project_add(ux, uy, uz, P.kf, cwx, cwy, cwz, G, Sx, Sy, Sz, Fx, Fy, Fz);
        }
    }
}

template <int CUT>
__global__ __launch_bounds__(kCtlThreads) void k_control(Scn sc, Agt ag, Prm pr, Ctl c)
{
    __shared__ float4 red[kCtlWaves];
    __shared__ float st[6];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int a = c.best[0];
    const bool ok = a >= 0 && a < ag.n;
    if (tid == 0 && c.n_switch) {
        const int prev = c.prev ? c.prev[0] : c.prev_host;
        if (prev >= 0 && ok && a != prev) c.n_switch[0] += 1;
    }
    long long n_pts = sc.n_cap;
    if (sc.n_dev) n_pts = min(max(*sc.n_dev, 0ll), sc.n_cap);
    Agent P;
    const int ai = ok ? a : 0;
    P.ka = ok ? ag.k_a[ai] : 0.f;
    P.da = ok ? ag.d_a[ai] : 0.f;
    P.kf = ok ? ag.k_f[ai] : 0.f;
    P.rd = ok ? ag.r_d[ai] : 1.f;
    P.R = sc.r_obs + (ok ? ag.r_a[ai] : 0.f);
    P.wx = ok ? ag.omega[3 * ai] : 0.f;
    P.wy = ok ? ag.omega[3 * ai + 1] : 0.f;
    P.wz = ok ? ag.omega[3 * ai + 2] : 0.f;
    P.tb_a = 1.0f / (pr.band * P.rd);
    P.tb_b = P.rd * P.tb_a;
    P.hz = (ok && ag.heur) ? ag.heur[ai] : 0;
    if (P.hz != 1 && P.hz != 2) P.hz = 0;
    P.ird = 1.0f / P.rd;

    float px = c.state[0], py = c.state[1], pz = c.state[2];
    float vx = c.state[3], vy = c.state[4], vz = c.state[5];
    float cpx = 0, cpy = 0, cpz = 0, cvx = 0, cvy = 0, cvz = 0;     // Kahan terms (lane 0)
    const float gx = pr.goal[0], gy = pr.goal[1], gz = pr.goal[2];
    const float h = 0.5f * c.dt * pr.inv_mass;
    const int iters = c.steps > 0 ? c.steps : 1;
    for (int j = 0; j < iters; ++j) {
        const float t = fmaf((float)j, c.dt, c.t0);
        float Fx = 0, Fy = 0, Fz = 0, m2 = INFINITY;
        if (ok) control_share<CUT>(sc, n_pts, P, pr.eps, px, py, pz, vx, vy, vz, t, tid, Fx, Fy, Fz, m2);
        Fx = agent_allreduce<1, false>(Fx);
        Fy = agent_allreduce<1, false>(Fy);
        Fz = agent_allreduce<1, false>(Fz);
        m2 = agent_allreduce<1, true>(m2);
        if (lane == 0) red[wave] = make_float4(Fx, Fy, Fz, m2);
        __syncthreads();
        if (tid == 0) {
            float4 acc = red[0];
            for (int w = 1; w < kCtlWaves; ++w) {
                const float4 q = red[w];
                acc.x += q.x; acc.y += q.y; acc.z += q.z; acc.w = fminf(acc.w, q.w);
            }
            float rho = (acc.w < INFINITY) ? fmaxf(sqrtf(acc.w) - P.R, pr.eps) : INFINITY;
            if (!ok) rho = NAN;
            if (c.steps == 0) {
                c.f_out[0] = ok ? acc.x : NAN;
                c.f_out[1] = ok ? acc.y : NAN;
                c.f_out[2] = ok ? acc.z : NAN;
                if (c.clear) c.clear[0] = rho;
            } else {
                if (ok) {
                    const float Ftx = fmaf(P.ka, gx - px, fmaf(-P.da, vx, acc.x));
                    const float Fty = fmaf(P.ka, gy - py, fmaf(-P.da, vy, acc.y));
                    const float Ftz = fmaf(P.ka, gz - pz, fmaf(-P.da, vz, acc.z));
                    kahan_add(vx, cvx, h * Ftx);
                    kahan_add(vy, cvy, h * Fty);
                    kahan_add(vz, cvz, h * Ftz);
                    kahan_add(px, cpx, c.dt * vx);
                    kahan_add(py, cpy, c.dt * vy);
                    kahan_add(pz, cpz, c.dt * vz);
                }
                float *row = c.state + 6 * (size_t)(j + 1);
                row[0] = px; row[1] = py; row[2] = pz; row[3] = vx; row[4] = vy; row[5] = vz;
                if (c.clear) c.clear[j] = rho;
                st[0] = px; st[1] = py; st[2] = pz; st[3] = vx; st[4] = vy; st[5] = vz;
            }
        }
        __syncthreads();
        px = st[0]; py = st[1]; pz = st[2]; vx = st[3]; vy = st[4]; vz = st[5];
    }
}

// Row 0 of the robot's states and N_sw = 0 (a kernel, so that the loop holds no memset node).
__global__ void k_loop_init(float *robot, float p0x, float p0y, float p0z, float v0x, float v0y, float v0z,
                            int *n_switch)
{
    robot[0] = p0x; robot[1] = p0y; robot[2] = p0z;
    robot[3] = v0x; robot[4] = v0y; robot[5] = v0z;
    n_switch[0] = 0;
}

gmapp_status launch_control(gmapp_ctx *ctx, const Scn &sc, const Agt &ag, const Prm &pr, const Ctl &c,
                            hipStream_t stream)
{
    if (pr.cutoff) hipLaunchKernelGGL(k_control<1>, dim3(1), dim3(kCtlThreads), 0, stream, sc, ag, pr, c);
    else hipLaunchKernelGGL(k_control<0>, dim3(1), dim3(kCtlThreads), 0, stream, sc, ag, pr, c);
    GM_HIP(ctx, hipGetLastError());
    return GMAPP_OK;
}

}  // namespace

gmapp_status launch_plan_loop(gmapp_ctx *ctx, const Scn &sc, const Agt &ag, const Prm &pr0, const Tiling &t,
                              const gmapp_loop_config &cfg, const gmapp_loop_outputs &o, hipStream_t stream)
{
    hipLaunchKernelGGL(k_loop_init, dim3(1), dim3(1), 0, stream, o.robot, pr0.p0[0], pr0.p0[1], pr0.p0[2],
                       pr0.v0[0], pr0.v0[1], pr0.v0[2], o.n_switches);
    GM_HIP(ctx, hipGetLastError());
    const size_t steps = (size_t)cfg.ctrl_steps;
    for (int cy = 0; cy < cfg.n_cycles; ++cy) {
        Prm pr = pr0;
        float *row = o.robot + 6 * steps * (size_t)cy;
        pr.start = row;
        pr.inc_dev = cy > 0 ? o.best + (cy - 1) : nullptr;
        pr.t0 = (float)((double)pr0.t0 + (double)cy * (double)cfg.ctrl_steps * (double)cfg.ctrl_dt);
        Out out{nullptr, o.cost + (size_t)cy * (size_t)ag.n * 5, nullptr, o.best + cy};
        gmapp_status st = launch_rollout(ctx, sc, ag, pr, out, nullptr, t, stream);
        if (st) return st;
        Ctl c{row, o.robot_clear ? o.robot_clear + steps * (size_t)cy : nullptr, o.best + cy,
              cy > 0 ? o.best + (cy - 1) : nullptr, pr0.incumbent, o.n_switches, nullptr, pr.t0, cfg.ctrl_dt,
              cfg.ctrl_steps};
        if ((st = launch_control(ctx, sc, ag, pr, c, stream))) return st;
    }
    return GMAPP_OK;
}

gmapp_status launch_control_force(gmapp_ctx *ctx, const Scn &sc, const Agt &ag, const Prm &pr, const int *agent,
                                  const float *state, float t, float *f_r, float *rho_min, hipStream_t stream)
{
    Ctl c{const_cast<float *>(state), rho_min, agent, nullptr, -1, nullptr, f_r, t, 0.0f, 0};
    return launch_control(ctx, sc, ag, pr, c, stream);
}

}  // namespace gm
