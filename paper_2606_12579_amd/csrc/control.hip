// The closed planning loop of Sec. V-B on the device.
//
// A cycle is one rollout (k_rollout) whose start state and incumbent are read
// from device memory, followed by the robot's control steps under the selected
// agent i* (k_control).  Nothing returns to the host between cycles, so a loop
// of C cycles is 2 C + 1 launches in stream order.
//
// k_control spreads each control step over NG workgroups of 256 lanes (a
// cooperative launch; NG = 1 for small clouds).  Workgroup g owns a contiguous
// chunk of the spheres, which it copies into LDS once (the chunk is the same at
// every control step; chunks too large for LDS are read from memory instead).
// Every lane sums i*'s field (the same pair functions as the rollout: circular
// field with omega or with the velocity current, or the APF) over a strided part
// of the chunk, segment by segment, and each workgroup reduces its share in a
// fixed order.  The NG
// partials meet through the context's exchange area: one 4-lane device-scope
// store of four tagged words per workgroup, polled by lane g of wave 0 for
// workgroup g, then a DPP all-reduce across the wave, so every workgroup holds
// the same total bit for bit and integrates the robot identically (attractor of
// Eq. 7, Eqs. 9-11 with the control period, Kahan-compensated velocity and
// position).  Workgroup 0 writes the outputs.  With zero steps the kernel answers
// the control thread's query: f_r and rho_min at a given state.
#include "gmapp_internal.h"
#include "pairs.h"

#include <algorithm>
#include <cmath>

namespace gm {

using namespace dev;

namespace {

constexpr int kCtlThreads = 256;
constexpr int kCtlWaves = kCtlThreads / 64;
constexpr int kCtlMaxGroups = 64;                 // one wave polls every workgroup's slot
constexpr long long kCtlPointsPerGroup = 2048;
constexpr size_t kCtlLdsBytes = 96 * 1024;        // largest chunk staged in LDS
constexpr int kCtlMaxRuns = kMaxControlSegments; // segment runs of a chunk held in LDS

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
    int staged;         // 1: each workgroup's chunk is held in LDS
};

// A run: the part [b, e) of one segment (moving with velocity v) inside a chunk.
struct Run {
    long long b, e;
    float vx, vy, vz;
};

// This lane's part of agent P's repulsive force at (p, v) and time t, and of min |d|^2,
// over the runs of its workgroup's chunk [c0, c1) (points in LDS at cl, or in memory
// when cl is null).
template <int CUT>
__device__ __forceinline__ void control_share(const Scn &sc, const Run *runs, int n_runs, long long c0,
                                              const float *cl, const Agent &P, float eps, float px, float py,
                                              float pz, float vx, float vy, float vz, float t, int tid, float &Fx,
                                              float &Fy, float &Fz, float &m2)
{
    auto point = [&](long long j, float &qx, float &qy, float &qz) {
        if (cl) {
            const float *q = cl + 3 * (j - c0);
            qx = q[0]; qy = q[1]; qz = q[2];
        } else {
            qx = sc.x[j]; qy = sc.y[j]; qz = sc.z[j];
        }
    };
    for (int r = 0; r < n_runs; ++r) {
        const Run rn = runs[r];
        // agent position relative to the moving segment
        const float psx = fmaf(-t, rn.vx, px), psy = fmaf(-t, rn.vy, py), psz = fmaf(-t, rn.vz, pz);
        if (P.hz == 2) {
            float Ax = 0, Ay = 0, Az = 0;
#pragma unroll 4
            for (long long j = rn.b + tid; j < rn.e; j += kCtlThreads) {
                float qx, qy, qz;
                point(j, qx, qy, qz);
                interact_apf<CUT>(qx, qy, qz, psx, psy, psz, P.R, eps, P.rd, P.ird, P.tb_a, P.tb_b, Ax, Ay, Az, m2);
            }
            Fx = fmaf(P.kf, Ax, Fx); Fy = fmaf(P.kf, Ay, Fy); Fz = fmaf(P.kf, Az, Fz);
        } else {
            const float ux = vx - rn.vx, uy = vy - rn.vy, uz = vz - rn.vz;
            const bool cur = P.hz == 1;
            const float cwx = cur ? ux : P.wx, cwy = cur ? uy : P.wy, cwz = cur ? uz : P.wz;
            float G = 0, Sx = 0, Sy = 0, Sz = 0;
#pragma unroll 4
            for (long long j = rn.b + tid; j < rn.e; j += kCtlThreads) {
                float qx, qy, qz;
                point(j, qx, qy, qz);
                interact<CUT>(qx, qy, qz, psx, psy, psz, cwx, cwy, cwz, P.R, eps, P.rd, P.tb_a, P.tb_b, G, Sx, Sy, Sz,
                              m2);
            }
            project_add(ux, uy, uz, P.kf, cwx, cwy, cwz, cur ? 0.0f : G, Sx, Sy, Sz, Fx, Fy, Fz);   // G w lies along w
        }
    }
}

template <int CUT>
__global__ __launch_bounds__(kCtlThreads) void k_control(Scn sc, Agt ag, Prm pr, Ctl c, Xch xc)
{
    __shared__ float4 red[kCtlWaves];
    __shared__ float st[8];
    __shared__ int s_last, s_nruns;
    __shared__ Run s_runs[kCtlMaxRuns];
    extern __shared__ float4 cl4[];           // staged chunk, x y z interleaved
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int NG = gridDim.x, wg = blockIdx.x;
    const bool out_wg = wg == 0;
    const int a = c.best[0];
    const bool ok = a >= 0 && a < ag.n;
    if (out_wg && tid == 0 && c.n_switch) {
        const int prev = c.prev ? c.prev[0] : c.prev_host;
        if (prev >= 0 && ok && a != prev) c.n_switch[0] += 1;
    }
    long long n_pts = sc.n_cap;
    if (sc.n_dev) n_pts = min(max(*sc.n_dev, 0ll), sc.n_cap);
    const long long c0 = n_pts * wg / NG, c1 = n_pts * (wg + 1) / NG;
    // the chunk's runs (segment parts and their velocities), listed once
    if (tid == 0) {
        int nr = 0;
        if (sc.n_seg <= 0) {
            if (c0 < c1) s_runs[nr++] = Run{c0, c1, 0.f, 0.f, 0.f};
        } else {
            for (int g = 0; g < sc.n_seg; ++g) {
                long long b = min(max((long long)sc.seg_begin[g], 0ll), n_pts);
                long long e = min(max((long long)sc.seg_begin[g + 1], b), n_pts);
                b = max(b, c0);
                e = min(e, c1);
                if (b >= e) continue;
                if (nr == kCtlMaxRuns) break;         // the host admits at most kCtlMaxRuns segments
                s_runs[nr++] = Run{b, e, sc.seg_vel[3 * g], sc.seg_vel[3 * g + 1], sc.seg_vel[3 * g + 2]};
            }
        }
        s_nruns = nr;
    }
    __syncthreads();
    const int n_runs = s_nruns;
    float *cl = nullptr;
    if (c.staged) {
        cl = reinterpret_cast<float *>(cl4);
        for (long long i = tid; i < c1 - c0; i += kCtlThreads) {
            cl[3 * i] = sc.x[c0 + i]; cl[3 * i + 1] = sc.y[c0 + i]; cl[3 * i + 2] = sc.z[c0 + i];
        }
        __syncthreads();
    }
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
    bool failed = false;
    for (int j = 0; j < iters && !failed; ++j) {
        const float t = fmaf((float)j, c.dt, c.t0);
        float Fx = 0, Fy = 0, Fz = 0, m2 = INFINITY;
        if (ok) control_share<CUT>(sc, s_runs, n_runs, c0, cl, P, pr.eps, px, py, pz, vx, vy, vz, t, tid, Fx, Fy, Fz, m2);
        Fx = agent_allreduce<1, false>(Fx);
        Fy = agent_allreduce<1, false>(Fy);
        Fz = agent_allreduce<1, false>(Fz);
        m2 = agent_allreduce<1, true>(m2);
        if (lane == 0) red[wave] = make_float4(Fx, Fy, Fz, m2);
        __syncthreads();
        if (wave == 0) {
            float4 acc = red[0];
            for (int w = 1; w < kCtlWaves; ++w) {
                const float4 q = red[w];
                acc.x += q.x; acc.y += q.y; acc.z += q.z; acc.w = fminf(acc.w, q.w);
            }
            if (NG > 1) {
                // publish this workgroup's four words, then gather every workgroup's
                const unsigned tag = (unsigned)(j + 1);
                unsigned long long *area = xc.partial + (size_t)(j & 1) * 4 * NG;
                if (lane < 4) {
                    const float v = lane == 0 ? acc.x : lane == 1 ? acc.y : lane == 2 ? acc.z : acc.w;
                    st64_agent(area + 4 * wg + lane, xword(v, tag));
                }
                unsigned long long q0 = 0, q1 = 0, q2 = 0, q3 = 0;
                const bool poller = lane < NG;
                unsigned spins = 0;
                unsigned long long t_wait = xc.fine ? __builtin_amdgcn_s_memrealtime() : 0ull;
                while (true) {
                    if (poller) {
                        const unsigned long long *slot = area + 4 * lane;
                        q0 = ld64_agent(slot); q1 = ld64_agent(slot + 1); q2 = ld64_agent(slot + 2);
                        q3 = ld64_agent(slot + 3);
                    }
                    const bool mine = !poller || (xtag(q0) == tag && xtag(q1) == tag && xtag(q2) == tag &&
                                                  xtag(q3) == tag);
                    if (__all(mine)) break;
                    if (((++spins & 63u) == 0 || xc.fine) && slow_check(xc, t_wait, spins)) {
                        failed = true;
                        break;
                    }
                }
                float sx = poller ? xval(q0) : 0.f, sy = poller ? xval(q1) : 0.f;
                float sz = poller ? xval(q2) : 0.f, sm = poller ? xval(q3) : INFINITY;
                sx = agent_allreduce<1, false>(sx);
                sy = agent_allreduce<1, false>(sy);
                sz = agent_allreduce<1, false>(sz);
                sm = agent_allreduce<1, true>(sm);
                acc = make_float4(sx, sy, sz, sm);
            }
            if (lane == 0) {
                float rho = (acc.w < INFINITY) ? fmaxf(sqrtf(acc.w) - P.R, pr.eps) : INFINITY;
                if (!ok || failed) rho = NAN;
                if (c.steps == 0) {
                    if (out_wg) {
                        c.f_out[0] = (ok && !failed) ? acc.x : NAN;
                        c.f_out[1] = (ok && !failed) ? acc.y : NAN;
                        c.f_out[2] = (ok && !failed) ? acc.z : NAN;
                        if (c.clear) c.clear[0] = rho;
                    }
                } else {
                    if (failed) {
                        px = py = pz = vx = vy = vz = NAN;
                    } else if (ok) {
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
                    if (out_wg) {
                        float *row = c.state + 6 * (size_t)(j + 1);
                        row[0] = px; row[1] = py; row[2] = pz; row[3] = vx; row[4] = vy; row[5] = vz;
                        if (c.clear) c.clear[j] = rho;
                    }
                    st[0] = px; st[1] = py; st[2] = pz; st[3] = vx; st[4] = vy; st[5] = vz;
                }
                st[6] = failed ? 1.f : 0.f;
            }
        }
        __syncthreads();
        px = st[0]; py = st[1]; pz = st[2]; vx = st[3]; vy = st[4]; vz = st[5];
        failed = st[6] != 0.f;
    }
    if (NG > 1) {
        // the last workgroup out clears the exchange words and the counters for the next launch
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0) {
            const unsigned prev = __hip_atomic_fetch_add(xc.done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            s_last = prev == (unsigned)(NG - 1) ? 1 : 0;
        }
        __syncthreads();
        if (!s_last) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        for (int i = tid; i < 8 * NG; i += kCtlThreads) st64_agent(xc.partial + i, 0ull);
        if (tid == 0) {
            st_agent(xc.status, 0u);
            st_agent(xc.done, 0u);
        }
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
    const long long ng = (sc.n_cap + kCtlPointsPerGroup - 1) / kCtlPointsPerGroup;
    const int cap = std::max(1, std::min(kCtlMaxGroups, ctx->n_cu));
    const int NG = (int)std::min<long long>(std::max<long long>(ng, 1), cap);
    // largest chunk: n * (g + 1) / NG - n * g / NG <= ceil(n / NG) for the capacity n >= N_O
    const size_t chunk = (size_t)((sc.n_cap + NG - 1) / NG);
    const size_t shm = chunk * 3 * sizeof(float);
    Ctl c_ = c;
    c_.staged = (shm > 0 && shm <= kCtlLdsBytes) ? 1 : 0;
    const unsigned dyn = c_.staged ? (unsigned)shm : 0u;
    Xch xc = make_xch(ctx, NG, 1);
    const void *fn = pr.cutoff ? reinterpret_cast<const void *>(k_control<1>)
                               : reinterpret_cast<const void *>(k_control<0>);
    Scn s_ = sc;
    Agt a_ = ag;
    Prm p_ = pr;
    void *args[] = {(void *)&s_, (void *)&a_, (void *)&p_, (void *)&c_, (void *)&xc};
    GM_HIP(ctx, hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCtlLdsBytes));
    if (NG > 1) GM_HIP(ctx, hipLaunchCooperativeKernel(fn, dim3(NG), dim3(kCtlThreads), args, dyn, stream));
    else GM_HIP(ctx, hipLaunchKernel(fn, dim3(1), dim3(kCtlThreads), args, dyn, stream));
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
