// Many planning problems in one persistent launch: scenes with their own N_O,
// N_a, N_k, cut-off mode and query (the same rollout as k_rollout: Sec. IV-A,
// Alg. 1, Eqs. 6-11 and 15-20).
//
// The grid is fixed (a few workgroups per CU) and its workgroups pull work items
// from a device queue until it is empty.  An item is one block of agents of one
// job; the item's workgroup sweeps the job's whole sphere world every step (LDS
// resident when it fits, else streamed in tiles that all its waves share), so
// items never wait for one another: any workgroup can run any item, and a job's
// result does not depend on what else is in the launch.  Per job the host picks
// one of two item shapes:
//   wave items: every wave is an agent group of AW agents (W * AW per item), the
//               64 lanes of an agent's wave split the points, no barrier per step
//               when the points are resident;
//   workgroup items: AW agents per item, the W * 64 lanes split the points, one
//               LDS reduction and barrier per step (for large worlds: W times
//               shorter items).
// A job may run a step range [k_begin, k_end) of its horizon and keep its agents'
// state (position, velocity, their compensation terms, the last two net forces,
// the running cost sums) in a device buffer between launches.  The last item of a
// job to finish the job's final step applies the selection rule.  The job table
// lives in device memory, so one instantiated graph (table copy + kernel) replays
// every cycle; the queue and completion counters return to zero inside the kernel.
#include "gmapp_internal.h"
#include "pairs.h"

#include <algorithm>
#include <cmath>

namespace gm {

using namespace dev;

namespace {

constexpr int kW = kBatchWaves;

// dynamic LDS: points [cap][3] (x, y, z interleaved) · red float4 [2][W][8] · runs int4 [runs_cap] · rvel float4 [runs_cap] · sel [64 W] x 8 B
struct BPlan {
    size_t cx, cy, cz, red, runs, rvel, sel, total;
};

__host__ __device__ inline BPlan b_plan(const BatchLay &l)
{
    BPlan p;
    const size_t plane = ((size_t)l.cap * 4 + 15) / 16 * 16;
    p.cx = 0; p.cy = plane; p.cz = 2 * plane;
    p.red = 3 * plane;
    p.runs = p.red + (size_t)2 * kW * 8 * 16;
    p.rvel = p.runs + (size_t)l.runs_cap * 16;
    p.sel = p.rvel + (size_t)l.runs_cap * 16;
    p.total = p.sel + (size_t)64 * kW * 8;
    return p;
}

struct Lds {
    float *pt;          // points, interleaved x, y, z per point
    float4 *red;
    int4 *runs;
    float4 *rvel;
    char *sel;
};

// Whether the job was cancelled (its word) or the launch aborted (the context's word):
// system-scope loads of mapped host memory, by one thread.
__device__ __forceinline__ int job_stopped(const BatchJob &jb, const unsigned *abort)
{
    return (abort && ld_system(abort) != 0u) || (jb.cancel && ld_system(jb.cancel) != 0u);
}

// One item: agents [a0, a0 + W * AW) (WS = 1) or [a0, a0 + AW) (WS = W) of job `jb`.
// chk: two LDS flags for the stop checks inside the step loop, used alternately, so that
// between two writes of one flag every wave has passed the barrier after its last read.
template <int AW, int WS, int CUT>
__device__ __forceinline__ void run_item(const BatchJob &jb, int a0, const Lds &m, const BatchLay &lay,
                                                   int &n_runs_sh, int &split_sh, int *chk, const unsigned *abort)
{
    constexpr int NT = 64 * kW;
    constexpr int L = 64 * WS / AW;            // slices per agent
    const Scn &sc = jb.sc;
    const Agt &ag = jb.ag;
    const Prm &pr = jb.pr;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int a_w = lane % AW;
    const int slice = ((wave % WS) * 64 + lane) / AW;
    const int first = a0 + (WS == 1 ? wave * AW : 0);  // the wave's first agent
    const int agent = first + a_w;
    const bool valid = agent < ag.n;
    const bool active = first < ag.n;              // the wave holds at least one agent
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
    P.tb_a = 1.0f / (pr.band * P.rd);
    P.tb_b = P.rd * P.tb_a;

    long long n_pts = sc.n_cap;
    if (sc.n_dev) n_pts = min(max(*sc.n_dev, 0ll), sc.n_cap);
    const bool resident = n_pts <= (long long)lay.cap;
    if (tid == 0) {
        int split = 0;
        n_runs_sh = build_runs(sc, n_pts, 0, n_pts, m.runs, m.rvel, lay.runs_cap, L, split);
        split_sh = split;
    }
    if (resident)
        for (int i = tid; i < (int)n_pts; i += NT) {
            m.pt[3 * i] = sc.x[i]; m.pt[3 * i + 1] = sc.y[i]; m.pt[3 * i + 2] = sc.z[i];
        }
    __syncthreads();
    const int n_runs = n_runs_sh;
    const bool split = resident && split_sh;
    int my_j0 = 0, my_n = 0, my_stride = 1;
    float4 my_v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (split) lane_run(m.runs, m.rvel, n_runs, slice, my_j0, my_n, my_stride, my_v);

    // agent state: initial, or resumed from the job's state buffer
    const int k_begin = jb.k_begin, k_end = jb.k_end;
    float px, py, pz, cpx = 0, cpy = 0, cpz = 0, vx, vy, vz, cvx = 0, cvy = 0, cvz = 0;
    float F1x = 0, F1y = 0, F1z = 0, F2x = 0, F2y = 0, F2z = 0;
    float sg = 0, cg = 0, so = 0, co = 0, sp = 0, cp = 0, sj = 0, cj = 0;
    if (k_begin > 1 && valid) {
        const float *s = jb.state + (size_t)agent * kStateFloats;
        px = s[0]; py = s[1]; pz = s[2]; cpx = s[3]; cpy = s[4]; cpz = s[5];
        vx = s[6]; vy = s[7]; vz = s[8]; cvx = s[9]; cvy = s[10]; cvz = s[11];
        F1x = s[12]; F1y = s[13]; F1z = s[14]; F2x = s[15]; F2y = s[16]; F2z = s[17];
        sg = s[18]; cg = s[19]; so = s[20]; co = s[21]; sp = s[22]; cp = s[23]; sj = s[24]; cj = s[25];
    } else {
        px = pr.p0[0]; py = pr.p0[1]; pz = pr.p0[2];
        vx = pr.v0[0]; vy = pr.v0[1]; vz = pr.v0[2];
    }
    const float gx = pr.goal[0], gy = pr.goal[1], gz = pr.goal[2];
    const float h = 0.5f * pr.dt * pr.inv_mass;
    const float hj = h * pr.dt;                    // dt^2 / 2m
    const float inv_rc = 1.0f / pr.r_cost;
    const bool writer = valid && slice == 0;
    const size_t traj_row = (size_t)(pr.n_steps + 1) * 3;
    if (writer && jb.out.traj && k_begin == 1) {
        float *tr = jb.out.traj + (size_t)agent * traj_row;
        tr[0] = px; tr[1] = py; tr[2] = pz;
    }

    for (int k = k_begin; k < k_end; ++k) {
        // every 64 steps the workgroup looks at the cancel and abort words (one decision for
        // all its waves, which share barriers); a stopped item leaves partial results
        if (((k - k_begin) & 63) == 63) {
            int &f = chk[((k - k_begin) >> 6) & 1];
            if (tid == 0) f = job_stopped(jb, abort);
            __syncthreads();
            if (f) break;
        }
        const float t = fmaf((float)(k - 1), pr.dt, pr.t0);
        float Fx = 0, Fy = 0, Fz = 0, m2 = INFINITY;
        if (split) {
            if (active) {
                const float psx = fmaf(-t, my_v.x, px), psy = fmaf(-t, my_v.y, py), psz = fmaf(-t, my_v.z, pz);
                float Gs = 0, Sx = 0, Sy = 0, Sz = 0;
                const float *q = m.pt + 3 * my_j0;
                const int step3 = 3 * my_stride;
#pragma unroll 4
                for (int i = 0; i < my_n; ++i, q += step3)
                    interact<CUT>(q[0], q[1], q[2], psx, psy, psz, P.wx, P.wy, P.wz, P.R, pr.eps, P.rd, P.tb_a,
                                  P.tb_b, Gs, Sx, Sy, Sz, m2);
                project_add(vx - my_v.x, vy - my_v.y, vz - my_v.z, P.kf, P.wx, P.wy, P.wz, Gs, Sx, Sy, Sz, Fx, Fy,
                            Fz);
            }
        } else {
            const int tile = resident ? (int)max(n_pts, 1ll) : lay.cap;
            for (long long tb = 0; tb < n_pts; tb += tile) {
                const int tn = (int)min((long long)tile, n_pts - tb);
                if (!resident) {
                    __syncthreads();
                    for (int i = tid; i < tn; i += NT) {
                        m.pt[3 * i] = sc.x[tb + i]; m.pt[3 * i + 1] = sc.y[tb + i]; m.pt[3 * i + 2] = sc.z[tb + i];
                    }
                    __syncthreads();
                }
                if (!active) continue;
                const int t0r = (int)tb, t1r = t0r + tn;
                for (int r = 0; r < n_runs; ++r) {
                    const int4 rr = m.runs[r];
                    const int b = max(rr.x, t0r), e = min(rr.y, t1r);
                    if (b >= e) continue;
                    const float4 ov = m.rvel[r];
                    const float psx = fmaf(-t, ov.x, px), psy = fmaf(-t, ov.y, py), psz = fmaf(-t, ov.z, pz);
                    float Gs = 0, Sx = 0, Sy = 0, Sz = 0;
                    interact_run_aos<L, CUT>(m.pt, b - t0r, e - t0r, slice, psx, psy, psz, P.wx, P.wy, P.wz,
                                         P.R, pr.eps, P.rd, P.tb_a, P.tb_b, Gs, Sx, Sy, Sz, m2);
                    project_add(vx - ov.x, vy - ov.y, vz - ov.z, P.kf, P.wx, P.wy, P.wz, Gs, Sx, Sy, Sz, Fx, Fy, Fz);
                }
            }
        }
        // reduce over the agent's slices: inside the wave, then (WS = W) across the waves
        Fx = agent_allreduce<AW, false>(Fx);
        Fy = agent_allreduce<AW, false>(Fy);
        Fz = agent_allreduce<AW, false>(Fz);
        m2 = agent_allreduce<AW, true>(m2);
        if constexpr (WS > 1) {
            const int par = k & 1;                 // double buffer: one barrier per step
            if (lane < AW) m.red[(par * kW + wave) * 8 + lane] = make_float4(Fx, Fy, Fz, m2);
            __syncthreads();
            float4 acc = m.red[(par * kW) * 8 + a_w];
#pragma unroll
            for (int r = 1; r < kW; ++r) {
                const float4 q = m.red[(par * kW + r) * 8 + a_w];
                acc.x += q.x; acc.y += q.y; acc.z += q.z; acc.w = fminf(acc.w, q.w);
            }
            Fx = acc.x; Fy = acc.y; Fz = acc.z; m2 = acc.w;
        }
        const float rho_min = (m2 < INFINITY) ? fmaxf(__builtin_amdgcn_sqrtf(m2) - P.R, pr.eps) : INFINITY;
        const float ex = gx - px, ey = gy - py, ez = gz - pz;
        const float Ftx = fmaf(P.ka, ex, fmaf(-P.da, vx, Fx));
        const float Fty = fmaf(P.ka, ey, fmaf(-P.da, vy, Fy));
        const float Ftz = fmaf(P.ka, ez, fmaf(-P.da, vz, Fz));
        const float dgoal = __builtin_amdgcn_sqrtf(fmaf(ez, ez, fmaf(ey, ey, ex * ex)));
        kahan_add(sg, cg, fminf(dgoal, pr.r_cost) * inv_rc);
        kahan_add(so, co, 1.0f - fminf(rho_min, pr.r_cost) * inv_rc);
        if (k >= 2) kahan_add(sp, cp, pr.dt * __builtin_amdgcn_sqrtf(fmaf(vz, vz, fmaf(vy, vy, vx * vx))));
        if (k >= 4) {
            const float jx = hj * (F1x - F2x), jy = hj * (F1y - F2y), jz = hj * (F1z - F2z);
            kahan_add(sj, cj, fmaf(jz, jz, fmaf(jy, jy, jx * jx)));
        }
        F2x = F1x; F2y = F1y; F2z = F1z;
        F1x = Ftx; F1y = Fty; F1z = Ftz;
        kahan_add(vx, cvx, h * Ftx);
        kahan_add(vy, cvy, h * Fty);
        kahan_add(vz, cvz, h * Ftz);
        kahan_add(px, cpx, pr.dt * vx);
        kahan_add(py, cpy, pr.dt * vy);
        kahan_add(pz, cpz, pr.dt * vz);
        if (writer) {
            if (jb.out.traj) {
                float *tr = jb.out.traj + (size_t)agent * traj_row + 3 * (size_t)k;
                tr[0] = px; tr[1] = py; tr[2] = pz;
            }
            if (jb.out.min_clear) jb.out.min_clear[(size_t)agent * pr.n_steps + (k - 1)] = rho_min;
        }
    }

    const bool final = k_end > pr.n_steps;
    if (writer && !final) {
        float *s = jb.state + (size_t)agent * kStateFloats;
        s[0] = px; s[1] = py; s[2] = pz; s[3] = cpx; s[4] = cpy; s[5] = cpz;
        s[6] = vx; s[7] = vy; s[8] = vz; s[9] = cvx; s[10] = cvy; s[11] = cvz;
        s[12] = F1x; s[13] = F1y; s[14] = F1z; s[15] = F2x; s[16] = F2y; s[17] = F2z;
        s[18] = sg; s[19] = cg; s[20] = so; s[21] = co; s[22] = sp; s[23] = cp; s[24] = sj; s[25] = cj;
    }
    if (writer && final) {                         // Eqs. 16-20
        const float N = (float)pr.n_steps;
        const float Cg = sg / N, Co = so / N;
        const float e1x = gx - pr.p0[0], e1y = gy - pr.p0[1], e1z = gz - pr.p0[2];
        const float d1 = sqrtf(fmaf(e1z, e1z, fmaf(e1y, e1y, e1x * e1x)));
        float Cp;
        if (sp >= d1) Cp = (sp > 0.0f) ? 1.0f - d1 / sp : 0.0f;
        else Cp = 1.0f - sp / d1;
        const float dt2 = pr.dt * pr.dt;
        const float Cs = fminf(1.0f, sj / (N * dt2 * dt2 * pr.a_max * pr.a_max));
        float *co5 = jb.out.cost + 5 * (size_t)agent;
        co5[0] = Cg; co5[1] = Co; co5[2] = Cp; co5[3] = Cs;
        co5[4] = pr.w0 * Cg + pr.w1 * Co + pr.w2 * Cp + pr.w3 * Cs;
    }
}

// Selection rule (argmin over C_i < alpha C_best, ties to the lowest index, NaN
// never wins) by the whole workgroup, after all the job's costs are written.
__device__ void select_best(const BatchJob &jb, char *sel)
{
    constexpr int NT = 64 * kW;
    const int tid = threadIdx.x;
    const int n = jb.ag.n;
    const int inc = (jb.pr.incumbent >= 0 && jb.pr.incumbent < n) ? jb.pr.incumbent : -1;
    const float bound = inc >= 0 ? jb.pr.alpha * jb.out.cost[5 * (size_t)inc + 4] : INFINITY;
    float bv = INFINITY;
    int bi = -1;
    for (int i = tid; i < n; i += NT) {
        const float c = jb.out.cost[5 * (size_t)i + 4];
        if (!(c == c)) continue;
        if (inc >= 0 && !(c < bound)) continue;
        if (bi < 0 || c < bv) { bv = c; bi = i; }
    }
    float *rv = reinterpret_cast<float *>(sel);
    int *ri = reinterpret_cast<int *>(sel) + NT;
    rv[tid] = bv;
    ri[tid] = bi;
    __syncthreads();
    for (int off = NT / 2; off > 0; off >>= 1) {
        if (tid < off) {
            const float v2 = rv[tid + off];
            const int i2 = ri[tid + off];
            if (i2 >= 0 && (ri[tid] < 0 || v2 < rv[tid] || (v2 == rv[tid] && i2 < ri[tid]))) {
                rv[tid] = v2;
                ri[tid] = i2;
            }
        }
        __syncthreads();
    }
    if (tid == 0) jb.out.best[0] = ri[0] >= 0 ? ri[0] : inc;
}

__global__ __launch_bounds__(64 * kW) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_batch(const BatchTable *__restrict__ tab, unsigned *__restrict__ queue,
                                                   unsigned *__restrict__ done, BatchLay lay,
                                                   const unsigned *__restrict__ abort)
{
    extern __shared__ float4 lds4[];
    const BPlan lp = b_plan(lay);
    char *lds = reinterpret_cast<char *>(lds4);
    Lds m;
    m.pt = reinterpret_cast<float *>(lds + lp.cx);
    m.red = reinterpret_cast<float4 *>(lds + lp.red);
    m.runs = reinterpret_cast<int4 *>(lds + lp.runs);
    m.rvel = reinterpret_cast<float4 *>(lds + lp.rvel);
    m.sel = lds + lp.sel;
    __shared__ int s_item, s_nruns, s_split, s_last, s_stop, s_chk[2];
    const int tid = threadIdx.x;
    const int n_jobs = tab->n_jobs, n_items = tab->n_items;
    const BatchJob *jobs = tab->jobs;

    while (true) {
        if (tid == 0) s_item = (int)__hip_atomic_fetch_add(queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int item = s_item;
        if (item >= n_items) break;
        int lo = 0, hi = n_jobs - 1;               // the job: last one whose first item <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].item_base <= item) lo = mid; else hi = mid - 1;
        }
        const BatchJob &jb = jobs[lo];
        const int blk = item - jb.item_base;
        const int a0 = blk * (jb.wg_items ? jb.aw : kW * jb.aw);
        if (tid == 0) s_stop = job_stopped(jb, abort);   // a cancelled job's items are skipped
        __syncthreads();
        const int code = (jb.ag.n <= 0 || s_stop) ? -1 :  // nothing to roll out, only the selection (-1)
                         (jb.wg_items ? 8 : 0) + (jb.pr.cutoff ? 4 : 0) +
                         (jb.aw == 1 ? 0 : jb.aw == 2 ? 1 : jb.aw == 4 ? 2 : 3);
        switch (code) {
        case -1: break;
        case 0: run_item<1, 1, 0>(jb, a0, m, lay, s_nruns, s_split, s_chk, abort); break;
        case 1: run_item<2, 1, 0>(jb, a0, m, lay, s_nruns, s_split, s_chk, abort); break;
        case 2: run_item<4, 1, 0>(jb, a0, m, lay, s_nruns, s_split, s_chk, abort); break;
        case 3: run_item<8, 1, 0>(jb, a0, m, lay, s_nruns, s_split, s_chk, abort); break;
        case 4: run_item<1, 1, 1>(jb, a0, m, lay, s_nruns, s_split, s_chk, abort); break;
        case 5: run_item<2, 1, 1>(jb, a0, m, lay, s_nruns, s_split, s_chk, abort); break;
        case 6: run_item<4, 1, 1>(jb, a0, m, lay, s_nruns, s_split, s_chk, abort); break;
        case 7: run_item<8, 1, 1>(jb, a0, m, lay, s_nruns, s_split, s_chk, abort); break;
        case 8: run_item<1, kW, 0>(jb, a0, m, lay, s_nruns, s_split, s_chk, abort); break;
        case 9: run_item<2, kW, 0>(jb, a0, m, lay, s_nruns, s_split, s_chk, abort); break;
        case 10: run_item<4, kW, 0>(jb, a0, m, lay, s_nruns, s_split, s_chk, abort); break;
        case 11: run_item<8, kW, 0>(jb, a0, m, lay, s_nruns, s_split, s_chk, abort); break;
        case 12: run_item<1, kW, 1>(jb, a0, m, lay, s_nruns, s_split, s_chk, abort); break;
        case 13: run_item<2, kW, 1>(jb, a0, m, lay, s_nruns, s_split, s_chk, abort); break;
        case 14: run_item<4, kW, 1>(jb, a0, m, lay, s_nruns, s_split, s_chk, abort); break;
        default: run_item<8, kW, 1>(jb, a0, m, lay, s_nruns, s_split, s_chk, abort); break;
        }
        if (jb.k_end > jb.pr.n_steps) {            // the job's last item applies the selection rule
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (tid == 0) {
                const unsigned prev =
                    __hip_atomic_fetch_add(&done[lo], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                s_last = (prev == (unsigned)(jb.n_items - 1)) ? 1 : 0;
            }
            __syncthreads();
            if (s_last) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                // the words stay raised until the launch ends, so a job any of whose items was
                // skipped or stopped is seen as cancelled here
                if (tid == 0) s_stop = job_stopped(jb, abort);
                __syncthreads();
                if (s_stop) {
                    if (tid == 0) jb.out.best[0] = GMAPP_ECANCELLED;
                } else {
                    select_best(jb, m.sel);
                }
                if (tid == 0) __hip_atomic_store(&done[lo], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();                           // LDS and s_item are reused by the next item
    }
    // the last workgroup to leave resets the queue for the next launch
    if (tid == 0) {
        const unsigned prev = __hip_atomic_fetch_add(queue + 1, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gridDim.x - 1) {
            __hip_atomic_store(queue, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(queue + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace

size_t batch_lds_bytes(const BatchLay &lay) { return b_plan(lay).total; }

gmapp_status batch_launch_shape(gmapp_ctx *ctx, const BatchLay &lay, int wg_per_cu, BatchLaunch &out)
{
    const void *fn = reinterpret_cast<const void *>(k_batch);
    const size_t shm = batch_lds_bytes(lay);
    if (lay.cap < 64 || shm > (size_t)ctx->lds_per_cu)
        return fail(ctx, GMAPP_ECAPACITY, "batch tile of %d points with %d segment runs needs %zu B of LDS (%d per CU)",
                    lay.cap, lay.runs_cap, shm, ctx->lds_per_cu);
    GM_HIP(ctx, hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    int per_cu = 0;
    GM_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * kW, shm));
    if (per_cu < 1) return fail(ctx, GMAPP_ECAPACITY, "batch kernel does not fit a CU with %zu B of LDS", shm);
    if (wg_per_cu > 0) per_cu = std::min(per_cu, wg_per_cu);
    out.fn = fn;
    out.grid = (unsigned)(per_cu * ctx->n_cu);
    out.block = 64 * kW;
    out.shm = shm;
    out.lay = lay;
    out.queue = ctx->sync + kBatchQueueWord;
    out.done = ctx->sync;
    out.abort = ctx->abort_word;
    return GMAPP_OK;
}

gmapp_status launch_batch(gmapp_ctx *ctx, const BatchTable *tab_dev, const BatchLaunch &l, hipStream_t stream)
{
    hipLaunchKernelGGL(k_batch, dim3(l.grid), dim3(l.block), l.shm, stream, tab_dev, l.queue, l.done, l.lay,
                       l.abort);
    GM_HIP(ctx, hipGetLastError());
    return GMAPP_OK;
}

}  // namespace gm
