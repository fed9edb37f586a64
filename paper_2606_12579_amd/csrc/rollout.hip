// Forward rollout of N_a circular-field agents over N_k steps (G-MAPP, Sec. IV-A
// and Alg. 1), one persistent launch per planning cycle, for gfx950 (CDNA4).
//
// Work decomposition
//   A workgroup owns A agents ("agent group") and one shard of the sphere world:
//   a contiguous range of the N_O points.  Its 64*W lanes are (agent, slice)
//   pairs: lane = agent + A * slice, so each agent's share of the shard is split
//   over L = 64*W/A slices.  The shard's points sit in LDS (SoA x|y|z) for the
//   whole rollout when they fit, else they are streamed through LDS tiles each
//   step.  Every point read from LDS is used by A lanes at once (LDS broadcast).
//   S workgroups (shards) cover one agent group; after each step they exchange
//   their partial sums through the context arena (one agent-scope release and
//   acquire per step) and each adds the S partials in shard order, so all
//   shards hold bit-identical agent states.  Shards of one group are placed on
//   one XCD (workgroups are dispatched round-robin over the 8 XCDs).
//
// Per interaction (agent i, sphere j) the lane evaluates the factored form of
// Eq. (2) with the current vector c = omega - n (n . omega):
//   f_j = g_j k_f |w| P_w (omega - n_j (n_j . omega)),  g_j = [rho_j <= r_d] / rho_j,
// where P_w projects out w (the relative velocity, uniform over a segment) so
//   sum_j f_j = k_f |w| P_w (omega G - S),  G = sum g_j,  S = sum g_j (d_j . omega) d_j / |d_j|^2.
// The lane accumulates G, S (4 floats) and min |d|^2 over its points with
// 20 VALU ops and 2 transcendentals (rsq, rcp) per interaction; P_w is applied
// once per segment run.  rho_min^(k) = max(sqrt(min |d|^2) - (r_O + r_a), eps).
//
// Integration (Eqs. 6, 7, 9-11; explicit: forces use v^(k-1)) and the running
// costs (Eqs. 17-20) are O(1) per agent per step; positions, velocities and
// cost sums carry Kahan compensation.  The jerk of Eq. (20) uses the identity
// p^(k) - 3p^(k-1) + 3p^(k-2) - p^(k-3) = (dt^2 / 2m) (F^(k-1) - F^(k-2)).
// The last workgroup to finish applies the selection rule and resets the
// exchange area to zero for the next launch.
#include "gmapp_internal.h"

#include <algorithm>
#include <cmath>

namespace gm {

namespace {

constexpr float kTiny = 1e-30f;                 // keeps |d|^2 > 0 (agent on a sphere centre)
constexpr unsigned long long kWatchdogTicks = 400000000ull;  // 4 s of the 100 MHz real-time clock

__device__ __forceinline__ void kahan_add(float &s, float &c, float x)
{
    float y = x - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
}

// One agent-sphere interaction (factored Eq. 2), accumulated into G, S, min r2.
template <int CUT>
__device__ __forceinline__ void interact(float qx, float qy, float qz, float psx, float psy, float psz, float wx,
                                         float wy, float wz, float R, float eps, float rd, float tb_a, float tb_b,
                                         float &G, float &Sx, float &Sy, float &Sz, float &m2)
{
    float dx = psx - qx, dy = psy - qy, dz = psz - qz;
    float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, kTiny)));
    float ri = __builtin_amdgcn_rsqf(r2);
    float rho = fmaxf(fmaf(r2, ri, -R), eps);
    float h = __builtin_amdgcn_rcpf(rho * r2);          // 1 / (rho |d|^2)
    if constexpr (CUT == 0) {
        h = (rho <= rd) ? h : 0.0f;
    } else {                                            // C1 smoothstep taper
        float s = __builtin_amdgcn_fmed3f(fmaf(-rho, tb_a, tb_b), 0.0f, 1.0f);
        h *= (s * s) * fmaf(-2.0f, s, 3.0f);
    }
    G = fmaf(h, r2, G);
    float dw = fmaf(dz, wz, fmaf(dy, wy, dx * wx));
    float sc = h * dw;
    Sx = fmaf(sc, dx, Sx);
    Sy = fmaf(sc, dy, Sy);
    Sz = fmaf(sc, dz, Sz);
    m2 = fminf(m2, r2);
}

// Points [b, e) of the LDS tile, slice `sl` of L.
template <int L, int CUT>
__device__ __forceinline__ void interact_run(const float *__restrict__ lx, const float *__restrict__ ly,
                                             const float *__restrict__ lz, int b, int e, int sl, float psx,
                                             float psy, float psz, float wx, float wy, float wz, float R,
                                             float eps, float rd, float tb_a, float tb_b, float &G, float &Sx,
                                             float &Sy, float &Sz, float &m2)
{
    const int n = e - b;
    const int full = n / L;
    int j = b + sl;
#pragma unroll 4
    for (int i = 0; i < full; ++i, j += L)
        interact<CUT>(lx[j], ly[j], lz[j], psx, psy, psz, wx, wy, wz, R, eps, rd, tb_a, tb_b, G, Sx, Sy, Sz, m2);
    if (sl < n - full * L)
        interact<CUT>(lx[j], ly[j], lz[j], psx, psy, psz, wx, wy, wz, R, eps, rd, tb_a, tb_b, G, Sx, Sy, Sz, m2);
}

__device__ __forceinline__ unsigned ld_agent(const unsigned *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned *p, unsigned v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct Agent {
    float ka, da, kf, rd, R, wx, wy, wz, tb_a, tb_b;
};

}  // namespace

// PROBE: one teacher-forced step at the given states (no integration, no costs).
template <int A, int W, int CUT, bool PROBE>
__global__ __launch_bounds__(64 * W) void k_rollout(Scn sc, Agt ag, Prm pr, Out out, Probe pb, Xch xc, int tile_cap)
{
    constexpr int NT = 64 * W;
    constexpr int L = NT / A;                     // slices per agent
    static_assert(A >= 1 && A <= NT && NT % A == 0, "agents per block");
    extern __shared__ float4 lds4[];
    float *lx = reinterpret_cast<float *>(lds4);
    float *ly = lx + tile_cap;
    float *lz = ly + tile_cap;
    float4 *red = lds4 + (3 * tile_cap + 3) / 4;  // [2][NT]
    float4 *tot = red + 2 * NT;                   // [A]
    __shared__ int s_last;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int a_loc = tid % A;
    const int slice = tid / A;
    const int S = xc.S, G = xc.G;

    // workgroup -> (agent group g, shard s); for S > 1 the S shards of a group
    // share an XCD (dispatch is round-robin over 8 XCDs)
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

    const int agent = g * A + a_loc;
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

    long long n_pts = sc.n_cap;
    if (sc.n_dev) n_pts = min(max(*sc.n_dev, 0ll), sc.n_cap);
    const long long sb = n_pts * s / S, se = n_pts * (s + 1) / S;
    const long long n_shard = se - sb;
    const bool resident = n_shard <= (long long)tile_cap;

    auto load_tile = [&](long long tb, int cnt) {
        for (int i = tid; i < cnt; i += NT) {
            lx[i] = sc.x[tb + i];
            ly[i] = sc.y[tb + i];
            lz[i] = sc.z[tb + i];
        }
    };
    if (resident) {
        load_tile(sb, (int)n_shard);
        __syncthreads();
    }

    // agent state
    float px, py, pz, vx, vy, vz, t_fixed = 0.0f;
    if constexpr (PROBE) {
        px = pb.p[3 * ai]; py = pb.p[3 * ai + 1]; pz = pb.p[3 * ai + 2];
        vx = pb.v[3 * ai]; vy = pb.v[3 * ai + 1]; vz = pb.v[3 * ai + 2];
        t_fixed = pb.t;
    } else {
        px = pr.p0[0]; py = pr.p0[1]; pz = pr.p0[2];
        vx = pr.v0[0]; vy = pr.v0[1]; vz = pr.v0[2];
    }
    float cpx = 0, cpy = 0, cpz = 0, cvx = 0, cvy = 0, cvz = 0;     // Kahan terms
    float F1x = 0, F1y = 0, F1z = 0, F2x = 0, F2y = 0, F2z = 0;     // F^(k-1), F^(k-2)
    float sg = 0, cg = 0, so = 0, co = 0, sp = 0, cp = 0, sj = 0, cj = 0;  // cost sums
    const float gx = pr.goal[0], gy = pr.goal[1], gz = pr.goal[2];
    const float h = 0.5f * pr.dt * pr.inv_mass;
    const float hj = h * pr.dt;                                     // dt^2 / 2m
    const bool writer = valid && s == 0 && slice == 0 && !PROBE;
    const int n_steps = PROBE ? 1 : pr.n_steps;
    const size_t traj_row = (size_t)(pr.n_steps + 1) * 3;
    if (writer && out.traj) {
        float *tr = out.traj + (size_t)agent * traj_row;
        tr[0] = px; tr[1] = py; tr[2] = pz;
    }
    const unsigned long long t_start = __builtin_amdgcn_s_memrealtime();

    for (int k = 1; k <= n_steps; ++k) {
        const float t = PROBE ? t_fixed : fmaf((float)(k - 1), pr.dt, pr.t0);
        float Fx = 0, Fy = 0, Fz = 0, m2 = INFINITY;

        // ---- pairwise pass over this shard (hot loop)
        for (long long tb = sb; tb < se; tb += tile_cap) {
            const int cnt = (int)min((long long)tile_cap, se - tb);
            if (!resident) {
                __syncthreads();
                load_tile(tb, cnt);
                __syncthreads();
            }
            const long long te = tb + cnt;
            // walk the segment runs covering [tb, te) (uniform control flow)
            int si = 0;
            if (sc.n_seg > 0) {
                int lo = 0, hi = sc.n_seg;               // first segment whose end > tb
                while (lo < hi) {
                    int mid = (lo + hi) >> 1;
                    long long e_mid = min(max((long long)sc.seg_begin[mid + 1], 0ll), n_pts);
                    if (e_mid > tb) hi = mid; else lo = mid + 1;
                }
                si = lo;
            }
            long long c = tb;
            while (c < te) {
                long long re;
                float ox = 0, oy = 0, oz = 0;
                if (si < sc.n_seg) {
                    long long b_s = min(max((long long)sc.seg_begin[si], 0ll), n_pts);
                    long long e_s = min(max((long long)sc.seg_begin[si + 1], 0ll), n_pts);
                    if (b_s <= c) {
                        re = min(e_s, te);
                        ox = sc.seg_vel[3 * si]; oy = sc.seg_vel[3 * si + 1]; oz = sc.seg_vel[3 * si + 2];
                    } else {
                        re = min(b_s, te);
                    }
                } else {
                    re = te;
                }
                if (re <= c) re = te;                    // malformed table: finish the tile as static
                // agent position relative to the moving segment, and relative velocity
                const float psx = fmaf(-t, ox, px), psy = fmaf(-t, oy, py), psz = fmaf(-t, oz, pz);
                float Gs = 0, Sx = 0, Sy = 0, Sz = 0;
                interact_run<L, CUT>(lx, ly, lz, (int)(c - tb), (int)(re - tb), slice, psx, psy, psz, P.wx, P.wy,
                                     P.wz, P.R, pr.eps, P.rd, P.tb_a, P.tb_b, Gs, Sx, Sy, Sz, m2);
                const float ux = vx - ox, uy = vy - oy, uz = vz - oz;
                const float w2 = fmaf(uz, uz, fmaf(uy, uy, ux * ux));
                if (w2 > 0.0f) {
                    const float cx = fmaf(P.wx, Gs, -Sx), cy = fmaf(P.wy, Gs, -Sy), cz = fmaf(P.wz, Gs, -Sz);
                    const float wn = sqrtf(w2);
                    const float wc = fmaf(uz, cz, fmaf(uy, cy, ux * cx)) / w2;
                    const float f = P.kf * wn;
                    Fx = fmaf(f, fmaf(-ux, wc, cx), Fx);
                    Fy = fmaf(f, fmaf(-uy, wc, cy), Fy);
                    Fz = fmaf(f, fmaf(-uz, wc, cz), Fz);
                }
                c = re;
                while (si < sc.n_seg && min(max((long long)sc.seg_begin[si + 1], 0ll), n_pts) <= c) ++si;
            }
        }

        // ---- reduce over the slices of each agent: inside the wave ...
        if constexpr (A < 64) {
#pragma unroll
            for (int off = A; off < 64; off <<= 1) {
                Fx += __shfl_xor(Fx, off, 64);
                Fy += __shfl_xor(Fy, off, 64);
                Fz += __shfl_xor(Fz, off, 64);
                m2 = fminf(m2, __shfl_xor(m2, off, 64));
            }
        }
        // ... then across waves and shards
        constexpr int NR = (A <= 64) ? W : L;    // partials per agent in the workgroup
        const int par = k & 1;
        if (NR > 1 || S > 1) {
            const bool rep = (A <= 64) ? (lane < A) : true;
            const int r_idx = (A <= 64) ? wave : slice;
            if (rep) red[par * NT + r_idx * A + a_loc] = make_float4(Fx, Fy, Fz, m2);
            __syncthreads();
            if (S == 1) {
                float4 acc = red[par * NT + a_loc];
#pragma unroll
                for (int r = 1; r < NR; ++r) {
                    float4 q = red[par * NT + r * A + a_loc];
                    acc.x += q.x; acc.y += q.y; acc.z += q.z; acc.w = fminf(acc.w, q.w);
                }
                Fx = acc.x; Fy = acc.y; Fz = acc.z; m2 = acc.w;
            } else {
                // A <= 64 here (checked on the host): wave 0 publishes and gathers
                if (wave == 0) {
                    float4 acc = make_float4(0.f, 0.f, 0.f, INFINITY);
                    if (lane < A) {
                        acc = red[par * NT + lane];
#pragma unroll
                        for (int r = 1; r < NR; ++r) {
                            float4 q = red[par * NT + r * A + lane];
                            acc.x += q.x; acc.y += q.y; acc.z += q.z; acc.w = fminf(acc.w, q.w);
                        }
                        xc.partial[((size_t)(par * G + g) * S + s) * A + lane] = acc;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    if (lane == 0) st_agent(&xc.flags[g * S + s], (unsigned)k);
                    if (lane < S) {
                        unsigned spins = 0;
                        while (ld_agent(&xc.flags[g * S + lane]) < (unsigned)k) {
                            __builtin_amdgcn_s_sleep(1);
                            if ((++spins & 255u) == 0) {
                                if (ld_agent(xc.status) != 0u) break;
                                if (__builtin_amdgcn_s_memrealtime() - t_start > kWatchdogTicks) {
                                    st_agent(xc.status, 1u);
                                    break;
                                }
                            }
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    if (lane < A) {
                        const float4 *pp = xc.partial + (size_t)(par * G + g) * S * A + lane;
                        float4 a4 = pp[0];
                        for (int r = 1; r < S; ++r) {
                            float4 q = pp[(size_t)r * A];
                            a4.x += q.x; a4.y += q.y; a4.z += q.z; a4.w = fminf(a4.w, q.w);
                        }
                        tot[lane] = a4;
                    }
                }
                __syncthreads();
                float4 a4 = tot[a_loc];
                Fx = a4.x; Fy = a4.y; Fz = a4.z; m2 = a4.w;
            }
        }

        const float rho_min = (m2 < INFINITY) ? fmaxf(sqrtf(m2) - P.R, pr.eps) : INFINITY;
        if constexpr (PROBE) {
            if (valid && s == 0 && slice == 0) {
                pb.f_r[3 * agent] = Fx; pb.f_r[3 * agent + 1] = Fy; pb.f_r[3 * agent + 2] = Fz;
                if (pb.rho_min) pb.rho_min[agent] = rho_min;
            }
            break;
        }

        // ---- net force (Eqs. 6, 7), running costs (Eqs. 17-20), integration (Eqs. 9-11)
        const float ex = gx - px, ey = gy - py, ez = gz - pz;
        const float Ftx = fmaf(P.ka, ex, fmaf(-P.da, vx, Fx));
        const float Fty = fmaf(P.ka, ey, fmaf(-P.da, vy, Fy));
        const float Ftz = fmaf(P.ka, ez, fmaf(-P.da, vz, Fz));
        const float dgoal = sqrtf(fmaf(ez, ez, fmaf(ey, ey, ex * ex)));
        kahan_add(sg, cg, fminf(dgoal, pr.r_cost) / pr.r_cost);
        kahan_add(so, co, 1.0f - fminf(rho_min, pr.r_cost) / pr.r_cost);
        if (k >= 2) kahan_add(sp, cp, pr.dt * sqrtf(fmaf(vz, vz, fmaf(vy, vy, vx * vx))));
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
            if (out.traj) {
                float *tr = out.traj + (size_t)agent * traj_row + 3 * (size_t)k;
                tr[0] = px; tr[1] = py; tr[2] = pz;
            }
            if (out.min_clear) out.min_clear[(size_t)agent * pr.n_steps + (k - 1)] = rho_min;
        }
    }
    // ---- final costs (Eqs. 16-20)
    if (writer) {
        const float N = (float)pr.n_steps;
        const float Cg = sg / N, Co = so / N;
        const float e1x = gx - pr.p0[0], e1y = gy - pr.p0[1], e1z = gz - pr.p0[2];
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

    // ---- last workgroup: selection rule, then reset the exchange area
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
    const int inc = (pr.incumbent >= 0 && pr.incumbent < ag.n) ? pr.incumbent : -1;
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
    float *rv = reinterpret_cast<float *>(red);
    int *ri = reinterpret_cast<int *>(red) + NT;
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
        if (best < 0) best = inc;                 // no candidate beats the incumbent (or N_a = 0)
        if (ld_agent(xc.status) != 0u) best = GMAPP_ETIMEOUT;
        out.best[0] = best;
    }
    }
    for (int i = tid; i < G * S; i += NT) st_agent(&xc.flags[i], 0u);
    if (tid == 0) {
        st_agent(xc.status, 0u);
        st_agent(xc.done, 0u);
    }
}

__global__ void k_write_best(int *best, int v)
{
    best[0] = v;
}

// ---------------------------------------------------------------- host side
namespace {

using KFn = void (*)(Scn, Agt, Prm, Out, Probe, Xch, int);

template <int A, int W>
KFn pick_cut(int cut, bool probe)
{
    if (probe) return cut ? k_rollout<A, W, 1, true> : k_rollout<A, W, 0, true>;
    return cut ? k_rollout<A, W, 1, false> : k_rollout<A, W, 0, false>;
}

template <int W>
KFn pick_a(int A, int cut, bool probe)
{
    switch (A) {
    case 1: return pick_cut<1, W>(cut, probe);
    case 2: return pick_cut<2, W>(cut, probe);
    case 4: return pick_cut<4, W>(cut, probe);
    case 8: return pick_cut<8, W>(cut, probe);
    case 16: return pick_cut<16, W>(cut, probe);
    case 32: return pick_cut<32, W>(cut, probe);
    case 64: return pick_cut<64, W>(cut, probe);
    case 128: if constexpr (W >= 2) return pick_cut<128, W>(cut, probe); else return nullptr;
    case 256: if constexpr (W >= 4) return pick_cut<256, W>(cut, probe); else return nullptr;
    default: return nullptr;
    }
}

KFn pick_kernel(int A, int W, int cut, bool probe)
{
    switch (W) {
    case 1: return pick_a<1>(A, cut, probe);
    case 2: return pick_a<2>(A, cut, probe);
    case 4: return pick_a<4>(A, cut, probe);
    case 8: return pick_a<8>(A, cut, probe);
    default: return nullptr;
    }
}

size_t lds_bytes(const Tiling &t)
{
    const int NT = 64 * t.W;
    return (size_t)((3 * t.tile + 3) / 4) * 16 + (size_t)2 * NT * 16 + (size_t)t.A * 16;
}

}  // namespace

gmapp_status check_tiling(gmapp_ctx *ctx, const Tiling &t, int n_agents, int cutoff)
{
    if (!pick_kernel(t.A, t.W, cutoff, false))
        return fail(ctx, GMAPP_EINVAL, "unsupported tiling: %d agents per block with %d waves", t.A, t.W);
    if (t.S < 1 || t.S > kMaxShards) return fail(ctx, GMAPP_EINVAL, "shards must be in [1, %d]", kMaxShards);
    if (t.S > 1 && t.A > 64) return fail(ctx, GMAPP_EINVAL, "sharded tilings need at most 64 agents per block");
    if (t.tile < 64) return fail(ctx, GMAPP_EINVAL, "tile_points must be >= 64");
    if (lds_bytes(t) > 160 * 1024) return fail(ctx, GMAPP_ECAPACITY, "tile of %d points exceeds LDS", t.tile);
    (void)n_agents;
    return GMAPP_OK;
}

Tiling choose_tiling(const gmapp_ctx *ctx, long long n_points, int n_agents, int n_steps, int n_seg, int cutoff)
{
    (void)n_steps; (void)n_seg; (void)cutoff;
    const int cus = ctx && ctx->n_cu > 0 ? ctx->n_cu : 256;
    Tiling t{8, 4, 1, 8192};
    if (n_agents >= 4 * cus) t.A = 16;
    int G = (n_agents + t.A - 1) / t.A;
    if (G < 1) G = 1;
    // shard the points until the chip is covered, keeping >= 1024 points per shard
    int S = 1;
    while (S * 2 <= kMaxShards && G * S * 2 <= cus && n_points / (S * 2) >= 1024) S *= 2;
    t.S = S;
    long long per = (n_points + S - 1) / S;
    t.tile = (int)std::min<long long>(std::max<long long>(per, 64), 8192);
    t.tile = (t.tile + 63) / 64 * 64;
    return t;
}

gmapp_status launch_rollout(gmapp_ctx *ctx, const Scn &sc, const Agt &ag, const Prm &pr, const Out &out,
                            const Probe *probe, const Tiling &t, hipStream_t stream)
{
    gmapp_status st = check_tiling(ctx, t, ag.n, pr.cutoff);
    if (st) return st;
    const bool is_probe = probe != nullptr;
    if (ag.n == 0) {
        if (!is_probe) hipLaunchKernelGGL(k_write_best, dim3(1), dim3(1), 0, stream, out.best, -1);
        GM_HIP(ctx, hipGetLastError());
        return GMAPP_OK;
    }
    KFn fn = pick_kernel(t.A, t.W, pr.cutoff, is_probe);
    const int G = (ag.n + t.A - 1) / t.A;
    const long long nwg_real = (long long)G * t.S;
    long long nwg = nwg_real;
    if (t.S > 1) nwg = (nwg + 7) / 8 * 8;
    if (nwg_real > kMaxWorkgroups || nwg > kMaxWorkgroups)
        return fail(ctx, GMAPP_ECAPACITY, "%lld workgroups exceed the limit %d", nwg, kMaxWorkgroups);
    const size_t need_partial = (size_t)2 * G * t.S * t.A * sizeof(float4);
    if (t.S > 1 && need_partial > ctx->scratch_bytes)
        return fail(ctx, GMAPP_ENOMEM, "exchange area needs %zu bytes, workspace has %zu", need_partial,
                    ctx->scratch_bytes);
    Xch xc;
    xc.partial = reinterpret_cast<float4 *>(ctx->scratch);
    xc.flags = ctx->sync;
    xc.done = ctx->sync + kMaxWorkgroups;
    xc.status = ctx->sync + kMaxWorkgroups + 16;
    xc.S = t.S;
    xc.G = G;
    Probe pb{};
    if (probe) pb = *probe;
    const size_t shm = lds_bytes(t);
    int tile = t.tile;
    void *args[] = {(void *)&sc, (void *)&ag, (void *)&pr, (void *)&out, (void *)&pb, (void *)&xc, (void *)&tile};
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
