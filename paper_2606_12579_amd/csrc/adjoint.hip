// Adjoint (reverse-mode) rollout: gradients of sum_i gC_i C_i (C_i the total cost
// of Eq. 16) with respect to each agent's k_a, d_a, k_f and rotation vector omega,
// for gfx950.  One persistent launch per call:
//   1. forward rollout storing the agent state every `ckpt_every` steps (LDS);
//   2. for each checkpoint segment, last to first: recompute the segment's steps
//      from its checkpoint, keeping (p^(k), v^(k-1), F^(k)) per step in LDS, then
//      sweep the steps backwards carrying the adjoints of p and v.
// Agent groups span the workgroup (AW agents, 64 W / AW lanes each).  When there
// are fewer groups than CUs, the points are split over S shards (workgroups of one
// cooperative launch, placed on one XCD): every per-step reduction is then
// completed by a tagged exchange through the context arena (as in the forward
// kernel), and all shards add the partials in shard order, so they carry
// bit-identical agent states and adjoints.
//
// Reverse step k (adjoints lp = dL/dp^(k+1), lv = dL/dv^(k)):
//   lv' = lv + dt lp;  lF = (dt / 2m) lv' + (jerk term of Eq. 20 on F^(k))
//   the pair pass at (p^(k), v^(k-1)) returns J_p^T lF, J_w^T lF, J_omega^T lF and
//   lF . F_r / k_f, from the factored force k_f |w| P_w (omega G - S):
//     lc = k_f |w| P_w lF,  a = lc . omega,  per sphere with g = sigma(rho) / rho:
//     d/dp [g (a - (d.omega)(d.lc) / |d|^2)],   d(omega) = G lc - sum g (d.lc) d / |d|^2,
//     d(w) = k_f [ (lF.c) w^ - (w^.lF) c - (w^.c)(lF - w^ (w^.lF)) ],  c = omega G - S
//   lp <- lp - k_a lF + J_p^T lF + dC/dp^(k) (goal, obstacle: the nearest sphere);
//   lv <- lv' - d_a lF + J_w^T lF + dC/dv^(k-1) (path length).
// The hard cut-off of Alg. 1 is differentiated almost everywhere (its jump is
// ignored); the C1 taper is differentiated exactly.
#include "gmapp_internal.h"
#include "pairs.h"

#include <algorithm>
#include <cmath>

namespace gm {

using namespace dev;

namespace {

struct AdjLay {
    int resident, cap, runs_cap, C, n_ckpt;
};

struct AdjPlan {
    size_t cx, cy, cz, runs, rvel, red, xt, ckpt, tape, total;
};

constexpr int kAdjWords = 16;   // exchange words per agent and shard: up to 3 sums + the nearest sphere

// ckpt: [n_ckpt][AW][5] float4 (p, cp, v, cv, F1 | F2 packed as 5 x float4 of 18 floats)
// tape: [C][AW][3] float4 (p^(k), v^(k-1), F^(k))
// red : [2][W][AW][4] float4
// xt  : [S][AW][4] float4 gathered shard partials (S > 1)
__host__ __device__ inline AdjPlan adj_plan(const AdjLay &l, int W, int AW, int S)
{
    AdjPlan p;
    const size_t plane = ((size_t)l.cap * 4 + 15) / 16 * 16;
    p.cx = 0; p.cy = plane; p.cz = 2 * plane;
    p.runs = 3 * plane;
    p.rvel = p.runs + (size_t)l.runs_cap * 16;
    p.red = p.rvel + (size_t)l.runs_cap * 16;
    p.xt = p.red + (size_t)2 * W * AW * 4 * 16;
    p.ckpt = p.xt + (S > 1 ? (size_t)S * AW * 4 * 16 : 0);
    p.tape = p.ckpt + (size_t)l.n_ckpt * AW * 5 * 16;
    p.total = p.tape + (size_t)l.C * AW * 3 * 16;
    return p;
}

struct AdjOut {
    const float *grad_total;
    float *g_ka, *g_da, *g_kf, *g_om;
};

// nearest sphere so far: smaller |d|^2 wins, ties broken on d (the same in every lane)
__device__ __forceinline__ bool nearer(float m2b, float bx, float by, float bz, float m2a, float ax, float ay, float az)
{
    if (m2b != m2a) return m2b < m2a;
    if (bx != ax) return bx < ax;
    if (by != ay) return by < ay;
    return bz < az;
}

template <int AW>
__device__ __forceinline__ void argmin_allreduce(float &m2, float &dx, float &dy, float &dz)
{
    auto step = [&](auto ctrl_tag, auto fetch) {
        (void)ctrl_tag;
        const float m = fetch(m2), x = fetch(dx), y = fetch(dy), z = fetch(dz);
        if (nearer(m, x, y, z, m2, dx, dy, dz)) { m2 = m; dx = x; dy = y; dz = z; }
    };
    auto dpp = [](float v, auto ctrl) {
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), decltype(ctrl)::value, 0xF, 0xF, false));
    };
    if constexpr (AW <= 8) step(0, [&](float v) { return dpp(v, std::integral_constant<int, 0x128>{}); });
    if constexpr (AW <= 4) step(0, [&](float v) { return dpp(v, std::integral_constant<int, 0x124>{}); });
    if constexpr (AW <= 2) step(0, [&](float v) { return dpp(v, std::integral_constant<int, 0x122>{}); });
    if constexpr (AW <= 1) step(0, [&](float v) { return dpp(v, std::integral_constant<int, 0x121>{}); });
    if constexpr (AW <= 16)
        step(0, [&](float v) { return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F)); });
    if constexpr (AW <= 32) {
        const int lane = threadIdx.x & 63;
        step(0, [&](float v) {
            auto sw = __builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v), false, false);
            return __int_as_float(lane < 32 ? sw[1] : sw[0]);
        });
    }
}

// One interaction of the reverse pass (see the file comment).
template <int CUT>
__device__ __forceinline__ void interact_rev(float qx, float qy, float qz, float psx, float psy, float psz,
                                             const Agent &P, float eps, float lcx, float lcy, float lcz, float a,
                                             float &G, float &Sx, float &Sy, float &Sz, float &gpx, float &gpy,
                                             float &gpz, float &gox, float &goy, float &goz, float &m2, float &mx,
                                             float &my, float &mz)
{
    const float dx = psx - qx, dy = psy - qy, dz = psz - qz;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, kTiny)));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float x = fmaf(r2, ri, -P.R);
    const float rho = fmaxf(x, eps);
    const float irho = __builtin_amdgcn_rcpf(rho);
    float sig, dsig;
    if constexpr (CUT == 0) {
        sig = (rho <= P.rd) ? 1.0f : 0.0f;
        dsig = 0.0f;
    } else {
        const float s = __builtin_amdgcn_fmed3f(fmaf(-rho, P.tb_a, P.tb_b), 0.0f, 1.0f);
        sig = (s * s) * fmaf(-2.0f, s, 3.0f);
        dsig = -6.0f * s * (1.0f - s) * P.tb_a;
    }
    const float g = sig * irho;
    const float gprime = (x > eps) ? (dsig - g) * irho : 0.0f;
    const float ir2 = ri * ri;
    const float al = fmaf(dz, P.wz, fmaf(dy, P.wy, dx * P.wx));   // d . omega
    const float be = fmaf(dz, lcz, fmaf(dy, lcy, dx * lcx));      // d . lc
    const float q = g * ir2;
    G += g;
    const float sa = q * al;
    Sx = fmaf(sa, dx, Sx);
    Sy = fmaf(sa, dy, Sy);
    Sz = fmaf(sa, dz, Sz);
    const float coef = gprime * fmaf(-al * be, ir2, a) * ri + 2.0f * q * al * be * ir2;
    const float qb = q * be, qa = q * al;
    gpx += coef * dx - fmaf(qb, P.wx, qa * lcx);
    gpy += coef * dy - fmaf(qb, P.wy, qa * lcy);
    gpz += coef * dz - fmaf(qb, P.wz, qa * lcz);
    gox = fmaf(qb, dx, gox);
    goy = fmaf(qb, dy, goy);
    goz = fmaf(qb, dz, goz);
    if (nearer(r2, dx, dy, dz, m2, mx, my, mz)) { m2 = r2; mx = dx; my = dy; mz = dz; }
}

template <int AW, int W, int CUT>
__global__ __launch_bounds__(64 * W) void k_adjoint(Scn sc, Agt ag, Prm pr, AdjOut io, AdjLay lay, Xch xc)
{
    constexpr int NT = 64 * W;
    constexpr int L = NT / AW;
    extern __shared__ float4 lds4[];
    const int S = xc.S, G = xc.G;
    const AdjPlan lp = adj_plan(lay, W, AW, S);
    char *lds = reinterpret_cast<char *>(lds4);
    float *lx = reinterpret_cast<float *>(lds + lp.cx);
    float *ly = reinterpret_cast<float *>(lds + lp.cy);
    float *lz = reinterpret_cast<float *>(lds + lp.cz);
    int4 *runs = reinterpret_cast<int4 *>(lds + lp.runs);
    float4 *rvel = reinterpret_cast<float4 *>(lds + lp.rvel);
    float4 *red = reinterpret_cast<float4 *>(lds + lp.red);
    float4 *xt = reinterpret_cast<float4 *>(lds + lp.xt);
    float4 *ckpt = reinterpret_cast<float4 *>(lds + lp.ckpt);
    float4 *tape = reinterpret_cast<float4 *>(lds + lp.tape);
    __shared__ int s_nruns, s_split, s_last;

    // workgroup -> (group g, shard s); the S shards of a group share an XCD
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

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int a_w = tid % AW;
    const int slice = tid / AW;
    const bool lead = slice == 0;                 // tid < AW, in wave 0: the agent's lane for tape and checkpoints
    const bool writer = lead && s == 0;
    const int agent = g * AW + a_w;
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
    P.tb_a = 1.0f / (pr.band * P.rd);
    P.tb_b = P.rd * P.tb_a;

    long long n_pts = sc.n_cap;
    if (sc.n_dev) n_pts = min(max(*sc.n_dev, 0ll), sc.n_cap);
    const long long sb = n_pts * s / S, se = n_pts * (s + 1) / S;
    const long long n_shard = se - sb;
    const float *gx_ = sc.x + sb, *gy_ = sc.y + sb, *gz_ = sc.z + sb;   // this shard's points
    if (tid == 0) {
        int split = 0;
        s_nruns = build_runs(sc, n_pts, sb, se, runs, rvel, lay.runs_cap, L, split);
        s_split = split;
    }
    const bool resident = lay.resident && n_shard <= (long long)lay.cap;
    if (resident)
        for (int i = tid; i < (int)n_shard; i += NT) {
            lx[i] = gx_[i]; ly[i] = gy_[i]; lz[i] = gz_[i];
        }
    __syncthreads();
    const int n_runs = s_nruns;
    const bool split = resident && s_split;
    int my_j0 = 0, my_n = 0, my_stride = 1;
    float4 my_v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (split) lane_run(runs, rvel, n_runs, slice, my_j0, my_n, my_stride, my_v);

    const float h = 0.5f * pr.dt * pr.inv_mass, hj = h * pr.dt, inv_rc = 1.0f / pr.r_cost;
    const float gx = pr.goal[0], gy = pr.goal[1], gz = pr.goal[2];
    const int N = pr.n_steps, C = lay.C;
    int par = 0;
    unsigned ev = 0;                              // exchange tag: one per reduction, the same sequence in all shards
    bool failed = false;                          // a wait was cut short: later waits are skipped (gradients NaN)

    // workgroup reduction: sum of up to 3 float4 and the nearest sphere (m2, d)
    auto wg_reduce = [&](float4 *v, int nsum, float &m2, float &mx, float &my, float &mz) {
        for (int i = 0; i < nsum; ++i) {
            v[i].x = agent_allreduce<AW, false>(v[i].x);
            v[i].y = agent_allreduce<AW, false>(v[i].y);
            v[i].z = agent_allreduce<AW, false>(v[i].z);
            v[i].w = agent_allreduce<AW, false>(v[i].w);
        }
        argmin_allreduce<AW>(m2, mx, my, mz);
        float4 *rb = red + (size_t)par * W * AW * 4;
        if (lane < AW) {
            for (int i = 0; i < nsum; ++i) rb[(wave * AW + lane) * 4 + i] = v[i];
            rb[(wave * AW + lane) * 4 + 3] = make_float4(m2, mx, my, mz);
        }
        __syncthreads();
        for (int i = 0; i < nsum; ++i) v[i] = rb[a_w * 4 + i];
        float4 m = rb[a_w * 4 + 3];
        for (int r = 1; r < W; ++r) {
            for (int i = 0; i < nsum; ++i) {
                const float4 q = rb[(r * AW + a_w) * 4 + i];
                v[i].x += q.x; v[i].y += q.y; v[i].z += q.z; v[i].w += q.w;
            }
            const float4 q = rb[(r * AW + a_w) * 4 + 3];
            if (nearer(q.x, q.y, q.z, q.w, m.x, m.y, m.z, m.w)) m = q;
        }
        if (S > 1) {                              // complete the reduction over the shards
            const unsigned tag = ++ev;
            if (wave == 0) {
                if (lane < AW) {
                    unsigned long long *slot =
                        xc.partial + (((size_t)((tag & 1) * G + g) * S + s) * AW + lane) * kAdjWords;
                    for (int i = 0; i < nsum; ++i) {
                        st64_agent(slot + 4 * i, xword(v[i].x, tag));
                        st64_agent(slot + 4 * i + 1, xword(v[i].y, tag));
                        st64_agent(slot + 4 * i + 2, xword(v[i].z, tag));
                        st64_agent(slot + 4 * i + 3, xword(v[i].w, tag));
                    }
                    st64_agent(slot + 4 * nsum, xword(m.x, tag));
                    st64_agent(slot + 4 * nsum + 1, xword(m.y, tag));
                    st64_agent(slot + 4 * nsum + 2, xword(m.z, tag));
                    st64_agent(slot + 4 * nsum + 3, xword(m.w, tag));
                }
                const int nw = 4 * (nsum + 1);
                for (int l = lane; l < S * AW; l += 64) {
                    const unsigned long long *slot =
                        xc.partial + (((size_t)((tag & 1) * G + g) * S + l / AW) * AW + l % AW) * kAdjWords;
                    unsigned long long q[kAdjWords] = {};
                    unsigned spins = 0;
                    unsigned long long t_wait = xc.fine ? __builtin_amdgcn_s_memrealtime() : 0ull;
                    while (!failed) {                // all words of the slot in flight together
                        bool all = true;
                        for (int i = 0; i < nw; ++i) q[i] = ld64_agent(slot + i);
                        for (int i = 0; i < nw; ++i) all = all && xtag(q[i]) == tag;
                        if (all) break;
                        __builtin_amdgcn_s_sleep(2);
                        if (((++spins & 63u) == 0 || xc.fine) && slow_check(xc, t_wait, spins)) {
                            failed = true;
                            break;
                        }
                    }
                    for (int i = 0; i < nsum + 1; ++i)
                        xt[l * 4 + i] = make_float4(xval(q[4 * i]), xval(q[4 * i + 1]), xval(q[4 * i + 2]),
                                                    xval(q[4 * i + 3]));
                }
            }
            __syncthreads();
            for (int i = 0; i < nsum; ++i) v[i] = xt[a_w * 4 + i];      // shard 0, then the others in order
            m = xt[a_w * 4 + nsum];
            for (int r = 1; r < S; ++r) {
                for (int i = 0; i < nsum; ++i) {
                    const float4 q = xt[(r * AW + a_w) * 4 + i];
                    v[i].x += q.x; v[i].y += q.y; v[i].z += q.z; v[i].w += q.w;
                }
                const float4 q = xt[(r * AW + a_w) * 4 + nsum];
                if (nearer(q.x, q.y, q.z, q.w, m.x, m.y, m.z, m.w)) m = q;
            }
        }
        m2 = m.x; mx = m.y; my = m.z; mz = m.w;
        par ^= 1;
    };

    // forward pair pass at (p, v, t): F_r and min |d|^2
    auto fwd_pairs = [&](float px, float py, float pz, float vx, float vy, float vz, float t, float &Fx, float &Fy,
                         float &Fz, float &m2) {
        Fx = Fy = Fz = 0.f;
        m2 = INFINITY;
        auto run = [&](const float4 ov, int b, int e, int j0, int n, int stride, const float *X, const float *Y,
                       const float *Z) {
            const float psx = fmaf(-t, ov.x, px), psy = fmaf(-t, ov.y, py), psz = fmaf(-t, ov.z, pz);
            float Gs = 0, Sx = 0, Sy = 0, Sz = 0;
            (void)b; (void)e;
            int j = j0;
            for (int i = 0; i < n; ++i, j += stride)
                interact<CUT>(X[j], Y[j], Z[j], psx, psy, psz, P.wx, P.wy, P.wz, P.R, pr.eps, P.rd, P.tb_a, P.tb_b, Gs,
                              Sx, Sy, Sz, m2);
            project_add(vx - ov.x, vy - ov.y, vz - ov.z, P.kf, P.wx, P.wy, P.wz, Gs, Sx, Sy, Sz, Fx, Fy, Fz);
        };
        if (split) {
            run(my_v, 0, 0, my_j0, my_n, my_stride, lx, ly, lz);
        } else {
            const int tile = resident ? (int)max(n_shard, 1ll) : lay.cap;
            for (long long tb = 0; tb < n_shard; tb += tile) {
                const int tn = (int)min((long long)tile, n_shard - tb);
                if (!resident) {
                    __syncthreads();
                    for (int i = tid; i < tn; i += NT) {
                        lx[i] = gx_[tb + i]; ly[i] = gy_[tb + i]; lz[i] = gz_[tb + i];
                    }
                    __syncthreads();
                }
                for (int r = 0; r < n_runs; ++r) {
                    const int b = max(runs[r].x, (int)tb), e = min(runs[r].y, (int)tb + tn);
                    if (b >= e) continue;
                    const int first = b - (int)tb + slice;
                    const int n = (e - (int)tb > first) ? (e - (int)tb - first + L - 1) / L : 0;
                    run(rvel[r], b, e, first, n, L, lx, ly, lz);
                }
            }
        }
        float4 v[1] = {make_float4(Fx, Fy, Fz, 0.f)};
        float mx = 0, my = 0, mz = 0;
        wg_reduce(v, 1, m2, mx, my, mz);
        Fx = v[0].x; Fy = v[0].y; Fz = v[0].z;
    };

    // ---- 1. forward rollout with checkpoints and costs
    float px = pr.p0[0], py = pr.p0[1], pz = pr.p0[2], vx = pr.v0[0], vy = pr.v0[1], vz = pr.v0[2];
    float cpx = 0, cpy = 0, cpz = 0, cvx = 0, cvy = 0, cvz = 0;
    float F1x = 0, F1y = 0, F1z = 0, F2x = 0, F2y = 0, F2z = 0;
    float sg = 0, cg = 0, so = 0, co = 0, sp = 0, cp = 0, sj = 0, cj = 0;
    auto step = [&](int k, bool costs) {
        const float t = fmaf((float)(k - 1), pr.dt, pr.t0);
        float Frx, Fry, Frz, m2;
        fwd_pairs(px, py, pz, vx, vy, vz, t, Frx, Fry, Frz, m2);
        const float ex = gx - px, ey = gy - py, ez = gz - pz;
        const float Ftx = fmaf(P.ka, ex, fmaf(-P.da, vx, Frx));
        const float Fty = fmaf(P.ka, ey, fmaf(-P.da, vy, Fry));
        const float Ftz = fmaf(P.ka, ez, fmaf(-P.da, vz, Frz));
        if (costs) {
            const float rho_min = (m2 < INFINITY) ? fmaxf(__builtin_amdgcn_sqrtf(m2) - P.R, pr.eps) : INFINITY;
            const float dgoal = __builtin_amdgcn_sqrtf(fmaf(ez, ez, fmaf(ey, ey, ex * ex)));
            kahan_add(sg, cg, fminf(dgoal, pr.r_cost) * inv_rc);
            kahan_add(so, co, 1.0f - fminf(rho_min, pr.r_cost) * inv_rc);
            if (k >= 2) kahan_add(sp, cp, pr.dt * __builtin_amdgcn_sqrtf(fmaf(vz, vz, fmaf(vy, vy, vx * vx))));
            if (k >= 4) {
                const float jx = hj * (F1x - F2x), jy = hj * (F1y - F2y), jz = hj * (F1z - F2z);
                kahan_add(sj, cj, fmaf(jz, jz, fmaf(jy, jy, jx * jx)));
            }
        }
        F2x = F1x; F2y = F1y; F2z = F1z;
        F1x = Ftx; F1y = Fty; F1z = Ftz;
        kahan_add(vx, cvx, h * Ftx);
        kahan_add(vy, cvy, h * Fty);
        kahan_add(vz, cvz, h * Ftz);
        kahan_add(px, cpx, pr.dt * vx);
        kahan_add(py, cpy, pr.dt * vy);
        kahan_add(pz, cpz, pr.dt * vz);
    };
    for (int k = 1; k <= N; ++k) {
        if ((k - 1) % C == 0 && lead) {
            float4 *c5 = ckpt + ((size_t)((k - 1) / C) * AW + a_w) * 5;
            c5[0] = make_float4(px, py, pz, cpx);
            c5[1] = make_float4(cpy, cpz, vx, vy);
            c5[2] = make_float4(vz, cvx, cvy, cvz);
            c5[3] = make_float4(F1x, F1y, F1z, F2x);
            c5[4] = make_float4(F2y, F2z, 0.f, 0.f);
        }
        step(k, true);
    }
    const float Nf = (float)N;
    const float e1x = gx - pr.p0[0], e1y = gy - pr.p0[1], e1z = gz - pr.p0[2];
    const float d1 = __builtin_amdgcn_sqrtf(fmaf(e1z, e1z, fmaf(e1y, e1y, e1x * e1x)));
    const float Lp = sp;
    const float dCp = (Lp >= d1) ? ((Lp > 0.f) ? d1 / (Lp * Lp) : 0.f) : -1.0f / d1;
    const float dt2 = pr.dt * pr.dt;
    const float jscale = 1.0f / (Nf * dt2 * dt2 * pr.a_max * pr.a_max);
    const float dCs = (sj * jscale < 1.0f) ? jscale : 0.0f;
    const float gC = valid ? io.grad_total[agent] : 0.0f;
    const float cjerk = gC * pr.w3 * dCs * 2.0f * hj * hj;   // d(gC w3 C_smooth) / dD, D = F^(m) - F^(m-1)
    const float cgoal = gC * pr.w0 / Nf * inv_rc, cobs = gC * pr.w1 / Nf * inv_rc, cpath = gC * pr.w2 * dCp * pr.dt;
    __syncthreads();

    // ---- 2. reverse sweep, one checkpoint segment at a time
    float lpx = 0, lpy = 0, lpz = 0, lvx = 0, lvy = 0, lvz = 0;
    float gka = 0, gda = 0, gkf = 0, gox = 0, goy = 0, goz = 0;
    float Fax = 0, Fay = 0, Faz = 0;              // F^(k1 + 1): first force of the later segment
    for (int seg = lay.n_ckpt - 1; seg >= 0; --seg) {
        const int k0 = seg * C + 1, k1 = min(k0 + C - 1, N);
        const float4 *c5 = ckpt + ((size_t)seg * AW + a_w) * 5;
        {
            const float4 c0 = c5[0], c1 = c5[1], c2 = c5[2], c3 = c5[3], c4 = c5[4];
            px = c0.x; py = c0.y; pz = c0.z; cpx = c0.w; cpy = c1.x; cpz = c1.y; vx = c1.z; vy = c1.w;
            vz = c2.x; cvx = c2.y; cvy = c2.z; cvz = c2.w; F1x = c3.x; F1y = c3.y; F1z = c3.z;
            F2x = c3.w; F2y = c4.x; F2z = c4.y;
        }
        const float Fbx = F1x, Fby = F1y, Fbz = F1z;   // F^(k0 - 1)
        for (int k = k0; k <= k1; ++k) {
            float4 *tp = tape + ((size_t)(k - k0) * AW + a_w) * 3;
            if (lead) {
                tp[0] = make_float4(px, py, pz, 0.f);
                tp[1] = make_float4(vx, vy, vz, 0.f);
            }
            step(k, false);
            if (lead) tp[2] = make_float4(F1x, F1y, F1z, 0.f);
        }
        __syncthreads();
        for (int k = k1; k >= k0; --k) {
            const float4 *tp = tape + ((size_t)(k - k0) * AW + a_w) * 3;
            const float4 P4 = tp[0], V4 = tp[1], F4 = tp[2];
            float4 Fm = make_float4(Fbx, Fby, Fbz, 0.f), Fp = make_float4(Fax, Fay, Faz, 0.f);
            if (k > k0) Fm = tape[((size_t)(k - 1 - k0) * AW + a_w) * 3 + 2];
            if (k < k1) Fp = tape[((size_t)(k + 1 - k0) * AW + a_w) * 3 + 2];
            const float lvtx = fmaf(pr.dt, lpx, lvx), lvty = fmaf(pr.dt, lpy, lvy), lvtz = fmaf(pr.dt, lpz, lvz);
            float lFx = h * lvtx, lFy = h * lvty, lFz = h * lvtz;
            if (k >= 3 && k <= N - 1) {               // D^(k) = F^(k) - F^(k-1)
                lFx = fmaf(cjerk, F4.x - Fm.x, lFx); lFy = fmaf(cjerk, F4.y - Fm.y, lFy); lFz = fmaf(cjerk, F4.z - Fm.z, lFz);
            }
            if (k + 1 >= 3 && k + 1 <= N - 1) {       // D^(k+1) = F^(k+1) - F^(k)
                lFx = fmaf(-cjerk, Fp.x - F4.x, lFx); lFy = fmaf(-cjerk, Fp.y - F4.y, lFy); lFz = fmaf(-cjerk, Fp.z - F4.z, lFz);
            }
            // reverse pair pass at (p^(k), v^(k-1), t_k)
            const float t = fmaf((float)(k - 1), pr.dt, pr.t0);
            float gpx = 0, gpy = 0, gpz = 0, lwx = 0, lwy = 0, lwz = 0, lox = 0, loy = 0, loz = 0, lkf = 0;
            float m2 = INFINITY, mx = 0, my = 0, mz = 0;
            auto rrun = [&](const float4 ov, int j0, int n, int stride) {
                const float ux = V4.x - ov.x, uy = V4.y - ov.y, uz = V4.z - ov.z;
                const float w2 = fmaf(uz, uz, fmaf(uy, uy, ux * ux));
                float ex = 0, ey = 0, ez = 0, hx = 0, hy = 0, hz = 0;
                if (w2 > 0.f) {
                    const float iw = __builtin_amdgcn_rsqf(w2), wn = w2 * iw;
                    hx = ux * iw; hy = uy * iw; hz = uz * iw;
                    const float hl = fmaf(hz, lFz, fmaf(hy, lFy, hx * lFx));
                    ex = wn * fmaf(-hx, hl, lFx); ey = wn * fmaf(-hy, hl, lFy); ez = wn * fmaf(-hz, hl, lFz);
                }
                const float lcx = P.kf * ex, lcy = P.kf * ey, lcz = P.kf * ez;
                const float a = fmaf(lcz, P.wz, fmaf(lcy, P.wy, lcx * P.wx));
                const float psx = fmaf(-t, ov.x, P4.x), psy = fmaf(-t, ov.y, P4.y), psz = fmaf(-t, ov.z, P4.z);
                float Gs = 0, Sx = 0, Sy = 0, Sz = 0, ox = 0, oy = 0, oz = 0;
                int j = j0;
                for (int i = 0; i < n; ++i, j += stride)
                    interact_rev<CUT>(lx[j], ly[j], lz[j], psx, psy, psz, P, pr.eps, lcx, lcy, lcz, a, Gs, Sx, Sy, Sz,
                                      gpx, gpy, gpz, ox, oy, oz, m2, mx, my, mz);
                const float cx = fmaf(P.wx, Gs, -Sx), cy = fmaf(P.wy, Gs, -Sy), cz = fmaf(P.wz, Gs, -Sz);
                lox += fmaf(Gs, lcx, -ox); loy += fmaf(Gs, lcy, -oy); loz += fmaf(Gs, lcz, -oz);
                lkf = fmaf(ez, cz, fmaf(ey, cy, fmaf(ex, cx, lkf)));
                if (w2 > 0.f) {
                    const float lc = fmaf(lFz, cz, fmaf(lFy, cy, lFx * cx));     // lF . c
                    const float hc = fmaf(hz, cz, fmaf(hy, cy, hx * cx));        // w^ . c
                    const float hl = fmaf(hz, lFz, fmaf(hy, lFy, hx * lFx));     // w^ . lF
                    lwx += P.kf * (lc * hx - hl * cx - hc * fmaf(-hx, hl, lFx));
                    lwy += P.kf * (lc * hy - hl * cy - hc * fmaf(-hy, hl, lFy));
                    lwz += P.kf * (lc * hz - hl * cz - hc * fmaf(-hz, hl, lFz));
                }
            };
            if (split) {
                rrun(my_v, my_j0, my_n, my_stride);
            } else {
                const int tile = resident ? (int)max(n_shard, 1ll) : lay.cap;
                for (long long tb = 0; tb < n_shard; tb += tile) {
                    const int tn = (int)min((long long)tile, n_shard - tb);
                    if (!resident) {
                        __syncthreads();
                        for (int i = tid; i < tn; i += NT) {
                            lx[i] = sc.x[tb + i]; ly[i] = sc.y[tb + i]; lz[i] = sc.z[tb + i];
                        }
                        __syncthreads();
                    }
                    for (int r = 0; r < n_runs; ++r) {
                        const int b = max(runs[r].x, (int)tb), e = min(runs[r].y, (int)tb + tn);
                        if (b >= e) continue;
                        const int first = b - (int)tb + slice;
                        const int n = (e - (int)tb > first) ? (e - (int)tb - first + L - 1) / L : 0;
                        rrun(rvel[r], first, n, L);
                    }
                }
            }
            float4 v3[3] = {make_float4(gpx, gpy, gpz, lkf), make_float4(lwx, lwy, lwz, 0.f),
                            make_float4(lox, loy, loz, 0.f)};
            wg_reduce(v3, 3, m2, mx, my, mz);
            // costs at step k: goal distance (Eq. 17), obstacle distance (Eq. 18), path length (Eq. 19)
            float cpx_ = 0, cpy_ = 0, cpz_ = 0, cvx_ = 0, cvy_ = 0, cvz_ = 0;
            {
                const float ex = gx - P4.x, ey = gy - P4.y, ez = gz - P4.z;
                const float dg2 = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
                const float dg = __builtin_amdgcn_sqrtf(dg2);
                if (dg < pr.r_cost && dg > 0.f) {
                    const float c = -cgoal / dg;
                    cpx_ += c * ex; cpy_ += c * ey; cpz_ += c * ez;
                }
                if (m2 < INFINITY) {
                    const float rs = __builtin_amdgcn_sqrtf(m2), x = rs - P.R;
                    if (x > pr.eps && x < pr.r_cost) {
                        const float c = -cobs / rs;
                        cpx_ += c * mx; cpy_ += c * my; cpz_ += c * mz;
                    }
                }
                if (k >= 2) {
                    const float vn2 = fmaf(V4.z, V4.z, fmaf(V4.y, V4.y, V4.x * V4.x));
                    if (vn2 > 0.f) {
                        const float c = cpath * __builtin_amdgcn_rsqf(vn2);
                        cvx_ = c * V4.x; cvy_ = c * V4.y; cvz_ = c * V4.z;
                    }
                }
            }
            gka += lFx * (gx - P4.x) + lFy * (gy - P4.y) + lFz * (gz - P4.z);
            gda -= lFx * V4.x + lFy * V4.y + lFz * V4.z;
            gkf += v3[0].w;
            gox += v3[2].x; goy += v3[2].y; goz += v3[2].z;
            lpx = lpx - P.ka * lFx + v3[0].x + cpx_;
            lpy = lpy - P.ka * lFy + v3[0].y + cpy_;
            lpz = lpz - P.ka * lFz + v3[0].z + cpz_;
            lvx = lvtx - P.da * lFx + v3[1].x + cvx_;
            lvy = lvty - P.da * lFy + v3[1].y + cvy_;
            lvz = lvtz - P.da * lFz + v3[1].z + cvz_;
        }
        const float4 F0 = tape[(size_t)a_w * 3 + 2];
        Fax = F0.x; Fay = F0.y; Faz = F0.z;
        __syncthreads();                           // the tape is rewritten by the next segment
    }
    if (writer && valid) {
        const bool bad = S > 1 && ld_agent(xc.status) != 0u;   // an exchange wait was cut short
        io.g_ka[agent] = bad ? NAN : gka;
        io.g_da[agent] = bad ? NAN : gda;
        io.g_kf[agent] = bad ? NAN : gkf;
        io.g_om[3 * agent] = bad ? NAN : gox;
        io.g_om[3 * agent + 1] = bad ? NAN : goy;
        io.g_om[3 * agent + 2] = bad ? NAN : goz;
    }
    if (S > 1) {                                  // the last workgroup clears the exchange area
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0) {
            const unsigned prev = __hip_atomic_fetch_add(xc.done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            s_last = (prev == (unsigned)(G * S - 1)) ? 1 : 0;
        }
        __syncthreads();
        if (!s_last) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const size_t words = (size_t)2 * G * S * AW * kAdjWords;
        for (size_t i = tid; i < words; i += NT) st64_agent(xc.partial + i, 0ull);
        if (tid == 0) {
            st_agent(xc.status, 0u);
            st_agent(xc.done, 0u);
        }
    }
}

using AFn = void (*)(Scn, Agt, Prm, AdjOut, AdjLay, Xch);

template <int AW, int W>
AFn pick_adj_cut(int cut)
{
    return cut ? k_adjoint<AW, W, 1> : k_adjoint<AW, W, 0>;
}

AFn pick_adjoint(int AW, int W, int cut)
{
    if (W == 4) {
        if (AW == 1) return pick_adj_cut<1, 4>(cut);
        if (AW == 2) return pick_adj_cut<2, 4>(cut);
        if (AW == 4) return pick_adj_cut<4, 4>(cut);
    }
    if (W == 8) {
        if (AW == 1) return pick_adj_cut<1, 8>(cut);
        if (AW == 2) return pick_adj_cut<2, 8>(cut);
        if (AW == 4) return pick_adj_cut<4, 8>(cut);
    }
    return nullptr;
}

}  // namespace

gmapp_status launch_adjoint(gmapp_ctx *ctx, const Scn &sc, const Agt &ag, const Prm &pr, const float *grad_total,
                            int ckpt_every, float *g_ka, float *g_da, float *g_kf, float *g_om, hipStream_t stream)
{
    if (ag.n == 0) return GMAPP_OK;
    const int cus = ctx->n_cu > 0 ? ctx->n_cu : 256;
    constexpr int W = 8;
    constexpr size_t budget = 160 * 1024;
    int AW = 1;
    while (AW < 4 && (ag.n + AW - 1) / AW > 2 * cus) AW *= 2;
    const int G = (ag.n + AW - 1) / AW;
    AFn fn = pick_adjoint(AW, W, pr.cutoff);
    AdjOut io{grad_total, g_ka, g_da, g_kf, g_om};
    // layout for S shards: each shard resident in LDS when it fits, else streamed tiles
    auto layout = [&](int S) {
        AdjLay l;
        l.runs_cap = 2 * sc.n_seg + 2;
        l.C = ckpt_every;
        l.n_ckpt = (pr.n_steps + ckpt_every - 1) / ckpt_every;
        l.resident = 1;
        l.cap = (int)std::max<long long>((sc.n_cap + S - 1) / S, 1);
        if (adj_plan(l, W, AW, S).total > budget) {
            l.resident = 0;
            l.cap = 2048;
        }
        return l;
    };
    // shards: fill the chip when there are fewer groups than CUs, within co-residency
    int S = 1;
    while (S < 8 && (long long)G * S * 2 <= cus && sc.n_cap / (S * 2) >= 256) S *= 2;
    for (; S > 1; S /= 2) {
        const AdjLay l = layout(S);
        const size_t shm = adj_plan(l, W, AW, S).total;
        if (shm > budget) continue;
        GM_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
        int per_cu = 0;
        GM_HIP(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(fn), 64 * W,
                                                                 shm));
        const long long nwg = ((long long)G * S + 7) / 8 * 8;
        const size_t xbytes = (size_t)2 * G * S * AW * kAdjWords * sizeof(unsigned long long);
        if ((long long)per_cu * cus >= nwg && xbytes <= kXchgBytes) break;
    }
    const AdjLay lay = layout(S);
    if (adj_plan(lay, W, AW, S).total > budget)
        return fail(ctx, GMAPP_ECAPACITY, "checkpoints of %d steps x %d segments exceed LDS; raise ckpt_every",
                    ckpt_every, lay.n_ckpt);
    const size_t shm = adj_plan(lay, W, AW, S).total;
    Xch xc = make_xch(ctx, S, G);
    void *args[] = {(void *)&sc, (void *)&ag, (void *)&pr, (void *)&io, (void *)&lay, (void *)&xc};
    GM_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)shm));
    if (S > 1) {
        const long long nwg = ((long long)G * S + 7) / 8 * 8;
        GM_HIP(ctx, hipLaunchCooperativeKernel(reinterpret_cast<const void *>(fn), dim3((unsigned)nwg), dim3(64 * W),
                                               args, (unsigned)shm, stream));
    } else {
        GM_HIP(ctx, hipLaunchKernel(reinterpret_cast<const void *>(fn), dim3((unsigned)G), dim3(64 * W), args, shm,
                                    stream));
    }
    return GMAPP_OK;
}

}  // namespace gm
