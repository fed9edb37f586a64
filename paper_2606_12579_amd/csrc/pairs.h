// Device helpers shared by the forward rollout and the adjoint rollout kernels.
#pragma once

#include "gmapp_internal.h"

#include <type_traits>

namespace gm {
namespace dev {

constexpr float kTiny = 1e-30f;                 // keeps |d|^2 > 0 (agent on a sphere centre)

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

// Points [b, e) of the LDS copy, slice `sl` of L (round-robin).
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

// The same over an interleaved (x, y, z per point) LDS copy: one address per
// point, the three coordinates at immediate offsets.
template <int L, int CUT>
__device__ __forceinline__ void interact_run_aos(const float *__restrict__ lp, int b, int e, int sl, float psx,
                                                 float psy, float psz, float wx, float wy, float wz, float R,
                                                 float eps, float rd, float tb_a, float tb_b, float &G, float &Sx,
                                                 float &Sy, float &Sz, float &m2)
{
    const int n = e - b;
    const int full = n / L;
    const float *q = lp + 3 * (b + sl);
#pragma unroll 4
    for (int i = 0; i < full; ++i, q += 3 * L)
        interact<CUT>(q[0], q[1], q[2], psx, psy, psz, wx, wy, wz, R, eps, rd, tb_a, tb_b, G, Sx, Sy, Sz, m2);
    if (sl < n - full * L)
        interact<CUT>(q[0], q[1], q[2], psx, psy, psz, wx, wy, wz, R, eps, rd, tb_a, tb_b, G, Sx, Sy, Sz, m2);
}

__device__ __forceinline__ unsigned ld_agent(const unsigned *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned *p, unsigned v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st64_agent(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld64_agent(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_system(const unsigned *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The wait settings, read from device memory when a wait needs them (they sit after the
// status word), so that they hold no registers across the step loop.
__device__ __forceinline__ unsigned long long wait_limit(const Xch &xc)
{
    return *reinterpret_cast<const unsigned long long *>(xc.status + kWaitLimitWord);
}
__device__ __forceinline__ const unsigned *abort_addr(const Xch &xc)
{
    return *reinterpret_cast<const unsigned *const *>(xc.status + kAbortAddrWord);
}

// The slow path of an exchange wait, taken every 64th poll that finds the words
// incomplete (every poll when xc.fine, i.e. limits below 1 ms): true when the wait
// must end -- another wave already ended one (status != 0), the host raised the abort
// word (status 2), or the wait has made no progress for longer than the limit (status
// 1).  The clock restarts with every wait: in the usual mode the wait's clock starts at
// its first slow check (t_wait = 0 until then), with xc.fine at the wait's start.  So
// only a stall, never the length of a launch, trips it; a wait that completes within
// 64 polls reads neither clock nor settings.
__device__ __forceinline__ bool slow_check(const Xch &xc, unsigned long long &t_wait, unsigned spins)
{
    if (ld_agent(xc.status) != 0u) return true;
    const unsigned *a = abort_addr(xc);
    if (a && ld_system(a) != 0u) {
        st_agent(xc.status, 2u);
        return true;
    }
    const unsigned long long now = __builtin_amdgcn_s_memrealtime();
    if (!xc.fine && spins == 64) {
        t_wait = now;
    } else if (now - t_wait > wait_limit(xc)) {
        st_agent(xc.status, 1u);
        return true;
    }
    return false;
}

// exchange word: float bits | step tag << 32
__device__ __forceinline__ unsigned long long xword(float v, unsigned tag)
{
    return (unsigned long long)__float_as_uint(v) | ((unsigned long long)tag << 32);
}
__device__ __forceinline__ float xval(unsigned long long q) { return __uint_as_float((unsigned)q); }
__device__ __forceinline__ unsigned xtag(unsigned long long q) { return (unsigned)(q >> 32); }

// Sum / min over the lanes of one agent (lanes congruent mod AW) of a wavefront,
// leaving the identical result in every such lane: rotations by 8, 4, 2, 1 inside
// 16-lane rows (DPP), then the xor-16 swizzle and the 32-lane swap.  Each stage
// adds a partner whose own partner holds an equal value, so commutativity makes
// every lane's result bit-identical.
template <int AW, bool MIN>
__device__ __forceinline__ float agent_allreduce(float x)
{
    auto op = [](float a, float b) { return MIN ? fminf(a, b) : a + b; };
    auto dpp = [](float v, auto ctrl) {
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), decltype(ctrl)::value, 0xF, 0xF, false));
    };
    if constexpr (AW <= 8) x = op(x, dpp(x, std::integral_constant<int, 0x128>{}));   // row_ror:8
    if constexpr (AW <= 4) x = op(x, dpp(x, std::integral_constant<int, 0x124>{}));   // row_ror:4
    if constexpr (AW <= 2) x = op(x, dpp(x, std::integral_constant<int, 0x122>{}));   // row_ror:2
    if constexpr (AW <= 1) x = op(x, dpp(x, std::integral_constant<int, 0x121>{}));   // row_ror:1
    if constexpr (AW <= 16) x = op(x, __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), 0x401F)));
    if constexpr (AW <= 32) {
        auto sw = __builtin_amdgcn_permlane32_swap(__float_as_int(x), __float_as_int(x), false, false);
        x = op(__int_as_float(sw[0]), __int_as_float(sw[1]));
    }
    return x;
}

// k_f |w| P_w (omega G - S) added to F (w = relative velocity, uniform over the segment)
__device__ __forceinline__ void project_add(float ux, float uy, float uz, float kf, float wx, float wy, float wz,
                                            float G, float Sx, float Sy, float Sz, float &Fx, float &Fy, float &Fz)
{
    const float w2 = fmaf(uz, uz, fmaf(uy, uy, ux * ux));
    if (w2 > 0.0f) {
        const float cx = fmaf(wx, G, -Sx), cy = fmaf(wy, G, -Sy), cz = fmaf(wz, G, -Sz);
        const float ri = __builtin_amdgcn_rsqf(w2);
        const float wc = fmaf(uz, cz, fmaf(uy, cy, ux * cx)) * (ri * ri);
        const float f = kf * (w2 * ri);
        Fx = fmaf(f, fmaf(-ux, wc, cx), Fx);
        Fy = fmaf(f, fmaf(-uy, wc, cy), Fy);
        Fz = fmaf(f, fmaf(-uz, wc, cz), Fz);
    }
}

struct Agent {
    float ka, da, kf, rd, R, wx, wy, wz, tb_a, tb_b;
    int hz = 0;               // heuristic: 0 rotation-vector field, 1 velocity current, 2 APF
    float ird = 0.f;          // 1 / r_d (APF)
    float kr = 0.f, dr = 0.f, ir = 0.f;   // 6-D pose agents: rotational stiffness, damping, inverse inertia
};

// One agent-sphere interaction of the artificial potential field (Eq. 1 with the
// surface distance rho): accumulates (1/rho - 1/r_d) / (rho^2 |d|) d, to be scaled by k_f.
template <int CUT>
__device__ __forceinline__ void interact_apf(float qx, float qy, float qz, float psx, float psy, float psz, float R,
                                             float eps, float rd, float ird, float tb_a, float tb_b, float &Ax,
                                             float &Ay, float &Az, float &m2)
{
    const float dx = psx - qx, dy = psy - qy, dz = psz - qz;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, kTiny)));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float rho = fmaxf(fmaf(r2, ri, -R), eps);
    const float irho = __builtin_amdgcn_rcpf(rho);
    float c = (irho - ird) * (irho * irho) * ri;
    if constexpr (CUT == 0) {
        c = (rho <= rd) ? c : 0.0f;
    } else {
        const float s = __builtin_amdgcn_fmed3f(fmaf(-rho, tb_a, tb_b), 0.0f, 1.0f);
        c *= (s * s) * fmaf(-2.0f, s, 3.0f);
    }
    Ax = fmaf(c, dx, Ax);
    Ay = fmaf(c, dy, Ay);
    Az = fmaf(c, dz, Az);
    m2 = fminf(m2, r2);
}

// The APF over points [b, e) of the interleaved LDS copy, slice `sl` of L.
template <int L, int CUT>
__device__ __forceinline__ void interact_run_apf_aos(const float *__restrict__ lp, int b, int e, int sl, float psx,
                                                     float psy, float psz, float R, float eps, float rd, float ird,
                                                     float tb_a, float tb_b, float &Ax, float &Ay, float &Az,
                                                     float &m2)
{
    const int n = e - b;
    const int full = n / L;
    const float *q = lp + 3 * (b + sl);
#pragma unroll 4
    for (int i = 0; i < full; ++i, q += 3 * L)
        interact_apf<CUT>(q[0], q[1], q[2], psx, psy, psz, R, eps, rd, ird, tb_a, tb_b, Ax, Ay, Az, m2);
    if (sl < n - full * L)
        interact_apf<CUT>(q[0], q[1], q[2], psx, psy, psz, R, eps, rd, ird, tb_a, tb_b, Ax, Ay, Az, m2);
}


// Segment runs of the shard [sb, se): [begin, end) relative to sb, the run's
// velocity (0 for static points), and -- when there are at most L runs -- the
// split of an agent's L slices over the runs in proportion to their length (at
// least one slice each: .z first slice, .w slice count), so that every lane
// walks one run only.  A table that is not non-decreasing still yields runs
// covering the shard exactly once.  Run by one thread.
__device__ inline int build_runs(const Scn &sc, long long n_pts, long long sb, long long se, int4 *runs,
                                 float4 *rvel, int runs_cap, int L, int &split)
{
    const long long n_shard = se - sb;
    int nr = 0;
    if (sc.n_seg == 0) {
        if (n_shard > 0) {
            runs[0] = make_int4(0, (int)n_shard, 0, 0);
            rvel[0] = make_float4(0.f, 0.f, 0.f, 0.f);
            nr = 1;
        }
    } else {
        auto clampi = [&](long long v) { return min(max(v, 0ll), n_pts); };
        int lo = 0, hi = sc.n_seg;                 // first segment whose end > sb
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (clampi(sc.seg_begin[mid + 1]) > sb) hi = mid; else lo = mid + 1;
        }
        int si = lo;
        long long c = sb;
        while (c < se && nr < runs_cap - 1) {
            long long re;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (si < sc.n_seg) {
                long long b_s = clampi(sc.seg_begin[si]), e_s = clampi(sc.seg_begin[si + 1]);
                if (b_s <= c) {
                    re = min(e_s, se);
                    v = make_float4(sc.seg_vel[3 * si], sc.seg_vel[3 * si + 1], sc.seg_vel[3 * si + 2], 0.f);
                } else {
                    re = min(b_s, se);
                }
            } else {
                re = se;
            }
            if (re <= c) re = se;
            runs[nr] = make_int4((int)(c - sb), (int)(re - sb), 0, 0);
            rvel[nr] = v;
            ++nr;
            c = re;
            while (si < sc.n_seg && clampi(sc.seg_begin[si + 1]) <= c) ++si;
        }
        if (c < se) {                               // out of slots (malformed table): rest static
            runs[nr] = make_int4((int)(c - sb), (int)n_shard, 0, 0);
            rvel[nr] = make_float4(0.f, 0.f, 0.f, 0.f);
            ++nr;
        }
    }
    split = (nr > 0 && nr <= L) ? 1 : 0;
    if (split) {
        int used = 0;
        for (int r = 0; r < nr; ++r) {
            const long long len = runs[r].y - runs[r].x;
            runs[r].w = max(1, (int)(len * L / max(n_shard, 1ll)));
            used += runs[r].w;
        }
        while (used > L) {                          // give back slices where they cost least
            int best = -1;
            for (int r = 0; r < nr; ++r)
                if (runs[r].w > 1 && (best < 0 || (long long)(runs[r].y - runs[r].x) * runs[best].w <
                                                   (long long)(runs[best].y - runs[best].x) * runs[r].w))
                    best = r;
            --runs[best].w;
            --used;
        }
        while (used < L) {                          // add slices where the points per slice are highest
            int best = 0;
            for (int r = 1; r < nr; ++r)
                if ((long long)(runs[r].y - runs[r].x) * runs[best].w >
                    (long long)(runs[best].y - runs[best].x) * runs[r].w)
                    best = r;
            ++runs[best].w;
            ++used;
        }
        int first = 0;
        for (int r = 0; r < nr; ++r) {
            runs[r].z = first;
            first += runs[r].w;
        }
    }
    return nr;
}

// This lane's run under the split: first point, point count and stride.
__device__ inline void lane_run(const int4 *runs, const float4 *rvel, int n_runs, int slice, int &j0, int &n,
                                int &stride, float4 &v)
{
    int r = 0;
    while (r + 1 < n_runs && runs[r + 1].z <= slice) ++r;
    const int4 rr = runs[r];
    j0 = rr.x + (slice - rr.z);
    stride = rr.w;
    n = (rr.y > j0) ? (rr.y - j0 + rr.w - 1) / rr.w : 0;
    v = rvel[r];
}

}  // namespace dev
}  // namespace gm
