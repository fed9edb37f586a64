// Serial-chain arm agents (Eqs. 12-14): forward kinematics of revolute joints
// about their local z axes, and the damped pseudo-inverse step of the joints.
//
// A chain of n joints is n + 1 fixed link transforms L_0 .. L_n (rotor and
// offset, 7 floats each): the end-effector pose is
//   M(q) = L_0 Rz(q_1) L_1 Rz(q_2) ... Rz(q_n) L_n.
// Joint i's axis z_i and origin o_i (world) are those of the frame
// L_0 Rz(q_1) ... L_{i-1}.  Its column of the world ("hybrid") Jacobian is
// (z_i, z_i x (p - o_i)) for the end-effector position p, and for the body twist
// v_b = (omega_b, u_b) the damped least-squares joint rates are
//   qdot = J^T (J J^T + lambda^2 I)^-1 (R omega_b, R u_b),
// the body-frame form J_b^T (J_b J_b^T + lambda^2 I)^-1 v_b written in the world
// frame (J_b = diag(R^T, R^T) J).
//
// Work is spread over the lanes of an agent.  In a wave, agent a's lanes are
// a + AW j (j = 0 .. 64 / AW - 1), and lane j owns joint j: its half-angle rotor
// (cos(q_j / 2), sin(q_j / 2)) in FP64 and its angle q_j, summed as q_j += dt qdot_j.
// Per step:
//   factor -- every lane walks the joint frames at the current angles (FP32),
//     accumulates A = J J^T + lambda^2 I (FP64; J J^T squares J's condition
//     number) and keeps its own column of J; A is factored as G G^T.  None of this
//     depends on the repulsive force, so it runs while the force is exchanged;
//   solve -- y = A^-1 (R omega_b, R u_b); the owner lane forms qdot_j = col_j . y
//     and advances its rotor through dt qdot_j / 2 (see advance), so the forward
//     kinematics of consecutive steps differ by their true increment (the jerk cost
//     of Eq. (20) takes third differences of these positions);
//   fk_tree -- each owner lane forms its joint's transform Rz(q_j) L_{j+1}, and the
//     FP64 forward kinematics is their product, taken as a tree over the lanes.
#pragma once

#include "gmapp_internal.h"
#include "pose.h"

namespace gm {
namespace arm {

constexpr int kMaxJoints = 7;
static_assert(kMaxJoints == kMaxArmJoints, "the chain length the host admits");
static_assert(kMaxArmAgentsPerGroup * kMaxJoints <= 64, "each agent holds one lane per joint in a wave");

struct QD {
    double w, x, y, z;
};

__device__ __forceinline__ QD qmul_d(const QD &a, const QD &b)
{
    return QD{a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z, a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
              a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x, a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}

// r (x) (c, 0, 0, s): a rotation about r's local z axis
__device__ __forceinline__ pose::Q qmul_z(const pose::Q &r, float c, float s)
{
    return pose::Q{r.w * c - r.z * s, r.x * c + r.y * s, r.y * c - r.x * s, r.z * c + r.w * s};
}

__device__ __forceinline__ void qrot_d(const QD &q, double vx, double vy, double vz, double &ox, double &oy,
                                       double &oz)
{
    const double cx = q.y * vz - q.z * vy, cy = q.z * vx - q.x * vz, cz = q.x * vy - q.y * vx;
    const double dx = q.y * cz - q.z * cy, dy = q.z * cx - q.x * cz, dz = q.x * cy - q.y * cx;
    ox = vx + 2.0 * (q.w * cx + dx);
    oy = vy + 2.0 * (q.w * cy + dy);
    oz = vz + 2.0 * (q.w * cz + dz);
}

// 1 / sqrt(x) for x in the FP32 normal range: the FP32 hardware estimate refined by
// two Newton steps y <- y (1 + (1 - x y^2) / 2), each of which squares the relative error
__device__ __forceinline__ double rsqrt_d(double x)
{
    double y = (double)__builtin_amdgcn_rsqf((float)x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// a double from lane src (every lane of the wave must be active)
__device__ __forceinline__ double lane_d(double v, int src)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(unsigned)b);
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// every lane of agent a_w receives the rotors (c[i], s[i]) held by the joints' owner lanes a_w + AW i
template <int AW>
__device__ __forceinline__ void gather(double c_own, double s_own, int a_w, double *c, double *s)
{
    static_assert(AW * kMaxJoints <= 64, "joint owners within the wave");
#pragma unroll
    for (int i = 0; i < kMaxJoints; ++i) {
        c[i] = lane_d(c_own, a_w + AW * i);
        s[i] = lane_d(s_own, a_w + AW * i);
    }
}

// A rigid transform (rotor r, translation t) in FP64: x -> R(r) x + t
struct TD {
    QD r;
    double x, y, z;
};

// a o b: first b, then a
__device__ __forceinline__ TD compose(const TD &a, const TD &b)
{
    double ox, oy, oz;
    qrot_d(a.r, b.x, b.y, b.z, ox, oy, oz);
    return TD{qmul_d(a.r, b.r), a.x + ox, a.y + oy, a.z + oz};
}

__device__ __forceinline__ TD lane_td(const TD &v, int src)
{
    return TD{QD{lane_d(v.r.w, src), lane_d(v.r.x, src), lane_d(v.r.y, src), lane_d(v.r.z, src)}, lane_d(v.x, src),
              lane_d(v.y, src), lane_d(v.z, src)};
}

// End-effector pose M(q) = L_0 T_0 T_1 ... T_7 with T_j = Rz(q_j) L_{j+1} for the joints
// j < n (identity beyond): each owner lane a_w + AW j forms its T_j from its half-angle
// rotor (c, s) -- Rz(q) turns offsets by (cos q, sin q) = (c^2 - s^2, 2 c s) -- and
// three rounds of pairwise products over the agent's first 8 lanes leave the product on
// lane a_w, which every lane of the agent then reads.  Every lane of the wave must be
// active.
template <int AW>
__device__ __forceinline__ void fk_tree(const float *L, int n, int a_w, int j, double c, double s, QD &r, double &tx,
                                        double &ty, double &tz)
{
    static_assert(AW * 8 <= 64, "8 lanes per agent in the wave");
    TD T{QD{1.0, 0.0, 0.0, 0.0}, 0.0, 0.0, 0.0};
    if (j < n && j < kMaxJoints) {
        const float *l = L + 7 * (j + 1);
        const double lw = l[0], lx = l[1], ly = l[2], lz = l[3];
        const double cq = c * c - s * s, sq = 2.0 * c * s;
        T = TD{QD{c * lw - s * lz, c * lx - s * ly, c * ly + s * lx, c * lz + s * lw}, cq * l[4] - sq * l[5],
               sq * l[4] + cq * l[5], (double)l[6]};
    }
    const int lane = a_w + AW * j;
#pragma unroll
    for (int stride = 1; stride < 8; stride *= 2) {
        const TD o = lane_td(T, (lane + AW * stride) & 63);   // lanes past the agent's 8 give unused results
        T = compose(T, o);
    }
    const TD P = lane_td(T, a_w);
    const TD M = compose(TD{QD{L[0], L[1], L[2], L[3]}, L[4], L[5], L[6]}, P);
    const double nr = rsqrt_d(M.r.w * M.r.w + M.r.x * M.r.x + M.r.y * M.r.y + M.r.z * M.r.z);
    r = QD{M.r.w * nr, M.r.x * nr, M.r.y * nr, M.r.z * nr};
    tx = M.x; ty = M.y; tz = M.z;
}

// The joint frames at the rotors (c, s) (FP32) give J; A = J J^T + lam2 I (FP64, lower
// triangle row-major, 21 entries) is factored in place as G G^T, G lower triangular,
// with G's diagonal stored as its reciprocals.  col receives column `mine` of J (zeros
// when mine >= n).  p: end-effector position.
__device__ __forceinline__ void factor(const float *L, int n, const double *c, const double *s, float px, float py,
                                       float pz, float lam2, int mine, double *A, float *col)
{
#pragma unroll
    for (int k = 0; k < 21; ++k) A[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) col[k] = 0.0f;
    pose::Q r{L[0], L[1], L[2], L[3]};
    float tx = L[4], ty = L[5], tz = L[6];
#pragma unroll
    for (int i = 0; i < kMaxJoints; ++i) {
        if (i >= n) break;
        // z axis of the frame r: the third column of its rotation matrix
        const float zx = 2.0f * (r.x * r.z + r.w * r.y), zy = 2.0f * (r.y * r.z - r.w * r.x);
        const float zz = 1.0f - 2.0f * (r.x * r.x + r.y * r.y);
        const float rx = px - tx, ry = py - ty, rz = pz - tz;
        const float cl[6] = {zx, zy, zz, zy * rz - zz * ry, zz * rx - zx * rz, zx * ry - zy * rx};
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            col[a] = (i == mine) ? cl[a] : col[a];
#pragma unroll
            for (int b = 0; b <= a; ++b) A[a * (a + 1) / 2 + b] = fma((double)cl[a], (double)cl[b], A[a * (a + 1) / 2 + b]);
        }
        r = qmul_z(r, (float)c[i], (float)s[i]);
        const float *l = L + 7 * (i + 1);
        float ox, oy, oz;
        pose::qrot(r, 1.0f, l[4], l[5], l[6], ox, oy, oz);
        tx += ox; ty += oy; tz += oz;
        r = pose::qmul(r, pose::Q{l[0], l[1], l[2], l[3]});
    }
    A[0] += lam2; A[2] += lam2; A[5] += lam2; A[9] += lam2; A[14] += lam2; A[20] += lam2;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        const int ra = a * (a + 1) / 2;
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int rb = b * (b + 1) / 2;
            double sum = A[ra + b];
#pragma unroll
            for (int k = 0; k < b; ++k) sum = fma(-A[ra + k], A[rb + k], sum);
            // the clamp keeps a singular undamped system finite (its rates are then huge)
            A[ra + b] = (a == b) ? rsqrt_d(fmax(sum, 1e-30)) : sum * A[rb + b];
        }
    }
}

// y <- (G G^T)^-1 y for the factor of factor()
__device__ __forceinline__ void solve(const double *A, double *y)
{
#pragma unroll
    for (int a = 0; a < 6; ++a) {                  // G z = y
        const int ra = a * (a + 1) / 2;
#pragma unroll
        for (int k = 0; k < a; ++k) y[a] = fma(-A[ra + k], y[k], y[a]);
        y[a] *= A[ra + a];
    }
#pragma unroll
    for (int a = 5; a >= 0; --a) {                 // G^T y = z
#pragma unroll
        for (int k = a + 1; k < 6; ++k) y[a] = fma(-A[k * (k + 1) / 2 + a], y[k], y[a]);
        y[a] *= A[a * (a + 1) / 2 + a];
    }
}

// advance a half-angle rotor (c, s) by the half angle h: rotation by (cos h, sin h), by
// series for |h| <= 0.05 (truncation under 1e-17), else by sincos.  Both factors are
// unit to rounding, so one Newton step from 1 renormalises the product.
__device__ __forceinline__ void advance(double &c, double &s, double h)
{
    const double h2 = h * h;
    double ch, sh;
    if (fabs(h) <= 0.05) {
        ch = 1.0 - h2 * (0.5 - h2 * (1.0 / 24.0 - h2 * (1.0 / 720.0 - h2 * (1.0 / 40320.0))));
        sh = h * (1.0 - h2 * (1.0 / 6.0 - h2 * (1.0 / 120.0 - h2 * (1.0 / 5040.0 - h2 * (1.0 / 362880.0)))));
    } else {
        sincos(h, &sh, &ch);
    }
    const double c1 = c * ch - s * sh, s1 = s * ch + c * sh;
    const double nr = fma(-0.5, fma(c1, c1, s1 * s1), 1.5);
    c = c1 * nr;
    s = s1 * nr;
}

}  // namespace arm
}  // namespace gm
