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
// (cos(q_j / 2), sin(q_j / 2)) in FP64, its angle q_j, summed as q_j += dt qdot_j, and its
// column of J.  Per step:
//   factor_cols -- A = J J^T + lambda^2 I (FP64; J J^T squares J's condition number) is
//     the sum of the joint lanes' outer products, taken by a butterfly over the lanes, and
//     is factored as G G^T.  None of this depends on the repulsive force, so it runs while
//     the force is exchanged;
//   solve -- y = A^-1 (R omega_b, R u_b); the owner lane forms qdot_j = col_j . y and
//     advances its rotor through dt qdot_j / 2 (see advance), so the forward kinematics of
//     consecutive steps differ by their true increment (the jerk cost of Eq. (20) takes
//     third differences of these positions);
//   fk_scan -- each owner lane forms its joint's transform Rz(q_j) L_{j+1}; an inclusive
//     scan of these over the lanes gives the FP64 end-effector pose and every joint's frame,
//     from which each lane takes its column of J for the next step.
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

// Forward kinematics by an inclusive scan of the joint transforms over the agent's first
// 8 lanes (three rounds; lane j ends with T_0 ... T_j), which also gives every joint its
// frame F_j = L_0 T_0 ... T_{j-1} (from lane j - 1).  Returns the end-effector pose
// L_0 T_0 ... T_7 and, in col, this lane's column of the world Jacobian (z_j,
// z_j x (p - o_j)) for joint j = mine (zeros when mine >= n).  Every lane of the wave must
// be active.
template <int AW>
__device__ __forceinline__ void fk_scan(const float *L, int n, int a_w, int j, double c, double s, QD &r, double &tx,
                                        double &ty, double &tz, float *col)
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
        const TD o = lane_td(T, (lane - AW * stride) & 63);   // the earlier lanes' product
        const TD u = compose(o, T);
        if (j >= stride) T = u;
    }
    const TD L0{QD{L[0], L[1], L[2], L[3]}, L[4], L[5], L[6]};
    const TD E = compose(L0, lane_td(T, a_w + AW * 7));          // L_0 T_0 ... T_7
    const TD prev = lane_td(T, (lane - AW) & 63);
    const TD F = j == 0 ? L0 : compose(L0, prev);               // joint j's frame
    const double nr = rsqrt_d(E.r.w * E.r.w + E.r.x * E.r.x + E.r.y * E.r.y + E.r.z * E.r.z);
    r = QD{E.r.w * nr, E.r.x * nr, E.r.y * nr, E.r.z * nr};
    tx = E.x; ty = E.y; tz = E.z;
    // z axis of F: the third column of its rotation matrix
    const double zx = 2.0 * (F.r.x * F.r.z + F.r.w * F.r.y), zy = 2.0 * (F.r.y * F.r.z - F.r.w * F.r.x);
    const double zz = 1.0 - 2.0 * (F.r.x * F.r.x + F.r.y * F.r.y);
    const double rx = tx - F.x, ry = ty - F.y, rz = tz - F.z;
    const bool own = j < n && j < kMaxJoints;
    col[0] = own ? (float)zx : 0.0f;
    col[1] = own ? (float)zy : 0.0f;
    col[2] = own ? (float)zz : 0.0f;
    col[3] = own ? (float)(zy * rz - zz * ry) : 0.0f;
    col[4] = own ? (float)(zz * rx - zx * rz) : 0.0f;
    col[5] = own ? (float)(zx * ry - zy * rx) : 0.0f;
}

// A = J J^T + lam2 I from the columns held by the agent's first 8 lanes (each lane's outer
// product, summed by a butterfly over the lanes a_w + AW j), factored in place as G G^T
// (lower triangle row-major, G's diagonal stored as its reciprocals).  Every lane of the
// wave must be active; every lane of the agent ends with the same factor.
template <int AW>
__device__ __forceinline__ void factor_cols(const float *col, float lam2, double *A)
{
    static_assert(AW * 8 <= 64, "8 lanes per agent in the wave");
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) A[a * (a + 1) / 2 + b] = (double)col[a] * (double)col[b];
    const int lane = __lane_id();
#pragma unroll
    for (int m = 1; m < 8; m *= 2) {
        const int src = lane ^ (AW * m);
#pragma unroll
        for (int k = 0; k < 21; ++k) A[k] += lane_d(A[k], src);
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
            A[ra + b] = (a == b) ? rsqrt_d(fmax(sum, 1e-30)) : sum * A[rb + b];
        }
    }
}

// y <- (G G^T)^-1 y for the factor of factor_cols()
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
