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
// frame (J_b = diag(R^T, R^T) J).  Joint angles are held as half-angle rotors
// (cos(q/2), sin(q/2)) in FP64 and advanced by a rotation through dt qdot / 2
// (see advance), so that the
// forward kinematics of consecutive steps differ by their true increment: the
// jerk cost of Eq. (20) takes third differences of these positions.
#pragma once

#include "gmapp_internal.h"
#include "pose.h"

namespace gm {
namespace arm {

constexpr int kMaxJoints = 7;
static_assert(kMaxJoints == kMaxArmJoints, "the chain length the host admits");

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

// end-effector pose (rotor, position) in FP64 for joint half-angle rotors (c[i], s[i])
__device__ __forceinline__ void fk_d(const float *L, int n, const double *c, const double *s, QD &r, double &tx,
                                     double &ty, double &tz)
{
    r = QD{L[0], L[1], L[2], L[3]};
    tx = L[4]; ty = L[5]; tz = L[6];
    for (int i = 0; i < kMaxJoints; ++i) {
        if (i >= n) break;
        r = qmul_d(r, QD{c[i], 0.0, 0.0, s[i]});
        const float *l = L + 7 * (i + 1);
        double ox, oy, oz;
        qrot_d(r, l[4], l[5], l[6], ox, oy, oz);
        tx += ox; ty += oy; tz += oz;
        r = qmul_d(r, QD{l[0], l[1], l[2], l[3]});
    }
    const double nr = 1.0 / sqrt(r.w * r.w + r.x * r.x + r.y * r.y + r.z * r.z);
    r = QD{r.w * nr, r.x * nr, r.y * nr, r.z * nr};
}

// visit every joint's axis z_i and origin o_i (FP32) at the half-angle rotors (c, s)
template <class F>
__device__ __forceinline__ void joints_f(const float *L, int n, const double *c, const double *s, F &&visit)
{
    pose::Q r{L[0], L[1], L[2], L[3]};
    float tx = L[4], ty = L[5], tz = L[6];
    for (int i = 0; i < kMaxJoints; ++i) {
        if (i >= n) break;
        float zx, zy, zz;
        pose::qrot(r, 1.0f, 0.0f, 0.0f, 1.0f, zx, zy, zz);
        visit(i, zx, zy, zz, tx, ty, tz);
        r = pose::qmul(r, pose::Q{(float)c[i], 0.0f, 0.0f, (float)s[i]});
        const float *l = L + 7 * (i + 1);
        float ox, oy, oz;
        pose::qrot(r, 1.0f, l[4], l[5], l[6], ox, oy, oz);
        tx += ox; ty += oy; tz += oz;
        r = pose::qmul(r, pose::Q{l[0], l[1], l[2], l[3]});
    }
}

// joint rates for the world twist (wa, wl) at end-effector position p:
// qdot = J^T y, (J J^T + lambda^2 I) y = (wa, wl): the FP32 columns are accumulated
// and the system is solved by Cholesky in FP64 (J J^T squares J's condition number)
__device__ __forceinline__ void joint_rates(const float *L, int n, const double *c, const double *s, float px,
                                            float py, float pz, const float wa[3], const float wl[3], float lam2,
                                            float *qd)
{
    double A[21];                                  // lower triangle of the 6x6 matrix, row-major
#pragma unroll
    for (int k = 0; k < 21; ++k) A[k] = 0.0;
    joints_f(L, n, c, s, [&](int, float zx, float zy, float zz, float ox, float oy, float oz) {
        const float rx = px - ox, ry = py - oy, rz = pz - oz;
        const double col[6] = {zx, zy, zz, zy * rz - zz * ry, zz * rx - zx * rz, zx * ry - zy * rx};
#pragma unroll
        for (int a = 0; a < 6; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b) A[a * (a + 1) / 2 + b] += col[a] * col[b];
    });
    A[0] += lam2; A[2] += lam2; A[5] += lam2; A[9] += lam2; A[14] += lam2; A[20] += lam2;
    // Cholesky in place: A = G G^T, G lower
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        const int ra = a * (a + 1) / 2;
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int rb = b * (b + 1) / 2;
            double sum = A[ra + b];
#pragma unroll
            for (int k = 0; k < b; ++k) sum -= A[ra + k] * A[rb + k];
            A[ra + b] = (a == b) ? sqrt(fmax(sum, 1e-300)) : sum / A[rb + b];
        }
    }
    double y[6] = {wa[0], wa[1], wa[2], wl[0], wl[1], wl[2]};
#pragma unroll
    for (int a = 0; a < 6; ++a) {                  // G z = b
        const int ra = a * (a + 1) / 2;
#pragma unroll
        for (int k = 0; k < a; ++k) y[a] -= A[ra + k] * y[k];
        y[a] /= A[ra + a];
    }
#pragma unroll
    for (int a = 5; a >= 0; --a) {                 // G^T y = z
#pragma unroll
        for (int k = a + 1; k < 6; ++k) y[a] -= A[k * (k + 1) / 2 + a] * y[k];
        y[a] /= A[a * (a + 1) / 2 + a];
    }
    joints_f(L, n, c, s, [&](int i, float zx, float zy, float zz, float ox, float oy, float oz) {
        const float rx = px - ox, ry = py - oy, rz = pz - oz;
        qd[i] = (float)(zx * y[0] + zy * y[1] + zz * y[2] + (zy * rz - zz * ry) * y[3] + (zz * rx - zx * rz) * y[4] +
                        (zx * ry - zy * rx) * y[5]);
    });
}

// advance a half-angle rotor (c, s) by the half angle h: rotation by (cos h, sin h), by
// series for |h| <= 0.05 (truncation under 1e-17), else by sincos
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
    const double nr = 1.0 / sqrt(c1 * c1 + s1 * s1);
    c = c1 * nr;
    s = s1 * nr;
}

}  // namespace arm
}  // namespace gm
