// Rigid-body pose arithmetic for 6-D agents in Spin(3) x| R^3 (FP32, device).
//
// A pose is a unit rotor q = (w, x, y, z) (the double cover of SO(3)) and a
// translation t; a twist is (omega, u) in the body frame.  The exponential and
// logarithm are those of the Lie group (screw motion):
//   exp(phi, rho) = (exp(phi), J(phi) rho),   log(R, t) = (log R, J(phi)^-1 t),
// with the left Jacobian of SO(3), theta = |phi|, [phi] the cross-product matrix:
//   J(phi)    = I + a(theta) [phi] + b(theta) [phi]^2,
//               a = (1 - cos theta) / theta^2 = 2 sin^2(theta/2) / theta^2,  b = (theta - sin theta) / theta^3
//   J(phi)^-1 = I - [phi] / 2 + c(theta) [phi]^2,   c = 1/theta^2 - cot(theta/2) / (2 theta).
// Below theta = 0.25 every coefficient comes from its Taylor series (truncation
// under 2e-8 relative), so the per-step rotation dt |omega| ~ 1e-3 rad keeps full
// FP32 accuracy.  Above it, a uses the cancellation-free 2 sin^2(theta/2) form;
// the cancellation left in b and c weighs at most about one FP32 rounding of J v,
// because they multiply the theta^2-sized [phi]^2 term.  Square roots, reciprocals
// and reciprocal square roots on the per-step path use the hardware instructions
// (about 1 ulp) instead of the correctly rounded library sequences.
#pragma once

#include <hip/hip_runtime.h>

namespace gm {
namespace pose {

struct Q {
    float w, x, y, z;
};

__device__ __forceinline__ Q qmul(const Q &a, const Q &b)
{
    return Q{a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z, a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
             a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x, a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}

__device__ __forceinline__ Q qnormalize(const Q &a)
{
    const float s = __builtin_amdgcn_rsqf(a.w * a.w + a.x * a.x + a.y * a.y + a.z * a.z);
    return Q{a.w * s, a.x * s, a.y * s, a.z * s};
}

// R(q) v = v + 2 w (r x v) + 2 r x (r x v), r = (x, y, z); sgn = -1 rotates by the inverse
__device__ __forceinline__ void qrot(const Q &q, float sgn, float vx, float vy, float vz, float &ox, float &oy,
                                     float &oz)
{
    const float rx = sgn * q.x, ry = sgn * q.y, rz = sgn * q.z;
    const float cx = ry * vz - rz * vy, cy = rz * vx - rx * vz, cz = rx * vy - ry * vx;      // r x v
    const float dx = ry * cz - rz * cy, dy = rz * cx - rx * cz, dz = rx * cy - ry * cx;      // r x (r x v)
    ox = vx + 2.0f * (q.w * cx + dx);
    oy = vy + 2.0f * (q.w * cy + dy);
    oz = vz + 2.0f * (q.w * cz + dz);
}

// exp of a rotation vector: (cos(theta/2), sin(theta/2) / theta * phi)
__device__ __forceinline__ Q so3_exp(float px, float py, float pz)
{
    const float t2 = px * px + py * py + pz * pz;
    const float th = __builtin_amdgcn_sqrtf(t2);
    float s, c;
    if (th < 0.25f) {                               // sin(th/2)/th and cos(th/2) by series
        s = 0.5f - t2 * (1.0f / 48.0f) + t2 * t2 * (1.0f / 3840.0f);
        c = 1.0f - t2 * 0.125f + t2 * t2 * (1.0f / 384.0f);
    } else {
        float sh, ch;
        sincosf(0.5f * th, &sh, &ch);
        s = sh / th;
        c = ch;
    }
    return Q{c, s * px, s * py, s * pz};
}

// log of a unit rotor, the rotation vector of angle <= pi (the rotor is taken with w >= 0)
__device__ __forceinline__ void so3_log(Q q, float &px, float &py, float &pz)
{
    if (q.w < 0.0f) { q.w = -q.w; q.x = -q.x; q.y = -q.y; q.z = -q.z; }
    const float n = __builtin_amdgcn_sqrtf(q.x * q.x + q.y * q.y + q.z * q.z);
    const float f = 2.0f * __builtin_amdgcn_rcpf(n > 1e-7f ? n : q.w) * (n > 1e-7f ? atan2f(n, q.w) : 1.0f);
    px = f * q.x; py = f * q.y; pz = f * q.z;
}

// coefficients (a, b) of J(phi) = I + a [phi] + b [phi]^2 (sgn = +1) or of J(phi)^-1 (sgn = -1)
__device__ __forceinline__ void jac_coeffs(float px, float py, float pz, float sgn, float &a, float &b);

// out = v + a (phi x v) + b phi x (phi x v)
__device__ __forceinline__ void jac_mul(float px, float py, float pz, float a, float b, float vx, float vy, float vz,
                                        float &ox, float &oy, float &oz)
{
    const float cx = py * vz - pz * vy, cy = pz * vx - px * vz, cz = px * vy - py * vx;     // phi x v
    const float dx = py * cz - pz * cy, dy = pz * cx - px * cz, dz = px * cy - py * cx;     // phi x (phi x v)
    ox = vx + a * cx + b * dx;
    oy = vy + a * cy + b * dy;
    oz = vz + a * cz + b * dz;
}

__device__ __forceinline__ void jac_coeffs(float px, float py, float pz, float sgn, float &a, float &b)
{
    const float t2 = px * px + py * py + pz * pz;
    const float th = __builtin_amdgcn_sqrtf(t2);
    if (sgn > 0.0f) {
        if (th < 0.25f) {
            a = 0.5f - t2 * (1.0f / 24.0f) + t2 * t2 * (1.0f / 720.0f);
            b = (1.0f / 6.0f) - t2 * (1.0f / 120.0f) + t2 * t2 * (1.0f / 5040.0f);
        } else {
            const float sh = sinf(0.5f * th);
            a = 2.0f * sh * sh / t2;
            b = (th - sinf(th)) / (t2 * th);
        }
    } else {
        a = -0.5f;
        if (th < 0.25f) {
            b = (1.0f / 12.0f) + t2 * (1.0f / 720.0f) + t2 * t2 * (1.0f / 30240.0f);
        } else {
            float sh, ch;
            sincosf(0.5f * th, &sh, &ch);
            b = __builtin_amdgcn_rcpf(t2) - ch * __builtin_amdgcn_rcpf(2.0f * th * sh);
        }
    }
}

// out = J(phi) v   (sgn = +1)   or   J(phi)^-1 v   (sgn = -1)
__device__ __forceinline__ void jac_apply(float px, float py, float pz, float sgn, float vx, float vy, float vz,
                                          float &ox, float &oy, float &oz)
{
    float a, b;
    jac_coeffs(px, py, pz, sgn, a, b);
    jac_mul(px, py, pz, a, b, vx, vy, vz, ox, oy, oz);
}

}  // namespace pose
}  // namespace gm
