// GPU perception for the sphere world (G-MAPP Sec. IV-B and V-A): depth image ->
// world points (pinhole back-projection and the camera-to-world transform), and
// the uniform voxel lattice whose occupied cells' centres form S_W (voxel size
// 2 r_O, voxel-centre clouds).
//
// The cell of a point is the exact lattice coordinate floor((p - lo) / s) of the
// real numbers the FP32 values p, lo, s denote: an FP64 estimate of the quotient
// and one exact correction step decide it (lattice_axis), so points on or next to
// a face land in the cell the lattice assigns them, not wherever a rounded
// quotient happens to fall.
//
// The voxel pass is bandwidth/latency bound.  It marks cells in a grid over the
// caller's workspace box (which is also the bounding-box filter) that the context
// keeps all-zero between calls:
//   min_count = 1: an occupancy grid of bytes, marked with plain stores (racing
//     writers store the same value; device-scope atomics from every XCD on shared
//     words would be serialised at memory);
//   min_count > 1: a count grid (4 bytes per cell), marked with atomic adds that the
//     wave first combines per cell.
// A thread takes up to four consecutive points (or pixels) and merges equal cells
// first: neighbouring pixels mostly share a voxel.  The occupied cells' centres are then
// written in increasing linear cell index (x fastest, then y, then z) without a sort: per
// block of the grid, a counting pass (the grid's last reader: it leaves a 128-byte
// occupancy mask and clears what was marked), then a local scan of the mask that writes
// the centres, each block adding the counts of the blocks before it itself (up to
// kLocalBlocks blocks; past that one exclusive scan of the block counts runs in between).
// Only blocks holding a marked cell are read.  The count of occupied cells stays on the
// device.
//
// The fused pass (cam != nullptr) back-projects each pixel with the same FP32
// operations as the back-projection kernels and marks its cell directly, so the
// points are never written to memory and its cells equal those of the two-kernel
// path bit for bit.
#include "gmapp_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>

namespace gm {
namespace {

constexpr int kCellBlock = 1024;        // cells per block of the finish (4 per thread)
constexpr int kLocalBlocks = 1024;      // up to this many blocks each block adds its predecessors' counts itself
constexpr int kMaskWords = kCellBlock / 32;   // occupancy mask words per block
// inputs of up to this many points (pixels) -- one frame -- are marked in XCD bands
constexpr long long kBandMax = 1ll << 19;

// pixel (u, v) with z-depth d -> world point; NaN when d is not a positive finite depth
__device__ __forceinline__ void back_project(int u, int v, float d, float fx, float fy, float cx, float cy,
                                             const float *__restrict__ t, float &X, float &Y, float &Z)
{
    X = NAN; Y = NAN; Z = NAN;
    if (d > 0.0f && d < INFINITY) {
        const float xc = ((float)u - cx) * d / fx;    // pinhole: X_c = (u - c_x) z / f_x
        const float yc = ((float)v - cy) * d / fy;
        X = fmaf(t[0], xc, fmaf(t[1], yc, fmaf(t[2], d, t[3])));
        Y = fmaf(t[4], xc, fmaf(t[5], yc, fmaf(t[6], d, t[7])));
        Z = fmaf(t[8], xc, fmaf(t[9], yc, fmaf(t[10], d, t[11])));
    }
}

__global__ void k_depth_to_points(const float *__restrict__ depth, int w, int h, float fx, float fy, float cx,
                                  float cy, Mat34 T, float *__restrict__ x, float *__restrict__ y,
                                  float *__restrict__ z)
{
    const int n = w * h;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int v = i / w, u = i - v * w;
        float X, Y, Z;
        back_project(u, v, depth[i], fx, fy, cx, cy, T.r, X, Y, Z);
        x[i] = X;
        y[i] = Y;
        z[i] = Z;
    }
}

// Many frames of one camera, each with its own pose (device [n_frames][12]); four
// consecutive pixels per thread (w * h divisible by 4, 16-byte aligned arrays),
// so that the depth read and the three coordinate writes are 16-byte accesses.
__global__ void k_depth_to_points_v4(const float4 *__restrict__ depth, long long n4, int w, int wh, float fx, float fy,
                                     float cx, float cy, const float *__restrict__ T, float4 *__restrict__ x,
                                     float4 *__restrict__ y, float4 *__restrict__ z)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n4; i += (long long)gridDim.x * blockDim.x) {
        const long long p = 4 * i;
        const int f = (int)(p / wh);
        const int q = (int)(p - (long long)f * wh);
        const float *t = T + 12 * (size_t)f;
        const float4 d4 = depth[i];
        const float dd[4] = {d4.x, d4.y, d4.z, d4.w};
        float ox[4], oy[4], oz[4];
        int v = q / w, u = q - v * w;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            back_project(u, v, dd[k], fx, fy, cx, cy, t, ox[k], oy[k], oz[k]);
            if (++u == w) { u = 0; ++v; }
        }
        x[i] = make_float4(ox[0], ox[1], ox[2], ox[3]);
        y[i] = make_float4(oy[0], oy[1], oy[2], oy[3]);
        z[i] = make_float4(oz[0], oz[1], oz[2], oz[3]);
    }
}

// Any shape: one pixel per thread.
__global__ void k_depth_to_points_n(const float *__restrict__ depth, long long n, int w, int wh, float fx, float fy,
                                    float cx, float cy, const float *__restrict__ T, float *__restrict__ x,
                                    float *__restrict__ y, float *__restrict__ z)
{
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        const int f = (int)(p / wh);
        const int q = (int)(p - (long long)f * wh);
        const int v = q / w, u = q - v * w;
        float X, Y, Z;
        back_project(u, v, depth[p], fx, fy, cx, cy, T + 12 * (size_t)f, X, Y, Z);
        x[p] = X;
        y[p] = Y;
        z[p] = Z;
    }
}

__global__ void k_zero_u32(unsigned *p, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Exact lattice coordinate k = floor((p - lo) / s) of the real values of p (FP32),
// lo and s (FP32 values); false when p is not finite or k lies outside [0, dim).
// Fast path in FP32: q = fl(fl(p - lo) * fl(1 / s)) is within |q| 1.8e-7 of the true
// quotient (three roundings of relative 2^-24), so when its fractional part keeps a
// margin of |q| 2.4e-7 + 1e-6 from both faces, floor(q) is the cell.  Otherwise
// (about one coordinate in ten thousand near a face, or a non-finite one) the
// exact path decides in FP64:
//   * p - lo is taken exactly as hi + err (two-sum);
//   * floor(hi * inv_s) is within one of k (the quotient's relative error is ~2^-51);
//   * the side of a face k s is the sign of (hi - k s) + err: the fused multiply-add
//     rounds hi - k s once from its exact value, and either that value is exact or it
//     is far larger than err, so the FP64 sum has the exact sign.
__device__ __forceinline__ bool lattice_axis_exact(float p, double lo, double s, double inv_s, int dim, int &k)
{
    const double P = (double)p;
    const double hi = __dadd_rn(P, -lo);
    const double bb = __dadd_rn(hi, -P);
    const double err = __dadd_rn(__dadd_rn(P, -__dadd_rn(hi, -bb)), __dadd_rn(-lo, -bb));
    double kf = floor(__dmul_rn(hi, inv_s));
    if (!(kf >= -1.0 && kf <= (double)dim)) return false;       // also NaN / infinite p
    if (__dadd_rn(__fma_rn(-kf, s, hi), err) < 0.0) kf -= 1.0;
    else if (__dadd_rn(__fma_rn(-(kf + 1.0), s, hi), err) >= 0.0) kf += 1.0;
    if (!(kf >= 0.0 && kf < (double)dim)) return false;
    k = (int)kf;
    return true;
}

__device__ __forceinline__ bool lattice_axis(float p, int a, const VoxGrid &g, int &k)
{
    const float q = __fmul_rn(__fsub_rn(p, g.lo[a]), g.inv_s32);
    const float fl = floorf(q);
    const float f = __fsub_rn(q, fl);
    const float m = fmaf(fabsf(q), 2.4e-7f, 1e-6f);
    if (f > m && __fsub_rn(1.0f, f) > m) {
        if (!(fl >= 0.0f && fl < (float)g.dims[a])) return false;
        k = (int)fl;
        return true;
    }
    return lattice_axis_exact(p, g.lod[a], g.sd, g.inv_s, g.dims[a], k);
}

// linear cell of a point (x fastest; below 2^31, the grid's limit), -1 when outside
// the box or not finite
__device__ __forceinline__ int cell_of(float px, float py, float pz, const VoxGrid &g)
{
    int kx, ky, kz;
    if (!lattice_axis(px, 0, g, kx)) return -1;
    if (!lattice_axis(py, 1, g, ky)) return -1;
    if (!lattice_axis(pz, 2, g, kz)) return -1;
    return (int)(((unsigned)kz * (unsigned)g.dims[1] + (unsigned)ky) * (unsigned)g.dims[0] + (unsigned)kx);
}

// Robot self-filter: a point within any of the robot's bounding spheres (centre c,
// radius r) is dropped.  The test |p - c|^2 <= r^2 is taken in FP64 with every
// rounding explicit and in a fixed order, (dx dx + dy dy) + dz dz, so it is
// reproducible on any IEEE machine.
__device__ __forceinline__ bool on_robot(float px, float py, float pz, const VoxGrid &g)
{
    for (int k = 0; k < g.n_excl; ++k) {
        const float *s = g.excl + 4 * k;
        const double dx = __dadd_rn((double)px, -(double)s[0]);
        const double dy = __dadd_rn((double)py, -(double)s[1]);
        const double dz = __dadd_rn((double)pz, -(double)s[2]);
        const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
        if (d2 <= __dmul_rn((double)s[3], (double)s[3])) return true;
    }
    return false;
}

// the cell a point marks, -1 when it is dropped (outside the box, not finite, or on the robot)
__device__ __forceinline__ int mark_cell(float px, float py, float pz, const VoxGrid &g)
{
    const int c = cell_of(px, py, pz, g);
    if (c >= 0 && g.n_excl > 0 && on_robot(px, py, pz, g)) return -1;
    return c;
}

// sum over the 64 lanes of a wave, the result in every lane: DPP row rotations by 8, 4,
// 2, 1, the xor-16 swizzle and the 32-lane swap (VALU work, no LDS)
__device__ __forceinline__ unsigned wave_sum(unsigned x)
{
    x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xF, 0xF, false);   // row_ror:8
    x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x124, 0xF, 0xF, false);   // row_ror:4
    x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x122, 0xF, 0xF, false);   // row_ror:2
    x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x121, 0xF, 0xF, false);   // row_ror:1
    x += (unsigned)__builtin_amdgcn_ds_swizzle((int)x, 0x401F);                      // xor 16
    auto sw = __builtin_amdgcn_permlane32_swap((int)x, (int)x, false, false);
    return (unsigned)sw[0] + (unsigned)sw[1];
}

// Logical block of this workgroup for the marking kernels.  Workgroups are dispatched to
// the 8 XCDs round-robin (workgroup i to XCD i mod 8); with `band` set they are renumbered
// so that the workgroups of one XCD take one contiguous range of the points (pixels).
// Within one frame neighbouring pixels mark neighbouring cells, which share grid lines: a
// line marked from one XCD is merged in that XCD's L2 and written back once, instead of
// once per XCD that touched it (a single frame writes 4x fewer grid bytes).  Many frames
// of one scene mark the same lines from every band anyway, and there the bands measured
// slower, so the host sets `band` for single-frame inputs only.
__device__ __forceinline__ unsigned xcd_block(int band)
{
    const unsigned nb = gridDim.x, b = blockIdx.x;
    if (!band) return b;
    const unsigned x = b & 7u, per = nb >> 3, rem = nb & 7u;
    return x * per + min(x, rem) + (b >> 3);
}

// Marks one cell per lane (-1: none).
//   occupancy (min_count = 1): a plain store of byte 1 -- racing writers store the same
//     value, and the caches merge byte writes, so no atomic is needed;
//   counts: the lanes holding the lowest pending lane's cell add their points across the
//     wave and that lane issues one atomic add; repeat until no cell is left (neighbouring
//     points mostly share a cell, so the atomics, serialised per address, stay few).
template <bool COUNT, bool FLAG = true>
__device__ __forceinline__ void wave_mark(int cell, unsigned cnt, unsigned *__restrict__ grid,
                                          unsigned char *__restrict__ dirty)
{
    if constexpr (!COUNT) {
        // the block's dirty byte is stored by the first lane of each run of lanes in one
        // block (FLAG = false: the caller flags the blocks itself)
        if constexpr (FLAG) {
            const int blk = cell >= 0 ? (int)((unsigned)cell / kCellBlock) : -1;
            const int prev = __builtin_amdgcn_update_dpp(-2, blk, 0x111, 0xF, 0xF, false);   // row_shr:1
            if (cell >= 0 && prev != blk) dirty[blk] = 1;
        }
        if (cell >= 0) reinterpret_cast<unsigned char *>(grid)[(unsigned)cell] = 1;
    } else {
        const int lane = threadIdx.x & 63;
        unsigned long long pending = __ballot(cell >= 0);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const int c0 = __builtin_amdgcn_readlane(cell, leader);
            const bool mine = cell == c0;
            const unsigned v = wave_sum(mine ? cnt : 0u);
            if (lane == leader) {
                atomicAdd(&grid[(unsigned)c0], v);
                dirty[(unsigned)c0 / kCellBlock] = 1;
            }
            pending &= ~__ballot(mine);
            if (mine) cell = -1;
        }
    }
}

// Four consecutive points of a thread: a cell equal to the one before it merges into
// it (the run's first entry carries the run's points), then one mark per remaining
// entry (uniform control flow, static indexing).
template <bool COUNT>
__device__ __forceinline__ void mark4(const float (&X)[4], const float (&Y)[4], const float (&Z)[4], bool live,
                                      const VoxGrid &g, unsigned *__restrict__ grid, unsigned char *__restrict__ dirty)
{
    int c[4];
    unsigned n[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        n[r] = 1u;
        c[r] = live ? mark_cell(X[r], Y[r], Z[r], g) : -1;
    }
#pragma unroll
    for (int r = 3; r >= 1; --r)
        if (c[r] >= 0 && c[r] == c[r - 1]) {
            n[r - 1] += n[r];
            c[r] = -1;
        }
    if constexpr (!COUNT) {
        // dirty bytes of the thread's blocks (its four points nearly always share one): each
        // block the thread marks after a different one is flagged, the first one only when the
        // previous lane's last block differs
        int first = -1, lastb = -1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (c[r] < 0) continue;
            const int b = (int)((unsigned)c[r] / kCellBlock);
            if (first < 0) first = b;
            else if (b != lastb) dirty[b] = 1;
            lastb = b;
        }
        const int prev = __builtin_amdgcn_update_dpp(-2, lastb, 0x111, 0xF, 0xF, false);   // row_shr:1
        if (first >= 0 && first != prev) dirty[first] = 1;
#pragma unroll
        for (int r = 0; r < 4; ++r) wave_mark<COUNT, false>(c[r], n[r], grid, dirty);
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) wave_mark<COUNT>(c[r], n[r], grid, dirty);
    }
}

// points, one per thread (the loop trip count is uniform across the wave)
template <bool COUNT>
__global__ __launch_bounds__(256) void k_mark(const float *__restrict__ x, const float *__restrict__ y,
                                              const float *__restrict__ z, long long n, VoxGrid g,
                                              unsigned *__restrict__ grid, unsigned char *__restrict__ dirty, int band)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long wbase = xcd_block(band) * (long long)blockDim.x + (threadIdx.x & ~63);
    for (long long w0 = wbase; w0 < n; w0 += stride) {
        const long long i = w0 + (threadIdx.x & 63);
        wave_mark<COUNT>(i < n ? mark_cell(x[i], y[i], z[i], g) : -1, 1u, grid, dirty);
    }
}

// points, four per thread from 16-byte loads of each coordinate stream (x, y, z
// 16-byte aligned); the last n - 4 n4 (< 4) points go to the first lanes of the
// grid's first wave
template <bool COUNT>
__global__ __launch_bounds__(256) void k_mark_v4(const float4 *__restrict__ x4, const float4 *__restrict__ y4,
                                                 const float4 *__restrict__ z4, long long n4,
                                                 const float *__restrict__ x, const float *__restrict__ y,
                                                 const float *__restrict__ z, long long n, VoxGrid g,
                                                 unsigned *__restrict__ grid, unsigned char *__restrict__ dirty,
                                                 int band)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long tid = xcd_block(band) * (long long)blockDim.x + threadIdx.x;
    const long long wbase = tid - (threadIdx.x & 63);        // the wave's first thread (wave-uniform)
    for (long long w0 = wbase; w0 < n4; w0 += stride) {
        const long long i = w0 + (threadIdx.x & 63);
        float X[4] = {0, 0, 0, 0}, Y[4] = {0, 0, 0, 0}, Z[4] = {0, 0, 0, 0};
        const bool live = i < n4;
        if (live) {
            const float4 a = x4[i], b = y4[i], c = z4[i];
            X[0] = a.x; X[1] = a.y; X[2] = a.z; X[3] = a.w;
            Y[0] = b.x; Y[1] = b.y; Y[2] = b.z; Y[3] = b.w;
            Z[0] = c.x; Z[1] = c.y; Z[2] = c.z; Z[3] = c.w;
        }
        mark4<COUNT>(X, Y, Z, live, g, grid, dirty);
    }
    if (wbase == 0) {
        const long long t = 4 * n4 + tid;
        wave_mark<COUNT>(t < n ? mark_cell(x[t], y[t], z[t], g) : -1, 1u, grid, dirty);
    }
}

// frame and pixel of a flat pixel index (32-bit division when the index fits)
__device__ __forceinline__ void pixel_of(long long p, int w, int wh, int &f, int &u, int &v)
{
    int q;
    if ((unsigned long long)p < (1ull << 32)) {
        const unsigned pu = (unsigned)p;
        f = (int)(pu / (unsigned)wh);
        q = (int)(pu - (unsigned)f * (unsigned)wh);
    } else {
        f = (int)(p / wh);
        q = (int)(p - (long long)f * wh);
    }
    v = q / w;
    u = q - v * w;
}

// fused back-projection and marking: four consecutive pixels per thread from one
// 16-byte depth load (w h divisible by 4, depth 16-byte aligned)
template <bool COUNT>
__global__ __launch_bounds__(256) void k_mark_depth_v4(const float4 *__restrict__ depth, long long n4, Cam cam,
                                                       VoxGrid g, unsigned *__restrict__ grid,
                                                       unsigned char *__restrict__ dirty, int band)
{
    const int wh = cam.w * cam.h;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long wbase = xcd_block(band) * (long long)blockDim.x + (threadIdx.x & ~63);
    for (long long w0 = wbase; w0 < n4; w0 += stride) {
        const long long i = w0 + (threadIdx.x & 63);
        float X[4] = {0, 0, 0, 0}, Y[4] = {0, 0, 0, 0}, Z[4] = {0, 0, 0, 0};
        const bool live = i < n4;
        if (live) {
            int f, u, v;
            pixel_of(4 * i, cam.w, wh, f, u, v);
            const float *t = cam.T + 12 * (size_t)f;
            const float4 d4 = depth[i];
            const float dd[4] = {d4.x, d4.y, d4.z, d4.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                back_project(u, v, dd[k], cam.fx, cam.fy, cam.cx, cam.cy, t, X[k], Y[k], Z[k]);
                if (++u == cam.w) { u = 0; ++v; }
            }
        }
        mark4<COUNT>(X, Y, Z, live, g, grid, dirty);
    }
}

// fused, any shape: one pixel per thread
template <bool COUNT>
__global__ __launch_bounds__(256) void k_mark_depth(const float *__restrict__ depth, long long n, Cam cam, VoxGrid g,
                                                    unsigned *__restrict__ grid, unsigned char *__restrict__ dirty,
                                                    int band)
{
    const int wh = cam.w * cam.h;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long wbase = xcd_block(band) * (long long)blockDim.x + (threadIdx.x & ~63);
    for (long long w0 = wbase; w0 < n; w0 += stride) {
        const long long p = w0 + (threadIdx.x & 63);
        int c = -1;
        if (p < n) {
            int f, u, v;
            pixel_of(p, cam.w, wh, f, u, v);
            float X, Y, Z;
            back_project(u, v, depth[p], cam.fx, cam.fy, cam.cx, cam.cy, cam.T + 12 * (size_t)f, X, Y, Z);
            c = mark_cell(X, Y, Z, g);
        }
        wave_mark<COUNT>(c, 1u, grid, dirty);
    }
}

// Lattice coordinates of a linear cell index (x fastest); 32-bit arithmetic (the grid
// holds at most 2^31 cells).
struct CellIdx {
    unsigned x, y, z;
};
__device__ __forceinline__ CellIdx cell_coords(unsigned c, const VoxGrid &g)
{
    const unsigned d0 = (unsigned)g.dims[0], d1 = (unsigned)g.dims[1];
    const unsigned r = c / d0;
    return CellIdx{c - r * d0, r % d1, r / d1};
}
// voxel centre lo + (k + 1/2) s, rounded once to FP32: k + 1/2 is exact (k < 2^23 per axis) and
// the fused multiply-add rounds the exact product-plus-corner once
__device__ __forceinline__ void write_centre(const CellIdx &k, const VoxGrid &g, long long pos, float *__restrict__ ox,
                                             float *__restrict__ oy, float *__restrict__ oz)
{
    ox[pos] = fmaf((float)k.x + 0.5f, g.voxel, g.lo[0]);
    oy[pos] = fmaf((float)k.y + 0.5f, g.voxel, g.lo[1]);
    oz[pos] = fmaf((float)k.z + 0.5f, g.voxel, g.lo[2]);
}

// sum over a workgroup of NT threads (every thread gets it)
template <int NT>
__device__ __forceinline__ unsigned block_sum(unsigned v, unsigned *wsum)
{
    constexpr int NW = NT / 64;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned t = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) t += wsum[q];
    __syncthreads();
    return t;
}

// exclusive scan of one value per thread over a workgroup of NT threads (NT / 64 <= 16
// waves); returns the thread's prefix, `total` gets the workgroup's sum
template <int NT>
__device__ __forceinline__ unsigned block_excl_scan(unsigned c, unsigned *wsum, unsigned &total)
{
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned incl = c;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    unsigned before = 0, all = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        const unsigned s = wsum[q];
        before += q < wave ? s : 0u;
        all += s;
    }
    __syncthreads();
    total = all;
    return before + incl - c;
}


// The four cells [base, base + 4) of a thread in the finish: their occupancy (bit q)
// and whether any of them was marked.  Occupancy grid: one 32-bit load of 4 bytes;
// count grid: one 16-byte load of 4 counts (base is a multiple of 4; the grid is
// allocated in whole blocks, so the loads stay inside it).
template <bool COUNT>
__device__ __forceinline__ unsigned cells4(const unsigned *__restrict__ grid, long long base, unsigned min_count,
                                           bool &marked)
{
    unsigned occ = 0;
    if constexpr (COUNT) {
        const uint4 v = reinterpret_cast<const uint4 *>(grid)[base >> 2];
        occ = (v.x >= min_count ? 1u : 0u) | (v.y >= min_count ? 2u : 0u) | (v.z >= min_count ? 4u : 0u) |
              (v.w >= min_count ? 8u : 0u);
        marked = (v.x | v.y | v.z | v.w) != 0u;
    } else {
        const unsigned w = grid[base >> 2];
        occ = ((w & 0xFFu) ? 1u : 0u) | ((w & 0xFF00u) ? 2u : 0u) | ((w & 0xFF0000u) ? 4u : 0u) |
              ((w & 0xFF000000u) ? 8u : 0u);
        marked = w != 0u;
    }
    return occ;
}

__device__ __forceinline__ void clear4(unsigned *__restrict__ grid, long long base, bool count)
{
    if (count) reinterpret_cast<uint4 *>(grid)[base >> 2] = make_uint4(0u, 0u, 0u, 0u);
    else grid[base >> 2] = 0u;
}

// finish, pass 1: occupied cells per block of kCellBlock cells (4 per thread).  The grid's
// last reader: the block's occupancy goes to its mask (kMaskWords words, bit c for cell
// c of the block) and every marked grid word is cleared, so the writing pass reads
// 128 bytes per block instead of the block's grid.
template <bool COUNT>
__global__ __launch_bounds__(256) void k_block_cells(unsigned *__restrict__ grid,
                                                     const unsigned char *__restrict__ dirty, unsigned min_count,
                                                     unsigned *__restrict__ bsum, unsigned *__restrict__ mask)
{
    __shared__ unsigned wsum[4];
    const unsigned b = blockIdx.x, tid = threadIdx.x;
    if (!dirty[b]) {                              // no point marked a cell of this block
        if (tid == 0) bsum[b] = 0u;
        return;
    }
    const long long base = (long long)b * kCellBlock + tid * 4;
    bool marked;
    const unsigned occ = cells4<COUNT>(grid, base, min_count, marked);
    if (marked) clear4(grid, base, COUNT);
    // eight neighbouring threads' 4 bits form one mask word
    unsigned m = occ << (4 * (tid & 7));
    m |= __shfl_xor(m, 1, 64);
    m |= __shfl_xor(m, 2, 64);
    m |= __shfl_xor(m, 4, 64);
    if ((tid & 7) == 0) mask[(size_t)b * kMaskWords + (tid >> 3)] = m;
    const unsigned t = block_sum<256>(__popc(occ), wsum);
    if (tid == 0) bsum[b] = t;
}

// exclusive scan of nb block counts in place (one workgroup of 1024 threads);
// total -> *n_out (many blocks only)
__global__ __launch_bounds__(1024) void k_scan_blocks(unsigned *__restrict__ bsum, long long nb,
                                                      long long *__restrict__ n_out)
{
    __shared__ unsigned wsum[16];
    unsigned long long carry = 0;
    for (long long b0 = 0; b0 < nb; b0 += 1024) {
        const long long i = b0 + threadIdx.x;
        const unsigned v = i < nb ? bsum[i] : 0u;
        unsigned total;
        const unsigned ex = block_excl_scan<1024>(v, wsum, total);
        if (i < nb) bsum[i] = (unsigned)(carry + ex);
        carry += total;
    }
    if (threadIdx.x == 0) *n_out = (long long)carry;
}

// finish, pass 2: the block's occupied cells (its mask) are compacted in LDS in cell order
// (local scan), then written out as centres by consecutive threads (coalesced stores); the
// block's dirty flag is cleared.  Clean blocks write nothing (the last one still reports
// the total in local mode).
__global__ __launch_bounds__(256) void k_write_cells(const unsigned *__restrict__ mask,
                                                     unsigned char *__restrict__ dirty,
                                                     const unsigned *__restrict__ bsum, int local,
                                                     long long *__restrict__ n_out, VoxGrid g, float *__restrict__ ox,
                                                     float *__restrict__ oy, float *__restrict__ oz, long long capacity)
{
    __shared__ unsigned wsum[16];
    __shared__ unsigned short cellbuf[kCellBlock];
    const unsigned b = blockIdx.x, tid = threadIdx.x;
    const bool d = dirty[b] != 0;
    const bool last = b == gridDim.x - 1;
    if (!d && !(local && last)) return;
    // the block's first position: the counts of the blocks before it (local: up to
    // kLocalBlocks of them, 4 per thread, loaded together with the mask) or the scanned table
    unsigned before = 0;
    if (local) {
#pragma unroll
        for (unsigned q = 0; q < kLocalBlocks / 256; ++q) {
            const unsigned i = tid + 256 * q;
            before += i < b ? bsum[i] : 0u;
        }
    }
    unsigned occ = d ? (mask[(size_t)b * kMaskWords + (tid >> 3)] >> (4 * (tid & 7))) & 0xFu : 0u;
    unsigned total;
    unsigned at = block_excl_scan<256>(__popc(occ), wsum, total);
    long long pos0;
    if (local) {
        pos0 = (long long)block_sum<256>(before, wsum + 4);
        if (last && tid == 0) *n_out = pos0 + total;
    } else {
        pos0 = (long long)bsum[b];
    }
    if (d && tid == 0) dirty[b] = 0;              // every thread read it before the scan's barriers
    while (occ) {
        cellbuf[at++] = (unsigned short)(4 * tid + (unsigned)(__ffs(occ) - 1));
        occ &= occ - 1u;
    }
    __syncthreads();
    const unsigned cbase = b * (unsigned)kCellBlock;
    for (unsigned j = tid; j < total; j += 256) {
        const long long pos = pos0 + j;
        if (pos < capacity) write_centre(cell_coords(cbase + cellbuf[j], g), g, pos, ox, oy, oz);
    }
}

}  // namespace

gmapp_status launch_depth_to_points(gmapp_ctx *ctx, const float *depth, int w, int h, const float K[4],
                                    const Mat34 &T, float *x, float *y, float *z, hipStream_t stream)
{
    const long long n = (long long)w * h;
    if (n == 0) return GMAPP_OK;
    const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_depth_to_points, dim3(blocks), dim3(256), 0, stream, depth, w, h, K[0], K[1], K[2], K[3], T,
                       x, y, z);
    GM_HIP(ctx, hipGetLastError());
    return GMAPP_OK;
}

namespace {
bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
}  // namespace

gmapp_status launch_depth_to_points_batch(gmapp_ctx *ctx, const float *depth, int n_frames, int w, int h,
                                          const float K[4], const float *T_dev, float *x, float *y, float *z,
                                          hipStream_t stream)
{
    const long long wh = (long long)w * h, n = wh * n_frames;
    if (n == 0) return GMAPP_OK;
    if (wh % 4 == 0 && aligned16(depth) && aligned16(x) && aligned16(y) && aligned16(z)) {
        const long long n4 = n / 4;
        const int blocks = (int)std::min<long long>((n4 + 255) / 256, 16384);
        hipLaunchKernelGGL(k_depth_to_points_v4, dim3(blocks), dim3(256), 0, stream,
                           reinterpret_cast<const float4 *>(depth), n4, w, (int)wh, K[0], K[1], K[2], K[3], T_dev,
                           reinterpret_cast<float4 *>(x), reinterpret_cast<float4 *>(y), reinterpret_cast<float4 *>(z));
    } else {
        const int blocks = (int)std::min<long long>((n + 255) / 256, 16384);
        hipLaunchKernelGGL(k_depth_to_points_n, dim3(blocks), dim3(256), 0, stream, depth, n, w, (int)wh, K[0], K[1],
                           K[2], K[3], T_dev, x, y, z);
    }
    GM_HIP(ctx, hipGetLastError());
    return GMAPP_OK;
}

namespace {

template <bool COUNT>
void launch_mark(gmapp_ctx *ctx, const float *x, const float *y, const float *z, long long n, const Cam *cam,
                 const VoxGrid &g, unsigned *grid, unsigned char *dirty, hipStream_t stream)
{
    if (n == 0) return;
    const int band = n <= kBandMax ? 1 : 0;
    // four points (pixels) per thread only when the quads still give every SIMD two waves;
    // below that one per thread hides more latency
    const long long fill = 2ll * 64 * 4 * std::max(ctx->n_cu, 1);
    if (cam) {
        const long long wh = (long long)cam->w * cam->h;
        if (wh % 4 == 0 && aligned16(x) && n / 4 >= fill) {
            const long long n4 = n / 4;
            const int pb = (int)std::min<long long>((n4 + 255) / 256, 16384);
            hipLaunchKernelGGL(k_mark_depth_v4<COUNT>, dim3(pb), dim3(256), 0, stream,
                               reinterpret_cast<const float4 *>(x), n4, *cam, g, grid, dirty, band);
        } else {
            const int pb = (int)std::min<long long>((n + 255) / 256, 16384);
            hipLaunchKernelGGL(k_mark_depth<COUNT>, dim3(pb), dim3(256), 0, stream, x, n, *cam, g, grid, dirty, band);
        }
        return;
    }
    if (n / 4 >= fill && aligned16(x) && aligned16(y) && aligned16(z)) {
        const long long n4 = n / 4;
        const int pb = (int)std::min<long long>((n4 + 255) / 256, 16384);
        hipLaunchKernelGGL(k_mark_v4<COUNT>, dim3(pb), dim3(256), 0, stream, reinterpret_cast<const float4 *>(x),
                           reinterpret_cast<const float4 *>(y), reinterpret_cast<const float4 *>(z), n4, x, y, z, n,
                           g, grid, dirty, band);
    } else {
        const int pb = (int)std::min<long long>((n + 255) / 256, 16384);
        hipLaunchKernelGGL(k_mark<COUNT>, dim3(pb), dim3(256), 0, stream, x, y, z, n, g, grid, dirty, band);
    }
}

}  // namespace

namespace {

VoxGrid with_derived(const VoxGrid &g_in)
{
    VoxGrid g = g_in;
    for (int a = 0; a < 3; ++a) g.lod[a] = (double)g.lo[a];
    g.sd = (double)g.voxel;
    g.inv_s = 1.0 / g.sd;
    g.inv_s32 = 1.0f / g.voxel;
    return g;
}

long long cells_of(const VoxGrid &g) { return (long long)g.dims[0] * g.dims[1] * g.dims[2]; }
long long blocks_of(const VoxGrid &g) { return (cells_of(g) + kCellBlock - 1) / kCellBlock; }
// u32 words of grid for a pass: whole blocks, 1 word per cell (counts) or per 4 cells (occupancy bytes)
size_t grid_words(const VoxGrid &g, unsigned min_count)
{
    return (size_t)blocks_of(g) * (min_count > 1 ? kCellBlock : kCellBlock / 4);
}

// Words of a block table for up to nb blocks: nb block counts (padded to 4 words), one
// dirty byte per block (all zero between passes), then kMaskWords mask words per block.
size_t count_words(long long nb) { return ((size_t)nb + 3) & ~(size_t)3; }
size_t dirty_words(long long nb) { return ((size_t)nb + 3) / 4; }
size_t table_words(long long nb) { return count_words(nb) + dirty_words(nb) + (size_t)nb * kMaskWords; }

// marking and finish on an all-zero grid and all-zero dirty bytes (both left so)
gmapp_status run_voxel(gmapp_ctx *ctx, const float *x, const float *y, const float *z, long long n, const Cam *cam,
                       const VoxGrid &g, unsigned min_count, unsigned *grid, unsigned *bsum, unsigned char *dirty,
                       unsigned *mask, float *ox, float *oy, float *oz, long long capacity, long long *n_out_dev,
                       hipStream_t stream)
{
    const long long nb = blocks_of(g);
    const int local = nb <= kLocalBlocks ? 1 : 0;
    if (min_count > 1) {
        launch_mark<true>(ctx, x, y, z, n, cam, g, grid, dirty, stream);
        hipLaunchKernelGGL(k_block_cells<true>, dim3((unsigned)nb), dim3(256), 0, stream, grid, dirty, min_count,
                           bsum, mask);
    } else {
        launch_mark<false>(ctx, x, y, z, n, cam, g, grid, dirty, stream);
        hipLaunchKernelGGL(k_block_cells<false>, dim3((unsigned)nb), dim3(256), 0, stream, grid, dirty, min_count,
                           bsum, mask);
    }
    if (!local) hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, stream, bsum, nb, n_out_dev);
    hipLaunchKernelGGL(k_write_cells, dim3((unsigned)nb), dim3(256), 0, stream, mask, dirty, bsum, local, n_out_dev,
                       g, ox, oy, oz, capacity);
    GM_HIP(ctx, hipGetLastError());
    return GMAPP_OK;
}

}  // namespace

// The context's grid stays all-zero between calls: it is zero-filled when (re)allocated,
// and every finish kernel clears what the marking set.
gmapp_status launch_voxel_downsample(gmapp_ctx *ctx, const float *x, const float *y, const float *z, long long n,
                                     const Cam *cam, const VoxGrid &g_in, unsigned min_count, float *ox, float *oy,
                                     float *oz, long long capacity, long long *n_out_dev, hipStream_t stream)
{
    const VoxGrid g = with_derived(g_in);
    const long long nb = blocks_of(g);
    const size_t need = grid_words(g, min_count);
    if (need > ctx->vgrid_words) {
        if (ctx->vgrid) {
            GM_HIP(ctx, hipStreamSynchronize(stream));
            (void)hipFree(ctx->vgrid);
            ctx->vgrid = nullptr;
            ctx->vgrid_words = 0;
        }
        void *p = nullptr;
        if (hipMalloc(&p, need * sizeof(unsigned)) != hipSuccess)
            return fail(ctx, GMAPP_ENOMEM, "voxel grid of %lld cells: cannot allocate %zu bytes", cells_of(g),
                        need * sizeof(unsigned));
        ctx->vgrid = static_cast<unsigned *>(p);
        ctx->vgrid_words = need;
        const int zb = (int)std::min<long long>(((long long)need + 255) / 256, 8192);
        hipLaunchKernelGGL(k_zero_u32, dim3(zb), dim3(256), 0, stream, ctx->vgrid, (long long)need);
    }
    const size_t tw = table_words(nb);
    if (tw > table_words((long long)ctx->vbsum_blocks)) {
        if (ctx->vbsum) {
            GM_HIP(ctx, hipStreamSynchronize(stream));
            (void)hipFree(ctx->vbsum);
            ctx->vbsum = nullptr;
            ctx->vbsum_blocks = 0;
        }
        void *p = nullptr;
        if (hipMalloc(&p, tw * sizeof(unsigned)) != hipSuccess)
            return fail(ctx, GMAPP_ENOMEM, "voxel block table of %lld entries: cannot allocate", nb);
        ctx->vbsum = static_cast<unsigned *>(p);
        ctx->vbsum_blocks = (size_t)nb;
        hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)std::min<size_t>((tw + 255) / 256, 8192)), dim3(256), 0, stream,
                           ctx->vbsum, (long long)tw);
    }
    unsigned *dirty = ctx->vbsum + count_words((long long)ctx->vbsum_blocks);
    return run_voxel(ctx, x, y, z, n, cam, g, min_count, ctx->vgrid, ctx->vbsum,
                     reinterpret_cast<unsigned char *>(dirty), dirty + dirty_words((long long)ctx->vbsum_blocks), ox,
                     oy, oz, capacity, n_out_dev, stream);
}

// ---------------------------------------------------------------- the pass without allocation
// A statically sized grid and block table for callers that cannot allocate: one copy per
// device, for the life of the process (the count grid of kStaticCells cells, its block
// table after it).  In host code `scratch` names a host-side stand-in, not device memory:
// its device address per device comes from hipGetSymbolAddress at set-up and is the only
// way the host ever refers to it.
namespace {
constexpr size_t kStaticBlocks = (size_t)kStaticCells / kCellBlock;
constexpr size_t kStaticWords = (size_t)kStaticCells + kStaticBlocks + kStaticBlocks / 4 +
                                kStaticBlocks * kMaskWords;     // grid, counts, dirty bytes, masks
static __device__ __align__(256) unsigned scratch[kStaticWords];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned *g_scratch_dev[kMaxDevices] = {};
}  // namespace

gmapp_status static_scratch_init(gmapp_ctx *ctx)
{
    if (ctx->device < 0 || ctx->device >= kMaxDevices)
        return fail(ctx, GMAPP_EDEVICE, "device %d is beyond the %d devices the static grid covers", ctx->device,
                    kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[ctx->device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                   "hipGetSymbolAddress(scratch)");
        unsigned *d = static_cast<unsigned *>(p);
        // all-zero before the first pass (every pass leaves the grid as it found it)
        hipLaunchKernelGGL(k_zero_u32, dim3(2048), dim3(256), 0, nullptr, d, (long long)kStaticWords);
        GM_HIP(ctx, hipGetLastError());
        GM_HIP(ctx, hipDeviceSynchronize());
        g_scratch_dev[ctx->device] = d;
    }
    ctx->static_grid = g_scratch_dev[ctx->device];
    return GMAPP_OK;
}

gmapp_status launch_voxel_downsample_static(gmapp_ctx *ctx, const float *x, const float *y, const float *z,
                                            long long n, const VoxGrid &g_in, unsigned min_count, float *ox,
                                            float *oy, float *oz, long long capacity, long long *n_out_dev,
                                            hipStream_t stream)
{
    const VoxGrid g = with_derived(g_in);
    if (cells_of(g) > kStaticCells)
        return fail(ctx, GMAPP_ECAPACITY, "voxel grid of %lld cells exceeds the static grid's %lld cells",
                    cells_of(g), kStaticCells);
    if (!ctx->static_grid) return fail(ctx, GMAPP_EDEVICE, "the static voxel grid was not set up");
    unsigned *grid = ctx->static_grid;
    unsigned *bsum = ctx->static_grid + kStaticCells;
    unsigned *dirty = bsum + kStaticBlocks;
    return run_voxel(ctx, x, y, z, n, nullptr, g, min_count, grid, bsum, reinterpret_cast<unsigned char *>(dirty),
                     dirty + dirty_words((long long)kStaticBlocks), ox, oy, oz, capacity, n_out_dev, stream);
}

}  // namespace gm
