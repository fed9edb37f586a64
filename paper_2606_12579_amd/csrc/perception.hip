// GPU perception for the sphere world (G-MAPP Sec. IV-B and V-A): depth image ->
// world points (pinhole back-projection and the camera-to-world transform), and
// the uniform voxel lattice whose occupied cells' centres form S_W (voxel size
// 2 r_O, voxel-centre clouds).
//
// The voxel pass is bandwidth/latency bound.  It works on a dense count grid
// over the caller's workspace box (which is also the bounding-box filter):
//   1. clear the grid,  2. mark each point's cell (atomic increments when min_count > 1),
//   3. per 1024-cell block: count the cells holding >= min_count points,
//   4. exclusive scan of the block counts (one workgroup),
//   5. per block: local scan and write the occupied cells' centres.
// The output is therefore sorted by linear cell index (x fastest, then y, then
// z) without any sort, and the count of occupied cells stays on the device.
#include "gmapp_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdint>

namespace gm {
namespace {

constexpr int kScanBlock = 1024;   // cells per block in steps 3 and 5 (256 threads x 4)

__global__ void k_depth_to_points(const float *__restrict__ depth, int w, int h, float fx, float fy, float cx,
                                  float cy, Mat34 T, float *__restrict__ x, float *__restrict__ y,
                                  float *__restrict__ z)
{
    const int n = w * h;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int v = i / w, u = i - v * w;
        const float d = depth[i];
        float X = NAN, Y = NAN, Z = NAN;
        if (d > 0.0f && d < INFINITY) {
            const float xc = ((float)u - cx) * d / fx;    // pinhole: X_c = (u - c_x) z / f_x
            const float yc = ((float)v - cy) * d / fy;
            const float zc = d;
            X = fmaf(T.r[0], xc, fmaf(T.r[1], yc, fmaf(T.r[2], zc, T.r[3])));
            Y = fmaf(T.r[4], xc, fmaf(T.r[5], yc, fmaf(T.r[6], zc, T.r[7])));
            Z = fmaf(T.r[8], xc, fmaf(T.r[9], yc, fmaf(T.r[10], zc, T.r[11])));
        }
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
            const float d = dd[k];
            float X = NAN, Y = NAN, Z = NAN;
            if (d > 0.0f && d < INFINITY) {
                const float xc = ((float)u - cx) * d / fx;
                const float yc = ((float)v - cy) * d / fy;
                X = fmaf(t[0], xc, fmaf(t[1], yc, fmaf(t[2], d, t[3])));
                Y = fmaf(t[4], xc, fmaf(t[5], yc, fmaf(t[6], d, t[7])));
                Z = fmaf(t[8], xc, fmaf(t[9], yc, fmaf(t[10], d, t[11])));
            }
            ox[k] = X; oy[k] = Y; oz[k] = Z;
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
        const float *t = T + 12 * (size_t)f;
        const float d = depth[p];
        float X = NAN, Y = NAN, Z = NAN;
        if (d > 0.0f && d < INFINITY) {
            const float xc = ((float)u - cx) * d / fx;
            const float yc = ((float)v - cy) * d / fy;
            X = fmaf(t[0], xc, fmaf(t[1], yc, fmaf(t[2], d, t[3])));
            Y = fmaf(t[4], xc, fmaf(t[5], yc, fmaf(t[6], d, t[7])));
            Z = fmaf(t[8], xc, fmaf(t[9], yc, fmaf(t[10], d, t[11])));
        }
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

// cell of a point: floor((p - lo) / voxel) per axis in FP32; -1 when outside the box
__device__ __forceinline__ long long cell_of(float px, float py, float pz, const VoxGrid &g)
{
    if (!(px == px) || !(py == py) || !(pz == pz)) return -1;
    const float fx = floorf((px - g.lo[0]) / g.voxel);
    const float fy = floorf((py - g.lo[1]) / g.voxel);
    const float fz = floorf((pz - g.lo[2]) / g.voxel);
    if (!(fx >= 0.0f && fy >= 0.0f && fz >= 0.0f)) return -1;
    if (!(fx < (float)g.dims[0] && fy < (float)g.dims[1] && fz < (float)g.dims[2])) return -1;
    return ((long long)fz * g.dims[1] + (long long)fy) * g.dims[0] + (long long)fx;
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

// mark a point's cell: occupancy (min_count 1: a plain store of 1, racing writers
// store the same value) or counts (atomic increments)
template <bool COUNT>
__device__ __forceinline__ void mark(float px, float py, float pz, const VoxGrid &g, unsigned *__restrict__ grid)
{
    long long c = cell_of(px, py, pz, g);
    if (c >= 0 && g.n_excl > 0 && on_robot(px, py, pz, g)) c = -1;
    if (c >= 0) {
        if constexpr (COUNT) atomicAdd(&grid[c], 1u);
        else grid[c] = 1u;
    }
}

template <bool COUNT>
__global__ void k_count(const float *__restrict__ x, const float *__restrict__ y, const float *__restrict__ z,
                        long long n, VoxGrid g, unsigned *__restrict__ grid)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        mark<COUNT>(x[i], y[i], z[i], g, grid);
}

// The same with four points per thread from 16-byte loads of each coordinate stream
// (x, y, z 16-byte aligned); the last n - 4 n4 (< 4) points go to the first threads.
template <bool COUNT>
__global__ __launch_bounds__(256) void k_count_v4(const float4 *__restrict__ x4, const float4 *__restrict__ y4,
                                                  const float4 *__restrict__ z4, long long n4,
                                                  const float *__restrict__ x, const float *__restrict__ y,
                                                  const float *__restrict__ z, long long n, VoxGrid g,
                                                  unsigned *__restrict__ grid)
{
    const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    for (long long i = tid; i < n4; i += (long long)gridDim.x * blockDim.x) {
        const float4 a = x4[i], b = y4[i], c = z4[i];
        mark<COUNT>(a.x, b.x, c.x, g, grid);
        mark<COUNT>(a.y, b.y, c.y, g, grid);
        mark<COUNT>(a.z, b.z, c.z, g, grid);
        mark<COUNT>(a.w, b.w, c.w, g, grid);
    }
    const long long t = 4 * n4 + tid;
    if (t < n) mark<COUNT>(x[t], y[t], z[t], g, grid);
}

__device__ __forceinline__ unsigned block_sum(unsigned v, unsigned *sh)
{
    // 256 threads: wave sums, then the 4 wave totals
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[wave] = v;
    __syncthreads();
    const unsigned t = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(256) void k_block_counts(const unsigned *__restrict__ grid, long long cells,
                                                      unsigned min_count, unsigned *__restrict__ bsum)
{
    __shared__ unsigned sh[4];
    const long long base = (long long)blockIdx.x * kScanBlock + threadIdx.x * 4;
    unsigned c = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (base + q < cells && grid[base + q] >= min_count) ++c;
    const unsigned t = block_sum(c, sh);
    if (threadIdx.x == 0) bsum[blockIdx.x] = t;
}

// exclusive scan of nb block counts in place (one workgroup of 1024 threads);
// total -> *n_out
__global__ __launch_bounds__(1024) void k_scan_blocks(unsigned *__restrict__ bsum, long long nb,
                                                      long long *__restrict__ n_out)
{
    __shared__ unsigned wsum[16];
    __shared__ unsigned long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (long long b0 = 0; b0 < nb; b0 += 1024) {
        const long long i = b0 + threadIdx.x;
        const unsigned v = i < nb ? bsum[i] : 0u;
        unsigned incl = v;                           // inclusive scan inside the wave
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned o = __shfl_up(incl, off, 64);
            if (lane >= off) incl += o;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        unsigned before = 0;
        for (int q = 0; q < wave; ++q) before += wsum[q];
        unsigned chunk_total = 0;
        for (int q = 0; q < 16; ++q) chunk_total += wsum[q];
        const unsigned long long base = carry;
        if (i < nb) bsum[i] = (unsigned)(base + before + incl - v);
        __syncthreads();
        if (threadIdx.x == 0) carry = base + chunk_total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_out = (long long)carry;
}

__global__ __launch_bounds__(256) void k_write_centres(const unsigned *__restrict__ grid, long long cells,
                                                       unsigned min_count, const unsigned *__restrict__ boff,
                                                       VoxGrid g, float *__restrict__ ox, float *__restrict__ oy,
                                                       float *__restrict__ oz, long long capacity)
{
    __shared__ unsigned wsum[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long base = (long long)blockIdx.x * kScanBlock + threadIdx.x * 4;
    unsigned f[4], c = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        f[q] = (base + q < cells && grid[base + q] >= min_count) ? 1u : 0u;
        c += f[q];
    }
    unsigned incl = c;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    unsigned before = 0;
    for (int q = 0; q < wave; ++q) before += wsum[q];
    long long pos = (long long)boff[blockIdx.x] + before + incl - c;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (f[q]) {
            if (pos < capacity) {
                const long long cell = base + q;
                const long long kx = cell % g.dims[0];
                const long long r = cell / g.dims[0];
                const long long ky = r % g.dims[1];
                const long long kz = r / g.dims[1];
                ox[pos] = fmaf((float)kx + 0.5f, g.voxel, g.lo[0]);   // voxel centre lo + (k + 1/2) s
                oy[pos] = fmaf((float)ky + 0.5f, g.voxel, g.lo[1]);
                oz[pos] = fmaf((float)kz + 0.5f, g.voxel, g.lo[2]);
            }
            ++pos;
        }
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

gmapp_status launch_depth_to_points_batch(gmapp_ctx *ctx, const float *depth, int n_frames, int w, int h,
                                          const float K[4], const float *T_dev, float *x, float *y, float *z,
                                          hipStream_t stream)
{
    const long long wh = (long long)w * h, n = wh * n_frames;
    if (n == 0) return GMAPP_OK;
    auto aligned = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
    if (wh % 4 == 0 && aligned(depth) && aligned(x) && aligned(y) && aligned(z)) {
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

size_t voxel_workspace_bytes(long long cells)
{
    const long long nb = (cells + kScanBlock - 1) / kScanBlock;
    return ((size_t)cells * 4 + 255) / 256 * 256 + (size_t)nb * 4;
}

gmapp_status launch_voxel_downsample(gmapp_ctx *ctx, const float *x, const float *y, const float *z, long long n,
                                     const VoxGrid &g, unsigned min_count, float *ox, float *oy, float *oz,
                                     long long capacity, long long *n_out_dev, hipStream_t stream)
{
    const long long cells = (long long)g.dims[0] * g.dims[1] * g.dims[2];
    const long long nb = (cells + kScanBlock - 1) / kScanBlock;
    if (voxel_workspace_bytes(cells) > ctx->scratch_bytes)
        return fail(ctx, GMAPP_ENOMEM, "voxel grid of %lld cells needs %zu workspace bytes, the context has %zu",
                    cells, voxel_workspace_bytes(cells), ctx->scratch_bytes);
    unsigned *grid = reinterpret_cast<unsigned *>(ctx->scratch);
    unsigned *bsum = reinterpret_cast<unsigned *>(ctx->scratch + ((size_t)cells * 4 + 255) / 256 * 256);
    const int zb = (int)std::min<long long>((cells + 255) / 256, 8192);
    hipLaunchKernelGGL(k_zero_u32, dim3(zb), dim3(256), 0, stream, grid, cells);
    // four points per thread only when the quads still give every SIMD two waves; below that
    // one point per thread hides more latency
    auto aligned = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
    const long long fill = 2ll * 64 * 4 * std::max(ctx->n_cu, 1);
    if (n / 4 >= fill && aligned(x) && aligned(y) && aligned(z)) {
        const long long n4 = n / 4;
        const int pb = (int)std::min<long long>((n4 + 255) / 256, 16384);
        const float4 *x4 = reinterpret_cast<const float4 *>(x), *y4 = reinterpret_cast<const float4 *>(y);
        const float4 *z4 = reinterpret_cast<const float4 *>(z);
        if (min_count > 1)
            hipLaunchKernelGGL(k_count_v4<true>, dim3(pb), dim3(256), 0, stream, x4, y4, z4, n4, x, y, z, n, g, grid);
        else
            hipLaunchKernelGGL(k_count_v4<false>, dim3(pb), dim3(256), 0, stream, x4, y4, z4, n4, x, y, z, n, g, grid);
    } else if (n > 0) {
        const int pb = (int)std::min<long long>((n + 255) / 256, 8192);
        if (min_count > 1) hipLaunchKernelGGL(k_count<true>, dim3(pb), dim3(256), 0, stream, x, y, z, n, g, grid);
        else hipLaunchKernelGGL(k_count<false>, dim3(pb), dim3(256), 0, stream, x, y, z, n, g, grid);
    }
    hipLaunchKernelGGL(k_block_counts, dim3((unsigned)nb), dim3(256), 0, stream, grid, cells, min_count, bsum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, stream, bsum, nb, n_out_dev);
    hipLaunchKernelGGL(k_write_centres, dim3((unsigned)nb), dim3(256), 0, stream, grid, cells, min_count, bsum, g, ox,
                       oy, oz, capacity);
    GM_HIP(ctx, hipGetLastError());
    return GMAPP_OK;
}

}  // namespace gm
