"""FP64 / exact reference of the perception pass -- TEST INFRASTRUCTURE ONLY.

  back_project(depth, K, T_wc)   pinhole back-projection and the camera-to-world
                                 transform (Sec. IV-B, V-A), FP64 from FP32 inputs
  voxel_keys(x, y, z, ...)       lattice coordinates of points in the uniform voxel
                                 lattice of size 2 r_O (Sec. IV-B, V-A): the exact
                                 floor((p - lo) / voxel) of the real quotient of the given
                                 coordinate, corner and voxel size (exact rationals where
                                 an FP64 quotient cannot decide the floor)
  voxel_cells(x, y, z, ...)      the occupied cells of that lattice
  voxel_centres(cells, ...)      the voxel-centre cloud: lo + (k + 1/2) voxel of the exact
                                 values, rounded once to FP32 (exact rationals where FP64
                                 cannot decide the rounding)
  on_robot(x, y, z, spheres)     the robot self-filter of Sec. V-A: points within any
                                 of the robot's bounding spheres (an integer decision,
                                 taken in FP64 as the library takes it)
"""
import math
from fractions import Fraction

import numpy as np


def back_project(depth, K, T_wc):
    """World points [h*w, 3] (NaN rows for depth <= 0 or non-finite)."""
    d = np.asarray(depth, np.float64)
    h, w = d.shape
    fx, fy, cx, cy = (float(np.float32(k)) for k in K)
    T = np.asarray(T_wc, np.float32).astype(np.float64).reshape(3, 4)
    u, v = np.meshgrid(np.arange(w, dtype=np.float64), np.arange(h, dtype=np.float64))
    with np.errstate(invalid="ignore", over="ignore"):
        Xc = np.stack([(u - cx) * d / fx, (v - cy) * d / fy, d], -1).reshape(-1, 3)
        P = Xc @ T[:, :3].T + T[:, 3]
    bad = ~(np.isfinite(d.reshape(-1)) & (d.reshape(-1) > 0))
    P[bad] = np.nan
    return P


def _exact_floor(p, lo, s):
    """floor((p - lo) / s) of the exact real numbers that the floats p, lo, s denote."""
    return math.floor((Fraction(float(p)) - Fraction(float(lo))) / Fraction(float(s)))


def voxel_keys(x, y, z, voxel, lo, dims):
    """Integer cell coordinates [n, 3] and a validity mask (inside the box, finite).

    The cell of a coordinate p is floor((p - lo) / voxel) of the real numbers that
    p (FP32 or FP64), lo and voxel (FP32) denote: the uniform lattice itself, with no
    rounding.  The FP64 quotient decides the floor wherever it is farther from an
    integer than its own rounding error (three roundings, relative 2^-53 each: far
    below the 1e-9 relative margin used); the remaining coordinates are decided with
    exact rationals."""
    P = np.stack([np.asarray(x), np.asarray(y), np.asarray(z)], 1)
    P = P.astype(np.float64) if P.dtype != np.float32 else P
    lo32 = np.asarray(lo, np.float32)
    s32 = np.float32(voxel)
    k = np.zeros(P.shape, np.int64)
    fin = np.isfinite(P).all(1)
    with np.errstate(invalid="ignore", over="ignore"):
        q = (P.astype(np.float64) - lo32.astype(np.float64)) / np.float64(s32)
        kf = np.floor(q)
        small = fin[:, None] & (np.abs(q) < 2.0 ** 52)      # beyond that no grid reaches: outside
        amb = small & (np.abs(q - np.round(q)) <= 1e-9 * np.maximum(1.0, np.abs(q)))
    k[small] = kf[small].astype(np.int64)
    for i, a in zip(*np.nonzero(amb)):
        k[i, a] = _exact_floor(P[i, a], lo32[a], s32)
    d = np.asarray(dims, np.int64)
    ok = fin & small.all(1) & (k >= 0).all(1) & (k < d).all(1)
    k[~ok] = 0
    return k, ok


def on_robot(x, y, z, spheres):
    """Mask of the points p with |p - c|^2 <= r^2 for some sphere (c, r) of spheres
    [K, 4] (FP32 values), in FP64 as ((dx dx + dy dy) + dz dz) -- each numpy
    operation rounds once, as each operation of the library does."""
    P = np.stack([np.asarray(x, np.float32), np.asarray(y, np.float32), np.asarray(z, np.float32)], 1)
    P = P.astype(np.float64)
    S = np.asarray(spheres, np.float32).astype(np.float64).reshape(-1, 4)
    hit = np.zeros(P.shape[0], bool)
    for c in S:
        dx, dy, dz = P[:, 0] - c[0], P[:, 1] - c[1], P[:, 2] - c[2]
        with np.errstate(invalid="ignore"):
            hit |= ((dx * dx + dy * dy) + dz * dz) <= c[3] * c[3]
    return hit


def voxel_cells(x, y, z, voxel, lo, dims, min_count=1, spheres=None):
    """Sorted linear indices (x fastest) of the cells holding >= min_count points
    (points on the robot, within spheres [K, 4], removed first)."""
    k, ok = voxel_keys(x, y, z, voxel, lo, dims)
    if spheres is not None and len(spheres):
        ok &= ~on_robot(x, y, z, spheres)
    dims = np.asarray(dims, np.int64)
    lin = (k[ok, 2] * dims[1] + k[ok, 1]) * dims[0] + k[ok, 0]
    cells, counts = np.unique(lin, return_counts=True)
    return cells[counts >= min_count]


def _nearest_f32(x):
    """The FP32 value nearest to the rational x (ties to the even significand): the
    answer is the FP32 rounding of float(x) or one of its two neighbours, compared
    exactly."""
    c0 = np.float32(float(x))
    cands = [np.nextafter(c0, np.float32(-np.inf)), c0, np.nextafter(c0, np.float32(np.inf))]
    return min(cands, key=lambda c: (abs(Fraction(float(c)) - x), int(np.float32(c).view(np.uint32)) & 1))


def voxel_centres(cells, voxel, lo, dims):
    """Centres [n, 3] (FP32) of the cells: lo + (k + 1/2) voxel of the exact values that
    the FP32 corner and voxel size denote, rounded once to FP32.  FP64 evaluates it
    with at most two roundings, which decide the FP32 value unless the FP64 result lies
    within a few FP64 ulps of a point halfway between two FP32 neighbours; those are
    redone with exact rationals (a round-to-FP64-then-FP32 there can break a tie the
    wrong way, e.g. when lo is far smaller than the offset)."""
    dims = np.asarray(dims, np.int64)
    k = np.stack([cells % dims[0], (cells // dims[0]) % dims[1], cells // (dims[0] * dims[1])], 1)
    lo32 = np.asarray(lo, np.float32)
    s32 = np.float32(voxel)
    v = lo32.astype(np.float64) + (k + 0.5) * np.float64(s32)
    c = v.astype(np.float32)
    c64 = c.astype(np.float64)
    with np.errstate(invalid="ignore", over="ignore"):
        up = np.nextafter(c, np.float32(np.inf)).astype(np.float64)
        dn = np.nextafter(c, np.float32(-np.inf)).astype(np.float64)
        tol = 4.0 * np.spacing(np.abs(v))
        amb = (np.abs(v - (c64 + up) / 2) <= tol) | (np.abs(v - (c64 + dn) / 2) <= tol)
    for i, a in zip(*np.nonzero(amb)):
        c[i, a] = _nearest_f32(Fraction(float(lo32[a])) + (int(k[i, a]) + Fraction(1, 2)) * Fraction(float(s32)))
    return c
