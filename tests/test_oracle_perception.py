"""Pins of the perception oracle: projection round trip, brute-force voxel sets,
geometric properties of voxel centres, idempotence."""
import math
from fractions import Fraction

import numpy as np

from oracle import perception as op
from paper_2606_12579_amd import scenes


def test_back_projection_round_trip():
    """Project known world points with the pinhole model, back-project their depth: same points."""
    rng = np.random.default_rng(0)
    fr = scenes.config3_frame(n_boxes=0, w=64, h=48)
    K = fr.K.astype(np.float64)
    T = fr.T_wc.astype(np.float64)
    R, t = T[:, :3], T[:, 3]
    # world points in front of the camera
    Pw = np.stack([rng.uniform(-0.03, 0.03, 200), rng.uniform(-0.02, 0.02, 200), rng.uniform(0.0, 0.5, 200)], 1)
    Pc = (Pw - t) @ R                                # R^T (p - t)
    u = K[0] * Pc[:, 0] / Pc[:, 2] + K[2]
    v = K[1] * Pc[:, 1] / Pc[:, 2] + K[3]
    # an image holding exactly these depths at integer pixels: use pixel centres instead
    ui, vi = np.round(u).astype(int), np.round(v).astype(int)
    keep = (ui >= 0) & (ui < 64) & (vi >= 0) & (vi < 48)
    _, first = np.unique(vi * 64 + ui, return_index=True)      # one world point per pixel
    keep &= np.isin(np.arange(len(ui)), first)
    assert keep.sum() > 20
    depth = np.zeros((48, 64))
    depth[vi[keep], ui[keep]] = Pc[keep, 2]
    P = op.back_project(depth, fr.K, fr.T_wc).reshape(48, 64, 3)
    # the back-projected pixel centre lies on the ray through that pixel at the given depth
    for j in np.flatnonzero(keep):
        p = P[vi[j], ui[j]]
        pc = (p - t) @ R
        assert abs(pc[2] - Pc[j, 2]) < 1e-12
        assert abs(K[0] * pc[0] / pc[2] + K[2] - ui[j]) < 1e-9
        assert abs(K[1] * pc[1] / pc[2] + K[3] - vi[j]) < 1e-9


def test_back_projection_plane_and_invalid():
    fr = scenes.config3_frame(n_boxes=0, w=32, h=24)
    P = op.back_project(fr.depth, fr.K, fr.T_wc)
    assert np.abs(P[:, 2]).max() < 1e-6                     # camera 1 m above the plane z = 0
    d = fr.depth.copy()
    d[0, 0], d[1, 1], d[2, 2] = 0.0, np.nan, -1.0
    P = op.back_project(d, fr.K, fr.T_wc)
    assert np.isnan(P[[0, 32 + 1, 64 + 2]]).all() and np.isfinite(P[3]).all()


def _as_int(v, scale=1100):
    """A float (FP32 or FP64) as the integer v * 2^scale, exactly (integer mantissa and
    exponent from frexp; every finite float is an integer multiple of 2^-1074)."""
    m, e = math.frexp(float(v))
    mi = int(m * (1 << 53))                      # exact: m has at most 53 significant bits
    sh = e - 53 + scale
    return mi << sh if sh >= 0 else -((-mi) >> -sh) if mi < 0 else mi >> -sh


def _int_floor(p, lo, s):
    """floor((p - lo) / s) in integer arithmetic on the scaled values (Python // floors)."""
    return (_as_int(p) - _as_int(lo)) // _as_int(s)


def _face_points(lo, s, ks):
    """FP32 coordinates at and around the faces lo + k s of a lattice: for each k the
    FP32 values nearest the real face and 1 and 2 steps either side, each with the
    cell that the position relative to the face fixes: k when at or above it, k - 1
    below it (decided by an integer comparison of the scaled values)."""
    lo, s = np.float32(lo), np.float32(s)
    pts, want = [], []
    for k in ks:
        face = _as_int(lo) + k * _as_int(s)
        c = np.float32(float(lo) + k * float(s))
        for step in (-2, -1, 0, 1, 2):
            p = c
            for _ in range(abs(step)):
                p = np.nextafter(p, np.float32(np.inf if step > 0 else -np.inf))
            pts.append(p)
            want.append(k if _as_int(p) >= face else k - 1)
    return np.array(pts, np.float32), np.array(want)


def test_voxel_keys_exact_at_faces():
    """Cells of FP32 coordinates on and one or two FP32 steps either side of lattice
    faces: a dyadic lattice (faces representable, points exactly on them) and the
    config-3 lattice of 1 cm cells (faces between FP32 values).  The oracle's key is
    the cell that the point's side of the face fixes; an FP32 quotient, floor(fl32(
    fl32(p - lo) / s)), misplaces some of these points, so the check can tell them apart."""
    fr = scenes.config3_frame(n_boxes=0, w=8, h=6)
    lattices = [(-0.5, 2.0 ** -6, 64), (fr.box_lo[0], fr.voxel, fr.dims[0]), (fr.box_lo[2], fr.voxel, fr.dims[2]),
                (0.0, fr.voxel, 100), (-0.0125, 0.003, 300)]
    fp32_wrong = 0
    for lo, s, dim in lattices:
        p, want = _face_points(lo, s, range(0, dim, 1))
        z = np.zeros_like(p)
        k, ok = op.voxel_keys(p, z, z, s, [lo, -1.0, -1.0], [dim + 1, 1 << 20, 1 << 20])
        inside = want >= 0
        assert np.array_equal(ok, inside)
        assert np.array_equal(k[inside, 0], want[inside]), (lo, s)
        # integer arithmetic agrees as well (a second exact route)
        assert all(_int_floor(a, np.float32(lo), np.float32(s)) == b for a, b in zip(p, want))
        q32 = np.floor((p - np.float32(lo)) / np.float32(s)).astype(np.int64)
        fp32_wrong += int((q32 != want).sum())
    assert fp32_wrong > 0


def test_voxel_keys_far_and_non_finite():
    """Coordinates whose quotient lies far outside any grid (|q| >= 2^52), infinities and
    NaN are outside the box; a point next to them still gets its cell."""
    P = np.array([1e30, -1e30, 3e38, np.inf, -np.inf, np.nan, 0.015], np.float32)
    z = np.zeros_like(P)
    k, ok = op.voxel_keys(P, z, z, np.float32(0.01), [0.0, -1.0, -1.0], [10, 1000, 1000])
    assert ok.tolist() == [False] * 6 + [True] and k[6, 0] == 1


def test_voxel_bruteforce_small():
    """Random FP32 points (and points pushed onto faces) against an integer-arithmetic
    brute force of floor((p - lo) / s) per axis."""
    rng = np.random.default_rng(1)
    s, lo, dims = np.float32(0.01), np.array([-0.05, -0.05, 0.0], np.float32), np.array([10, 10, 5])
    P = rng.uniform([-0.06, -0.06, -0.01], [0.06, 0.06, 0.06], (500, 3)).astype(np.float32)
    P[:40, 0] = [np.float32(float(lo[0]) + k * float(s)) for k in range(40)]     # nearest FP32 to faces
    cells = op.voxel_cells(P[:, 0], P[:, 1], P[:, 2], s, lo, dims)
    expect = set()
    for p in P:
        k = [_int_floor(p[a], lo[a], s) for a in range(3)]
        if all(0 <= k[a] < dims[a] for a in range(3)):
            expect.add((k[2] * dims[1] + k[1]) * dims[0] + k[0])
    assert list(cells) == sorted(expect)
    # min_count keeps exactly the cells with enough points
    k, ok = op.voxel_keys(P[:, 0], P[:, 1], P[:, 2], s, lo, dims)
    lin = (k[ok, 2] * dims[1] + k[ok, 1]) * dims[0] + k[ok, 0]
    for m in (2, 3):
        c2 = op.voxel_cells(P[:, 0], P[:, 1], P[:, 2], s, lo, dims, min_count=m)
        assert all((lin == c).sum() >= m for c in c2)
        assert all((lin == c).sum() < m for c in set(lin) - set(c2))


def _round_f32_by_integers(x):
    """Round the positive rational x to FP32 by integer arithmetic: scale it to a 24-bit
    significand, round half to even with an integer division (normal range only)."""
    e = x.numerator.bit_length() - x.denominator.bit_length()
    while Fraction(2) ** e > x:
        e -= 1
    while Fraction(2) ** (e + 1) <= x:
        e += 1
    q = x / Fraction(2) ** (e - 23)                 # in [2^23, 2^24)
    m, r = divmod(q.numerator, q.denominator)
    if 2 * r > q.denominator or (2 * r == q.denominator and m % 2 == 1):
        m += 1
    return np.float32(float(Fraction(m) * Fraction(2) ** (e - 23)))


def test_voxel_centres_rounded_once():
    """Centres are lo + (k + 1/2) s of the exact values rounded once to FP32.  With lo the
    smallest normal FP32 number and s = 0.001f, 1.5 s is an exact tie between two FP32
    neighbours, and the tiny lo breaks it upward; a sum rounded to FP64 first loses lo
    and ties to even instead.  A brute force over random corners, voxel sizes and cells
    (integer-arithmetic rounding of the exact rational) must agree everywhere."""
    s = np.float32(0.001)
    tiny = np.float32(np.finfo(np.float32).tiny)
    P = Fraction(3, 2) * Fraction(float(s))
    below = np.float32(float(P))                   # P lies exactly halfway between two FP32 values
    lo_n, hi_n = (np.nextafter(below, np.float32(-np.inf)), below) if Fraction(float(below)) > P else \
        (below, np.nextafter(below, np.float32(np.inf)))
    assert Fraction(float(lo_n)) + Fraction(float(hi_n)) == 2 * P
    c = op.voxel_centres(np.array([1 * 1]), s, [0.0, tiny, 0.0], [1, 2, 1])     # cell (0, 1, 0)
    assert c[0, 1] == hi_n and c[0, 1] == _round_f32_by_integers(P + Fraction(float(tiny)))
    rng = np.random.default_rng(5)
    for _ in range(400):
        s = np.float32(rng.choice([0.001, 0.003, 0.01, 0.25, 1e-5]) * rng.uniform(0.5, 2.0))
        lo = np.array([rng.choice([0.0, float(tiny), 1e-30, rng.uniform(-2, 2)]) for _ in range(3)], np.float32)
        lo = np.abs(lo)                              # positive centres for the integer rounding
        dims = rng.integers(1, 5000, 3)
        cells = rng.integers(0, int(np.prod(dims)), 4)
        C = op.voxel_centres(cells, s, lo, dims)
        k = np.stack([cells % dims[0], (cells // dims[0]) % dims[1], cells // (dims[0] * dims[1])], 1)
        for i in range(len(cells)):
            for a in range(3):
                x = Fraction(float(lo[a])) + (int(k[i, a]) + Fraction(1, 2)) * Fraction(float(s))
                assert C[i, a] == _round_f32_by_integers(x), (float(s), lo, k[i], a)


def test_voxel_centre_properties_and_idempotence():
    fr = scenes.config3_frame()
    P = op.back_project(fr.depth, fr.K, fr.T_wc).astype(np.float32)
    cells = op.voxel_cells(P[:, 0], P[:, 1], P[:, 2], fr.voxel, fr.box_lo, fr.dims)
    C = op.voxel_centres(cells, fr.voxel, fr.box_lo, fr.dims)
    assert 0 < len(cells) <= len(P)
    # every kept point lies in its cell: within sqrt(3) s / 2 of the centre
    k, ok = op.voxel_keys(P[:, 0], P[:, 1], P[:, 2], fr.voxel, fr.box_lo, fr.dims)
    d = np.asarray(fr.dims, np.int64)
    lin = (k[ok, 2] * d[1] + k[ok, 1]) * d[0] + k[ok, 0]
    centre = C[np.searchsorted(cells, lin)]
    assert (np.linalg.norm(P[ok].astype(np.float64) - centre, axis=1) <= math.sqrt(3) * fr.voxel / 2 * (1 + 1e-5)).all()
    # re-voxelising the centres gives the same cells
    C32 = C.astype(np.float32)
    again = op.voxel_cells(C32[:, 0], C32[:, 1], C32[:, 2], fr.voxel, fr.box_lo, fr.dims)
    assert np.array_equal(again, cells)
    # the scene really has boxes above the plane and the plane fills the footprint
    assert len(cells) > 11000 and (C[:, 2] > 0.03).sum() > 500


def test_robot_self_filter():
    """Points within the robot's bounding spheres are removed: exact boundary cases
    (|p - c| = r is removed, one FP32 step further out is kept) and, away from the
    boundaries, a k-d tree query of the sphere centres."""
    from scipy.spatial import cKDTree
    S = np.array([[0.0, 0.0, 0.0, 0.5], [1.0, 1.0, 1.0, 0.25]], np.float32)
    x = np.array([0.5, np.nextafter(np.float32(0.5), np.float32(1)), 1.0, 1.25, 0.0, 2.0], np.float32)
    y = np.array([0.0, 0.0, 1.0, 1.0, -0.5, 2.0], np.float32)
    z = np.array([0.0, 0.0, 1.25, 1.0, 0.0, 2.0], np.float32)
    assert op.on_robot(x, y, z, S).tolist() == [True, False, True, True, True, False]
    rng = np.random.default_rng(5)
    R = scenes.robot_spheres(rng)
    P = rng.uniform(-0.5, 0.5, (20000, 3)).astype(np.float32)
    hit = op.on_robot(P[:, 0], P[:, 1], P[:, 2], R)
    tree = cKDTree(P.astype(np.float64))
    want = np.zeros(len(P), bool)
    far = np.ones(len(P), bool)
    for c in R.astype(np.float64):
        want[tree.query_ball_point(c[:3], c[3])] = True
        d = np.linalg.norm(P.astype(np.float64) - c[:3], axis=1)
        far &= np.abs(d - c[3]) > 1e-6
    assert 0 < hit.sum() < len(P)
    assert np.array_equal(hit[far], want[far])
    cells = op.voxel_cells(P[:, 0], P[:, 1], P[:, 2], 0.01, np.full(3, -0.5, np.float32), [100, 100, 100], 1, R)
    keep = ~hit
    ref = op.voxel_cells(P[keep, 0], P[keep, 1], P[keep, 2], 0.01, np.full(3, -0.5, np.float32), [100, 100, 100])
    assert np.array_equal(cells, ref)
