"""Property sweep on the GPU for the perception front end (Sec. IV-B): random depth
frames straight to voxel centres.

Each draw takes 0-3 frames of a random size (one pixel up to 640 x 480, so both the
one-pixel-per-thread and the four-pixel paths, single frames and multi-view batches),
random pinhole intrinsics (either sign of focal length, principal point anywhere
near the image), a random camera pose per frame, depths over 0.1-3 m with repeated
values and invalid pixels (zero, negative, NaN, +-inf), a random lattice covering part
of the cloud, min_count 1-3, an optional set of robot spheres and a capacity below,
at or above the cell count.  Checked:
  - gmapp_depth_to_points_batch against the oracle's FP64 back-projection: the same
    invalid pixels, every coordinate within 10 FP32 roundings of the sum of the
    magnitudes of its terms (three roundings of the camera coordinate, three of the
    fused multiply-adds of the pose);
  - the voxel pass on those FP32 points against the oracle's exact cells: the count,
    every centre bit for bit, nothing written past the capacity;
  - gmapp_depth_to_voxels (back-projection fused into the voxel pass) bit for bit
    against the two-kernel path."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import perception as op

pytestmark = pytest.mark.gpu

SETTINGS = dict(deadline=None, derandomize=True,
                suppress_health_check=[HealthCheck.function_scoped_fixture, HealthCheck.too_slow])


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2606_12579_amd import gmapp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = gmapp.Context(0)
    yield c
    c.close()


def _rotation(rng):
    q = rng.standard_normal(4)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _frames(rng, n_frames, w, h, bad_frac, levels):
    depth = rng.uniform(0.1, 3.0, (n_frames, h, w))
    if levels:                                     # planes: many pixels share a depth
        depth = np.round(depth * levels) / levels + 0.05
    n = depth.size
    if n:
        k = int(bad_frac * n)
        idx = rng.choice(n, k, replace=False)
        depth.reshape(-1)[idx] = rng.choice([0.0, -0.5, np.nan, np.inf, -np.inf], k)
    T = np.zeros((n_frames, 3, 4))
    for f in range(n_frames):
        T[f, :, :3] = _rotation(rng)
        T[f, :, 3] = rng.uniform(-1.0, 1.0, 3)
    return depth.astype(np.float32), T.astype(np.float32)


def _intrinsics(rng, w, h):
    fx, fy = rng.uniform(50.0, 1000.0, 2) * np.where(rng.uniform(size=2) < 0.1, -1.0, 1.0)
    return np.array([fx, fy, rng.uniform(-5.0, w + 5.0), rng.uniform(-5.0, h + 5.0)], np.float32)


def _lattice(rng, P, voxel):
    """A lattice over part of the finite points: corner inside or just outside their box, at most 300
    cells an axis (the voxel grows for wide clouds)."""
    fin = np.isfinite(P).all(1)
    if not fin.any():
        return np.float32(voxel), np.zeros(3, np.float32), rng.integers(1, 50, 3).astype(np.int32)
    lo_b, hi_b = P[fin].min(0), P[fin].max(0)
    ext = np.maximum(hi_b - lo_b, 1e-3)
    s = np.float32(max(voxel, float(ext.max()) / 256.0))
    lo = (lo_b + ext * rng.uniform(-0.1, 0.3, 3)).astype(np.float32)
    dims = np.clip(np.ceil(ext * rng.uniform(0.5, 1.1, 3) / float(s)), 1, 300).astype(np.int32)
    return s, lo, dims


SIZES = [(1, 1), (7, 5), (16, 9), (33, 17), (40, 40), (160, 120), (640, 480)]


@settings(max_examples=60, **SETTINGS)
@given(seed=st.integers(0, 2 ** 31 - 1), n_frames=st.integers(0, 3), size=st.sampled_from(SIZES),
       bad_frac=st.sampled_from([0.0, 0.05, 0.5, 1.0]), levels=st.sampled_from([0, 20]),
       voxel=st.sampled_from([0.005, 0.01, 0.05, 0.2]), min_count=st.integers(1, 3),
       n_spheres=st.sampled_from([-1, 0, 1, 4]), cap_frac=st.sampled_from([0.0, 0.5, 1.0, 2.0]))
def test_random_frames_to_voxels(ctx, seed, n_frames, size, bad_frac, levels, voxel, min_count, n_spheres,
                                 cap_frac):
    import torch
    w, h = size
    if w * h >= 160 * 120 and n_frames > 2:
        n_frames = 2
    rng = np.random.default_rng(seed)
    depth, T = _frames(rng, n_frames, w, h, bad_frac, levels)
    K = _intrinsics(rng, w, h)
    ref = np.concatenate([op.back_project(depth[f], K, T[f]) for f in range(n_frames)]) if n_frames \
        else np.zeros((0, 3))
    s, lo, dims = _lattice(rng, ref, voxel)
    spheres = None
    if n_spheres >= 0:
        fin = np.nonzero(np.isfinite(ref).all(1))[0]
        m = n_spheres if len(fin) else 0
        c = ref[rng.choice(fin, m)] if m else np.zeros((0, 3))
        spheres = np.concatenate([c, float(s) * rng.uniform(0.5, 5.0, (m, 1))], 1).astype(np.float32)
    print(f"seed {seed} frames {n_frames} size {w}x{h} bad {bad_frac} levels {levels} K {K.tolist()} "
          f"voxel {float(s)} lo {lo.tolist()} dims {dims.tolist()} min_count {min_count} "
          f"spheres {None if spheres is None else len(spheres)} cap_frac {cap_frac}", flush=True)
    d = torch.as_tensor(depth, device="cuda")
    Td = torch.as_tensor(T, device="cuda")
    Rd = None if spheres is None else torch.as_tensor(spheres, device="cuda")
    x, y, z = ctx.depth_to_points_batch(d, K, Td)
    torch.cuda.synchronize()
    got = np.stack([x.cpu().numpy(), y.cpu().numpy(), z.cpu().numpy()], 1)

    # back-projection: bound from the magnitudes of the terms of each coordinate
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref[:, 0])
    if ok.any():
        fx, fy, cx, cy = (float(v) for v in K)
        dd = np.concatenate([depth[f].astype(np.float64).reshape(-1) for f in range(n_frames)])
        u = np.tile(np.tile(np.arange(w, dtype=np.float64), h), n_frames)
        v = np.tile(np.repeat(np.arange(h, dtype=np.float64), w), n_frames)
        Xc = np.stack([(u - cx) * dd / fx, (v - cy) * dd / fy, dd], 1)
        Tf = np.repeat(T.astype(np.float64), w * h, axis=0)
        mag = np.abs(Tf[:, :, :3] * Xc[:, None, :]).sum(2) + np.abs(Tf[:, :, 3])
        err = np.abs(got[ok].astype(np.float64) - ref[ok])
        bound = 10.0 * 2.0 ** -24 * mag[ok] + 1e-30
        assert (err <= bound).all(), float((err / bound).max())

    # the voxel pass on the device's points against the exact cells of those points
    cells = op.voxel_cells(got[:, 0], got[:, 1], got[:, 2], s, lo, dims, min_count, spheres)
    cap = int(len(cells) * cap_frac)
    k = min(cap, len(cells))
    C = op.voxel_centres(cells[:k], s, lo, dims).astype(np.float32)
    res = []
    for fused in (False, True):
        buf = [torch.full((cap + 8,), -7.0, dtype=torch.float32, device="cuda") for _ in range(3)]
        m = torch.zeros(1, dtype=torch.int64, device="cuda")
        out = (buf[0][:cap], buf[1][:cap], buf[2][:cap], m)
        if fused:
            ctx.depth_to_voxels(d, K, Td, s, lo, dims, min_count=min_count, capacity=cap, out=out, robot_spheres=Rd)
        else:
            ctx.voxel_downsample(x, y, z, s, lo, dims, min_count=min_count, capacity=cap, out=out, robot_spheres=Rd)
        torch.cuda.synchronize()
        assert int(m.item()) == len(cells), (fused, int(m.item()), len(cells))
        G = np.stack([buf[a][:k].cpu().numpy() for a in range(3)], 1)
        assert np.array_equal(G, C), fused
        for a in range(3):
            assert (buf[a][k:].cpu().numpy() == -7.0).all(), fused
        res.append(G)
    assert np.array_equal(res[0], res[1])
    print(f"  points {int(ok.sum())} of {len(ref)} valid, cells {len(cells)}, capacity {cap}", flush=True)
