"""GPU parity of the perception pass (gmapp_depth_to_points, gmapp_voxel_downsample)
against the oracle, and the rollout on the device-resident sphere world."""
import copy

import numpy as np
import pytest

import oracle
from oracle import perception as op
from paper_2606_12579_amd import scenes
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2606_12579_amd import gmapp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = gmapp.Context(0)
    yield c
    c.close()


def _gpu_points(ctx, fr):
    import torch
    d = torch.as_tensor(fr.depth, device="cuda")
    x, y, z = ctx.depth_to_points(d, fr.K, fr.T_wc)
    torch.cuda.synchronize()
    return np.stack([x.cpu().numpy(), y.cpu().numpy(), z.cpu().numpy()], 1)


def test_depth_to_points(ctx):
    fr = scenes.config3_frame()
    fr.depth[0, :7] = [0.0, -1.0, np.nan, np.inf, 1.0, 0.5, 2.0]      # invalid pixels, then valid ones
    ref = op.back_project(fr.depth, fr.K, fr.T_wc)
    got = _gpu_points(ctx, fr).astype(np.float64)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref[:, 0])
    err = np.abs(got[ok] - ref[ok])
    assert (err <= 4e-7 * np.abs(ref[ok]) + 2e-7).all(), err.max()


def test_depth_to_points_batch(ctx):
    """Several frames with their own poses in one launch, against the oracle's
    back-projection of each frame: the vectorised path (w h divisible by 4) and the
    one-pixel-per-thread path (a ragged 7 x 5 image)."""
    import torch
    fr = scenes.config3_frame()
    T = scenes.config3_poses(3)
    for depth in (np.stack([fr.depth, fr.depth * np.float32(1.01), fr.depth]),
                  np.stack([fr.depth[:5, :7], fr.depth[10:15, 20:27], fr.depth[30:35, 40:47]])):
        depth = np.ascontiguousarray(depth)
        depth[1, 0, :5] = [0.0, -1.0, np.nan, np.inf, 0.7]                # invalid pixels
        ref = np.concatenate([op.back_project(depth[f], fr.K, T[f]) for f in range(3)])
        x, y, z = ctx.depth_to_points_batch(torch.as_tensor(depth, device="cuda"), fr.K,
                                            torch.as_tensor(T, device="cuda"))
        torch.cuda.synchronize()
        got = np.stack([x.cpu().numpy(), y.cpu().numpy(), z.cpu().numpy()], 1).astype(np.float64)
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        ok = ~np.isnan(ref[:, 0])
        err = np.abs(got[ok] - ref[ok])
        assert (err <= 4e-7 * np.abs(ref[ok]) + 2e-7).all(), err.max()


def test_fused_voxels_multiview(ctx):
    """The voxel pass over the points of 4 frames (multi-view fusion) gives exactly
    the oracle's occupied cells of the concatenated FP32 points."""
    import torch
    fr = scenes.config3_frame()
    T = scenes.config3_poses(4)
    P = np.concatenate([op.back_project(fr.depth, fr.K, T[f]) for f in range(4)]).astype(np.float32)
    cells = op.voxel_cells(P[:, 0], P[:, 1], P[:, 2], fr.voxel, fr.box_lo, fr.dims, 2)
    C = op.voxel_centres(cells, fr.voxel, fr.box_lo, fr.dims).astype(np.float32)
    t = [torch.as_tensor(np.ascontiguousarray(P[:, a]), device="cuda") for a in range(3)]
    ox, oy, oz, n = ctx.voxel_downsample(*t, fr.voxel, fr.box_lo, fr.dims, min_count=2, capacity=65536)
    torch.cuda.synchronize()
    n = int(n.item())
    assert n == len(cells)
    G = np.stack([ox[:n].cpu().numpy(), oy[:n].cpu().numpy(), oz[:n].cpu().numpy()], 1)
    assert np.array_equal(G, C)


def test_voxel_pass_in_a_captured_graph(ctx):
    """Fused depth-to-voxel passes captured in a HIP graph: every replay (with eager passes on
    other frames and host synchronisations in between) gives the eager result bit for bit,
    for min_count 1 and 2 (the grid each pass leaves zeroed is what the next one needs)."""
    import torch
    fr = scenes.config3_frame()
    T = torch.as_tensor(scenes.config3_poses(3), device="cuda")
    d = torch.as_tensor(fr.depth, device="cuda")
    frames = [d.unsqueeze(0).contiguous(), torch.flip(d, [1]).unsqueeze(0).contiguous()]
    cap = 65536
    for min_count in (1, 2):
        want = []
        for f in frames:
            o = ctx.depth_to_voxels(f, fr.K, T[:1], fr.voxel, fr.box_lo, fr.dims, min_count=min_count, capacity=cap)
            torch.cuda.synchronize()
            want.append([x.clone() for x in o])
        outs = [tuple(torch.empty(cap, dtype=torch.float32, device="cuda") for _ in range(3)) +
                (torch.zeros(1, dtype=torch.int64, device="cuda"),) for _ in frames]
        gs = torch.cuda.Stream()
        gs.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=gs):
            for f, o in zip(frames, outs):
                ctx.depth_to_voxels(f, fr.K, T[:1], fr.voxel, fr.box_lo, fr.dims, min_count=min_count,
                                    capacity=cap, out=o)
        torch.cuda.synchronize()
        for rep in range(4):
            for o in outs:
                for x in o:
                    x.fill_(-1)
            g.replay()
            torch.cuda.synchronize()
            for o, w in zip(outs, want):
                n = int(w[3].item())
                assert int(o[3].item()) == n, (min_count, rep)
                for a in range(3):
                    assert torch.equal(o[a][:n], w[a][:n]), (min_count, rep, a)
            # eager passes between replays, on other frames and the other min_count
            ctx.depth_to_voxels(frames[rep % 2], fr.K, T[1:2], fr.voxel, fr.box_lo, fr.dims,
                                min_count=3 - min_count, capacity=cap)
            torch.cuda.synchronize()
        del g


def test_voxel_exact_on_oracle_points(ctx):
    """Same FP32 points on both sides: identical occupied cells, centres = FP32 rounding of the exact centres."""
    import torch
    fr = scenes.config3_frame()
    P = op.back_project(fr.depth, fr.K, fr.T_wc).astype(np.float32)
    for min_count in (1, 3):
        cells = op.voxel_cells(P[:, 0], P[:, 1], P[:, 2], fr.voxel, fr.box_lo, fr.dims, min_count)
        C = op.voxel_centres(cells, fr.voxel, fr.box_lo, fr.dims).astype(np.float32)
        t = [torch.as_tensor(np.ascontiguousarray(P[:, a]), device="cuda") for a in range(3)]
        ox, oy, oz, n = ctx.voxel_downsample(*t, fr.voxel, fr.box_lo, fr.dims, min_count=min_count)
        torch.cuda.synchronize()
        n = int(n.item())
        assert n == len(cells), (n, len(cells))
        G = np.stack([ox[:n].cpu().numpy(), oy[:n].cpu().numpy(), oz[:n].cpu().numpy()], 1)
        assert np.array_equal(G, C)


def _face_points(lo, s, ks):
    """FP32 coordinates on and 1-2 FP32 steps either side of the lattice faces lo + k s."""
    lo, s = np.float32(lo), np.float32(s)
    out = []
    for k in ks:
        c = np.float32(float(lo) + k * float(s))
        for step in (-2, -1, 0, 1, 2):
            p = c
            for _ in range(abs(step)):
                p = np.nextafter(p, np.float32(np.inf if step > 0 else -np.inf))
            out.append(p)
    return np.array(out, np.float32)


def test_voxel_exact_at_faces(ctx):
    """Points on and one or two FP32 steps either side of the faces of the config-3
    lattice (1 cm cells from a corner that is not a multiple of the voxel) and of a
    dyadic lattice (faces representable): the kernel's cells are the exact lattice
    cells of the oracle, bit for bit, for min_count 1 (occupancy bytes) and 2 (counts).  An
    FP32 quotient misplaces some of these points, so agreement is not a shared rounding."""
    import torch
    fr = scenes.config3_frame()
    rng = np.random.default_rng(23)
    for lo, s, dims in ((fr.box_lo, fr.voxel, fr.dims), (np.array([-0.5, -0.25, 0.0], np.float32), 2.0 ** -6,
                                                        np.array([64, 40, 24], np.int32))):
        lo = np.asarray(lo, np.float32)
        axes = [_face_points(lo[a], s, range(-1, int(dims[a]) + 2)) for a in range(3)]
        m = max(len(v) for v in axes)
        P = np.stack([rng.choice(axes[a], 4 * m) for a in range(3)], 1).astype(np.float32)
        P = np.concatenate([P, P[: len(P) // 2]])            # half the cells hold two points or more
        q32 = np.floor((P - lo) / np.float32(s))
        k_ex, ok = op.voxel_keys(P[:, 0], P[:, 1], P[:, 2], s, lo, dims)
        assert (q32[ok] != k_ex[ok]).any()
        t = [torch.as_tensor(np.ascontiguousarray(P[:, a]), device="cuda") for a in range(3)]
        for min_count in (1, 2):
            cells = op.voxel_cells(P[:, 0], P[:, 1], P[:, 2], s, lo, dims, min_count)
            ox, oy, oz, n = ctx.voxel_downsample(*t, s, lo, dims, min_count=min_count, capacity=len(P))
            torch.cuda.synchronize()
            n = int(n.item())
            assert n == len(cells), (min_count, n, len(cells))
            G = np.stack([ox[:n].cpu().numpy(), oy[:n].cpu().numpy(), oz[:n].cpu().numpy()], 1)
            assert np.array_equal(G, op.voxel_centres(cells, s, lo, dims).astype(np.float32))


def test_voxel_large_grid_paths(ctx):
    """Grids of more than 1024 blocks of 1024 cells take the multi-kernel finish (per-block
    counts, their scan, then the centres): a 1024 x 1024 x 2 lattice with points in a band
    across it, ragged point counts, min_count 1 and 3, and a capacity below the count."""
    import torch
    rng = np.random.default_rng(29)
    lo, s, dims = np.array([0.0, 0.0, 0.0], np.float32), np.float32(0.001), np.array([1024, 1024, 2], np.int32)
    for n in (1, 300001, 1 << 20):
        P = np.stack([rng.uniform(-0.01, 1.03, n), rng.uniform(0.2, 0.21, n) * rng.integers(1, 5, n),
                      rng.uniform(0.0, 0.0021, n)], 1).astype(np.float32)
        P[: n // 3, 0] = rng.choice(_face_points(lo[0], s, range(0, 1024, 7)), n // 3)
        t = [torch.as_tensor(np.ascontiguousarray(P[:, a]), device="cuda") for a in range(3)]
        for min_count in (1, 3):
            cells = op.voxel_cells(P[:, 0], P[:, 1], P[:, 2], s, lo, dims, min_count)
            for cap in (len(cells), max(len(cells) // 2, 1)):
                ox, oy, oz, m = ctx.voxel_downsample(*t, s, lo, dims, min_count=min_count, capacity=cap)
                torch.cuda.synchronize()
                assert int(m.item()) == len(cells), (n, min_count, int(m.item()), len(cells))
                k = min(cap, len(cells))
                C = op.voxel_centres(cells[:k], s, lo, dims).astype(np.float32)
                G = np.stack([ox[:k].cpu().numpy(), oy[:k].cpu().numpy(), oz[:k].cpu().numpy()], 1)
                assert np.array_equal(G, C), (n, min_count, cap)


def test_voxel_finish_across_block_counts(ctx):
    """Consecutive passes over grids of 1, 2, 3, 517, 1024 and 1025 blocks of 1024 cells,
    in an order that alternates the finish whose blocks add their predecessors' counts
    themselves (up to 1024 blocks) with the one that scans the counts first, min_count 1
    and 2: every pass gives the oracle's cells, on the grid and dirty bytes the passes
    before it left cleared."""
    import torch
    rng = np.random.default_rng(41)
    lo, s = np.array([0.0, 0.0, 0.0], np.float32), np.float32(0.001)
    seq = [1, 3, 1024, 1025, 517, 1, 1024, 2, 1025, 1024, 3, 517, 1]
    for i, nb in enumerate(seq):
        dims = np.array([1024, nb, 1], np.int32)
        n = int(rng.integers(1, 40000))
        P = np.stack([rng.uniform(-0.01, 1.03, n), rng.uniform(0.0, nb * 0.001, n) * rng.uniform(0.0, 1.0, n) ** 2,
                      rng.uniform(-0.0002, 0.0011, n)], 1).astype(np.float32)
        t = [torch.as_tensor(np.ascontiguousarray(P[:, a]), device="cuda") for a in range(3)]
        min_count = 1 + (i % 2)
        cells = op.voxel_cells(P[:, 0], P[:, 1], P[:, 2], s, lo, dims, min_count)
        ox, oy, oz, m = ctx.voxel_downsample(*t, s, lo, dims, min_count=min_count, capacity=len(cells) + 1)
        torch.cuda.synchronize()
        assert int(m.item()) == len(cells), (i, nb, n, min_count, int(m.item()), len(cells))
        C = op.voxel_centres(cells, s, lo, dims).astype(np.float32)
        G = np.stack([ox[:len(cells)].cpu().numpy(), oy[:len(cells)].cpu().numpy(), oz[:len(cells)].cpu().numpy()], 1)
        assert np.array_equal(G, C), (i, nb, n, min_count)


def _fused_vs_two_kernel(ctx, depth, K, T, fr, min_count=1, spheres=None, capacity=65536):
    """gmapp_depth_to_voxels against gmapp_depth_to_points_batch + the voxel pass: identical counts
    and centres (the same FP32 points, the same exact cells)."""
    import torch
    d = torch.as_tensor(np.ascontiguousarray(depth), device="cuda")
    Td = torch.as_tensor(np.ascontiguousarray(T), device="cuda")
    Rd = None if spheres is None else torch.as_tensor(spheres, device="cuda")
    x, y, z = ctx.depth_to_points_batch(d, K, Td)
    a = ctx.voxel_downsample(x, y, z, fr.voxel, fr.box_lo, fr.dims, min_count=min_count, capacity=capacity,
                             robot_spheres=Rd)
    b = ctx.depth_to_voxels(d, K, Td, fr.voxel, fr.box_lo, fr.dims, min_count=min_count, capacity=capacity,
                            robot_spheres=Rd)
    torch.cuda.synchronize()
    n = int(a[3].item())
    assert int(b[3].item()) == n
    k = min(n, capacity)
    for i in range(3):
        assert torch.equal(a[i][:k], b[i][:k])
    return n


def test_depth_to_voxels_equals_two_kernel_path(ctx):
    """The fused pass against back-projection + voxel pass, bit for bit: the config-3 frame,
    four frames from four poses (multi-view fusion), ragged 7 x 5 frames (one pixel per
    thread), invalid pixels, min_count 1 and 2, the robot self-filter, a capacity below
    the count, and no frames at all."""
    fr = scenes.config3_frame()
    T = scenes.config3_poses(4)
    R = scenes.robot_spheres(np.random.default_rng(9), base=(-0.3, -0.05, 0.0), tip=(0.2, 0.1, 0.3))
    one = fr.depth[None].copy()
    one[0, 0, :5] = [0.0, -1.0, np.nan, np.inf, 0.7]
    four = np.stack([fr.depth, fr.depth * np.float32(1.01), fr.depth, fr.depth * np.float32(0.98)])
    rag = np.ascontiguousarray(np.stack([fr.depth[:5, :7], fr.depth[100:105, 300:307], fr.depth[30:35, 40:47]]))
    n1 = _fused_vs_two_kernel(ctx, one, fr.K, T[:1], fr)
    assert n1 > 1000
    for mc in (1, 2):
        _fused_vs_two_kernel(ctx, four, fr.K, T, fr, min_count=mc)
        _fused_vs_two_kernel(ctx, four, fr.K, T, fr, min_count=mc, spheres=R)
    _fused_vs_two_kernel(ctx, rag, fr.K, T[:3], fr)
    _fused_vs_two_kernel(ctx, four, fr.K, T, fr, capacity=100)
    _fused_vs_two_kernel(ctx, np.zeros((0, 480, 640), np.float32), fr.K, T[:0], fr, capacity=4)


def test_depth_to_voxels_vs_oracle(ctx):
    """Depth image -> voxel centres in one pass against the oracle's pipeline (FP64
    back-projection, exact lattice cells): the cells agree except where an oracle
    point lies within 1e-5 voxel of a face (FP32 and FP64 points may straddle it);
    those points are counted and bound the difference."""
    import torch
    fr = scenes.config3_frame()
    ref_P = op.back_project(fr.depth, fr.K, fr.T_wc)
    ref = set(op.voxel_cells(ref_P[:, 0], ref_P[:, 1], ref_P[:, 2], fr.voxel, fr.box_lo, fr.dims))
    d = torch.as_tensor(fr.depth[None].copy(), device="cuda")
    Td = torch.as_tensor(fr.T_wc[None].copy(), device="cuda")
    ox, oy, oz, n = ctx.depth_to_voxels(d, fr.K, Td, fr.voxel, fr.box_lo, fr.dims, capacity=65536)
    torch.cuda.synchronize()
    nv = int(n.item())
    G = np.stack([ox[:nv].cpu().numpy(), oy[:nv].cpu().numpy(), oz[:nv].cpu().numpy()], 1).astype(np.float64)
    g_cells = np.round((G - fr.box_lo.astype(np.float64)) / fr.voxel - 0.5).astype(np.int64)
    dims = fr.dims.astype(np.int64)
    g_lin = (g_cells[:, 2] * dims[1] + g_cells[:, 1]) * dims[0] + g_cells[:, 0]
    assert np.all(np.diff(g_lin) > 0)
    q = (ref_P - fr.box_lo.astype(np.float64)) / np.float64(np.float32(fr.voxel))
    near = np.isfinite(q).all(1) & (np.abs(q - np.round(q)) < 1e-5).any(1)
    k, ok = op.voxel_keys(ref_P[:, 0], ref_P[:, 1], ref_P[:, 2], fr.voxel, fr.box_lo, fr.dims)
    sure = set(((k[:, 2] * dims[1] + k[:, 1]) * dims[0] + k[:, 0])[ok & ~near])
    assert sure <= set(g_lin)
    diff = ref ^ set(g_lin)
    assert len(diff) <= 2 * near.sum(), (len(diff), near.sum())
    print(f"fused depth->voxels: gpu {nv}, oracle {len(ref)}, differing cells {len(diff)}, "
          f"points within 1e-5 voxel of a face {near.sum()}", flush=True)


def test_voxel_edges(ctx):
    import torch
    rng = np.random.default_rng(3)
    lo, dims, s = np.array([0.0, 0.0, 0.0], np.float32), np.array([7, 5, 3], np.int32), 0.01
    P = rng.uniform(-0.02, 0.09, (3000, 3)).astype(np.float32)      # many outside the box
    P[:5] = np.nan
    cells = op.voxel_cells(P[:, 0], P[:, 1], P[:, 2], s, lo, dims)
    t = [torch.as_tensor(np.ascontiguousarray(P[:, a]), device="cuda") for a in range(3)]
    for cap in (len(cells), 10, 0):                                   # capacity overflow keeps the count
        ox, oy, oz, n = ctx.voxel_downsample(*t, s, lo, dims, capacity=cap)
        torch.cuda.synchronize()
        assert int(n.item()) == len(cells)
        C = op.voxel_centres(cells[:cap], s, lo, dims).astype(np.float32)
        if cap:
            assert np.array_equal(ox[:cap].cpu().numpy(), C[:, 0])
    e = [torch.empty(0, device="cuda") for _ in range(3)]
    ox, oy, oz, n = ctx.voxel_downsample(*e, s, lo, dims, capacity=4)
    torch.cuda.synchronize()
    assert int(n.item()) == 0
    # an axis longer than 2^23 cells is refused (k + 1/2 would not be exact in FP32)
    from paper_2606_12579_amd import gmapp
    with pytest.raises(gmapp.GmappError) as ei:
        ctx.voxel_downsample(*t, s, lo, np.array([(1 << 23) + 1, 1, 1], np.int32), capacity=4)
    assert ei.value.status == gmapp.ECAPACITY
    ox, oy, oz, n = ctx.voxel_downsample(*e, s, lo, np.array([1 << 23, 1, 1], np.int32), capacity=4)
    torch.cuda.synchronize()
    assert int(n.item()) == 0


def test_voxel_ragged_and_unaligned(ctx):
    """Above about 2^19 points (two waves per SIMD of four-point threads) the marking pass
    takes four points per thread from 16-byte loads when x, y, z are 16-byte aligned and
    hands the last n mod 4 points to single threads; shorter or unaligned inputs take the
    one-point path.  Every length and alignment gives the oracle's cells."""
    import torch
    rng = np.random.default_rng(17)
    lo, dims, s = np.array([0.0, 0.0, 0.0], np.float32), np.array([4, 3, 2], np.int32), 0.01
    P = rng.uniform(-0.005, 0.045, ((1 << 21) + 8, 3)).astype(np.float32)   # 24 cells, many points each
    for n in (1, 2, 3, 4, 5, 7, 8, 9, 4097, (1 << 21) + 1, (1 << 21) + 3, 1 << 21):
        for off in (0, 1):                                           # off 1: a view 4 bytes into the buffer
            Q = P[off:off + n]
            full = [torch.as_tensor(np.ascontiguousarray(P[:off + n, a]), device="cuda") for a in range(3)]
            t = [f[off:] for f in full]
            for min_count in (1, 2):
                cells = op.voxel_cells(Q[:, 0], Q[:, 1], Q[:, 2], s, lo, dims, min_count)
                ox, oy, oz, m = ctx.voxel_downsample(*t, s, lo, dims, min_count=min_count, capacity=64)
                torch.cuda.synchronize()
                m = int(m.item())
                assert m == len(cells), (n, off, min_count, m, len(cells))
                C = op.voxel_centres(cells, s, lo, dims).astype(np.float32)
                G = np.stack([ox[:m].cpu().numpy(), oy[:m].cpu().numpy(), oz[:m].cpu().numpy()], 1)
                assert np.array_equal(G, C), (n, off, min_count)


def test_pipeline_config3(ctx):
    """Depth image -> points -> voxel centres on the GPU against the oracle's
    pipeline; cells may differ only where an input point lies within 1e-5 of a
    voxel face (FP32 vs FP64 back-projection)."""
    import torch
    fr = scenes.config3_frame()
    ref_P = op.back_project(fr.depth, fr.K, fr.T_wc)
    ref_cells = op.voxel_cells(ref_P[:, 0], ref_P[:, 1], ref_P[:, 2], fr.voxel, fr.box_lo, fr.dims)
    d = torch.as_tensor(fr.depth, device="cuda")
    x, y, z = ctx.depth_to_points(d, fr.K, fr.T_wc)
    ox, oy, oz, n = ctx.voxel_downsample(x, y, z, fr.voxel, fr.box_lo, fr.dims)
    torch.cuda.synchronize()
    nv = int(n.item())
    G = np.stack([ox[:nv].cpu().numpy(), oy[:nv].cpu().numpy(), oz[:nv].cpu().numpy()], 1).astype(np.float64)
    g_cells = np.round((G - fr.box_lo.astype(np.float64)) / fr.voxel - 0.5).astype(np.int64)
    dims = fr.dims.astype(np.int64)
    g_lin = (g_cells[:, 2] * dims[1] + g_cells[:, 1]) * dims[0] + g_cells[:, 0]
    assert np.all(np.diff(g_lin) > 0)                                # sorted by cell, no duplicates
    # points whose cell is ambiguous: within 1e-5 (relative to the voxel) of a face
    q = (ref_P - fr.box_lo.astype(np.float64)) / fr.voxel
    near = np.isfinite(q).all(1) & (np.abs(q - np.round(q)) < 1e-5).any(1)
    k, ok = op.voxel_keys(ref_P[:, 0].astype(np.float32), ref_P[:, 1].astype(np.float32),
                          ref_P[:, 2].astype(np.float32), fr.voxel, fr.box_lo, fr.dims)
    lin = (k[:, 2] * dims[1] + k[:, 1]) * dims[0] + k[:, 0]
    sure = set(lin[ok & ~near])
    diff = set(ref_cells) ^ set(g_lin)
    assert sure <= set(g_lin)
    assert len(diff) <= 2 * near.sum(), (len(diff), near.sum())
    print(f"config3 voxels: gpu {nv}, oracle {len(ref_cells)}, ambiguous points {near.sum()}", flush=True)


def test_rollout_on_device_sphere_world(ctx):
    """Config 3 at full size: 256 agents over 1,000 steps on the sphere world of the
    depth frame, perceived on the GPU in one fused pass whose device count the rollout
    reads (no host sync).  The oracle rolls out on its own centres of the frame's FP32
    points (the GPU's cells, as the exact tests show) for 16 spread agents, each held to
    1e-4 m or, when ill-conditioned, to its FP64 envelope (reading R24)."""
    import torch
    from paper_2606_12579_amd import gmapp
    fr = scenes.config3_frame()
    d = torch.as_tensor(fr.depth[None].copy(), device="cuda")
    Td = torch.as_tensor(fr.T_wc[None].copy(), device="cuda")
    ox, oy, oz, n = ctx.depth_to_voxels(d, fr.K, Td, fr.voxel, fr.box_lo, fr.dims, capacity=32768)
    agents, q, prm = scenes.config3_agents(n_agents=256, n_steps=1000)
    sc = gmapp.DeviceScene(ox, oy, oz, scenes.R_OBS, n_points_dev=n)
    ag = gmapp.agents_to_device(agents)
    ctx.clear_tiling()
    out = ctx.rollout(sc, ag, q, prm)
    torch.cuda.synchronize()
    nv = int(n.item())
    G = np.stack([ox[:nv].cpu().numpy(), oy[:nv].cpu().numpy(), oz[:nv].cpu().numpy()], 1)
    # the GPU's sphere world: the FP32 points' cells from the depth image (FP32 back-projection)
    gp = np.stack([a.cpu().numpy() for a in ctx.depth_to_points(torch.as_tensor(fr.depth, device="cuda"), fr.K,
                                                                 fr.T_wc)], 1)
    cells = op.voxel_cells(gp[:, 0], gp[:, 1], gp[:, 2], fr.voxel, fr.box_lo, fr.dims)
    C = op.voxel_centres(cells, fr.voxel, fr.box_lo, fr.dims).astype(np.float32)
    assert np.array_equal(G, C)
    idx = np.arange(0, 256, 16)
    pb = scenes.Problem(scenes.Scene(C[:, 0].copy(), C[:, 1].copy(), C[:, 2].copy(), scenes.R_OBS), agents, q, prm)
    gpu = {"traj": out["traj"].cpu().numpy(), "cost": out["cost"].cpu().numpy(),
           "min_clear": out["min_clear"].cpu().numpy()}
    worst, n_ill = gu.compare_conditioned(pb, gpu, idx, "config3")
    assert 0 <= int(out["best"].item()) < 256
    print(f"config3 rollout, 256 agents x 1000 steps on {len(C)} voxel centres: pos err {worst:.2e} "
          f"({n_ill} of {len(idx)} sampled agents ill-conditioned)", flush=True)


def test_batched_rollout_on_device_sphere_world(ctx):
    """Perception -> batched planning without a host sync: two jobs of one
    launch read N_O from the voxel pass's device counter (capacity-sized arrays),
    one of them in two step ranges resumed from the device state."""
    import torch
    from paper_2606_12579_amd import gmapp
    fr = scenes.config3_frame()
    P = op.back_project(fr.depth, fr.K, fr.T_wc).astype(np.float32)
    cells = op.voxel_cells(P[:, 0], P[:, 1], P[:, 2], fr.voxel, fr.box_lo, fr.dims)
    C = op.voxel_centres(cells, fr.voxel, fr.box_lo, fr.dims).astype(np.float32)
    t = [torch.as_tensor(np.ascontiguousarray(P[:, a]), device="cuda") for a in range(3)]
    ox, oy, oz, n = ctx.voxel_downsample(*t, fr.voxel, fr.box_lo, fr.dims, capacity=32768)
    agents, q, prm = scenes.config3_agents(n_agents=24, n_steps=60)
    sc = gmapp.DeviceScene(ox, oy, oz, scenes.R_OBS, n_points_dev=n)
    ag = gmapp.agents_to_device(agents)
    q2 = copy.deepcopy(q)
    q2.p0 = np.asarray(q.p0, np.float32) + np.float32(0.05)
    st = torch.zeros((agents.n, gmapp.STATE_FLOATS), dtype=torch.float32, device="cuda")
    jobs = [gmapp.BatchJob(sc, ag, q, prm, ctx.outputs(agents.n, prm.n_steps)),
            gmapp.BatchJob(sc, ag, q2, prm, ctx.outputs(agents.n, prm.n_steps), st, 1, 25)]
    ctx.clear_batch_tuning()
    ctx.rollout_batch(jobs)
    jobs[1].k_begin, jobs[1].k_end = 25, prm.n_steps + 1
    ctx.rollout_batch([jobs[1]])
    torch.cuda.synchronize()
    idx = np.arange(0, 24, 5)
    for query, j in ((q, jobs[0]), (q2, jobs[1])):
        pb = scenes.Problem(scenes.Scene(C[:, 0].copy(), C[:, 1].copy(), C[:, 2].copy(), scenes.R_OBS),
                            agents.subset(idx), query, prm)
        ref = oracle.rollout(pb)
        gpu = {k: (v.cpu().numpy()[idx] if k != "best" else None) for k, v in j.out.items()}
        gu.compare_rollout(pb, gpu, ref)


def test_voxel_robot_self_filter(ctx):
    """The self-filtered voxel pass gives exactly the oracle's cells on the config-3
    frame with a synthetic arm's spheres across the scene, including points placed
    exactly on the sphere surfaces; no spheres is the plain voxel pass."""
    import torch
    fr = scenes.config3_frame()
    P = op.back_project(fr.depth, fr.K, fr.T_wc).astype(np.float32)
    R = scenes.robot_spheres(np.random.default_rng(9), base=(-0.3, -0.05, 0.0), tip=(0.2, 0.1, 0.3))
    surf = np.array([[c[0] + c[3], c[1], c[2]] for c in R], np.float32)      # on each surface (x + r)
    P = np.concatenate([P, surf, np.nextafter(surf, np.float32(9))], 0)
    hit = op.on_robot(P[:, 0], P[:, 1], P[:, 2], R)
    t = [torch.as_tensor(np.ascontiguousarray(P[:, a]), device="cuda") for a in range(3)]
    Rd = torch.as_tensor(R, device="cuda")
    for min_count in (1, 2):
        cells = op.voxel_cells(P[:, 0], P[:, 1], P[:, 2], fr.voxel, fr.box_lo, fr.dims, min_count, R)
        ox, oy, oz, n = ctx.voxel_downsample(*t, fr.voxel, fr.box_lo, fr.dims, min_count=min_count,
                                             robot_spheres=Rd)
        torch.cuda.synchronize()
        n = int(n.item())
        assert n == len(cells), (n, len(cells))
        G = np.stack([ox[:n].cpu().numpy(), oy[:n].cpu().numpy(), oz[:n].cpu().numpy()], 1)
        assert np.array_equal(G, op.voxel_centres(cells, fr.voxel, fr.box_lo, fr.dims).astype(np.float32))
    print(f"self-filter: {int(hit.sum())} of {len(P)} points on the robot", flush=True)
    plain = op.voxel_cells(P[:, 0], P[:, 1], P[:, 2], fr.voxel, fr.box_lo, fr.dims, 1)
    ox, oy, oz, n = ctx.voxel_downsample(*t, fr.voxel, fr.box_lo, fr.dims,
                                         robot_spheres=torch.zeros((0, 4), dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    assert int(n.item()) == len(plain)
