"""The voxel pass without allocation (gmapp_voxel_downsample_noalloc, through the C ABI)
against the allocating entry point (gmapp_voxel_downsample) on the same inputs: two
calls in a row, the second with a smaller input (a smaller grid, fewer points), both
occupancy and counts; grids beyond the static grid are refused."""
import numpy as np
import pytest

from paper_2606_12579_amd import scenes

pytestmark = pytest.mark.gpu


def test_noalloc_equals_voxel_downsample():
    import torch
    from paper_2606_12579_amd import gmapp
    from oracle import perception as op
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = gmapp.Context(0)
    try:
        fr = scenes.config3_frame()
        P = op.back_project(fr.depth, fr.K, fr.T_wc).astype(np.float32)
        rng = np.random.default_rng(41)
        small = rng.uniform([-0.1, -0.1, 0.0], [0.1, 0.1, 0.05], (5000, 3)).astype(np.float32)
        cases = [(P, fr.box_lo, fr.dims, 1), (small, np.array([-0.1, -0.1, 0.0], np.float32),
                                               np.array([20, 20, 5], np.int32), 1),
                 (P, fr.box_lo, fr.dims, 2), (small[:777], np.array([-0.1, -0.1, 0.0], np.float32),
                                              np.array([20, 20, 5], np.int32), 3)]
        cap = 32768
        out = tuple(torch.empty(cap, dtype=torch.float32, device="cuda") for _ in range(3)) + \
            (torch.zeros(1, dtype=torch.int64, device="cuda"),)
        for pts, lo, dims, mc in cases:
            t = [torch.as_tensor(np.ascontiguousarray(pts[:, a]), device="cuda") for a in range(3)]
            for o in out[:3]:
                o.fill_(float("nan"))
            ctx.voxel_downsample_noalloc(*t, fr.voxel, lo, dims, min_count=mc, out=out)
            ref = ctx.voxel_downsample(*t, fr.voxel, lo, dims, min_count=mc, capacity=cap)
            torch.cuda.synchronize()
            n = int(ref[3].item())
            assert int(out[3].item()) == n and n > 0, (len(pts), mc, int(out[3].item()), n)
            for i in range(3):
                assert torch.equal(out[i][:n], ref[i][:n]), (len(pts), mc, i)
            print(f"noalloc: {len(pts)} points, grid {tuple(int(d) for d in dims)}, min_count {mc}: {n} centres",
                  flush=True)
        with pytest.raises(gmapp.GmappError) as ei:
            ctx.voxel_downsample_noalloc(*t, fr.voxel, lo, np.array([2048, 1024, 2], np.int32), out=out)
        assert ei.value.status == gmapp.ECAPACITY
    finally:
        ctx.close()
