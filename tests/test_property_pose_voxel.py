"""Property sweeps on the GPU for the 6-D pose agents and the voxel pass.

Pose agents (gmapp_rollout_pose, Eqs. 6-11 on Spin(3) x| R^3): random tiny problems
(N_O 1-120, N_a 1-8, N_k 2-40, moving or static, cut-off or taper, random gains,
start rotor, goal and initial twist, homogeneous or mixed heuristics) under random tilings against the FP64 oracle
(positions, rotors, clearances and costs with the bounds of the fixed pose tests).

Voxel pass (Sec. IV-B lattice): random point clouds on random lattices (voxel size,
corner, dims, points on and next to faces, outside the box, non-finite, duplicated),
min_count and capacity, against the oracle's exact cells bit for bit, through
gmapp_voxel_downsample and the allocation-free pass alike."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from oracle import perception as op
from paper_2606_12579_amd import scenes
from tests.test_parity_pose import _compare, _gpu
from tests.test_property_loop import _mix

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
    c.clear_tiling()
    c.close()


POSE_TILINGS = [None, (1, 8, 4, 0, 0, 2), (2, 8, 2, 0, 1, 2), (1, 4, 1, 0, 1, 2), (2, 1, 2, 0, 1, 1),
                (4, 2, 1, 64, 2, 1), (8, 4, 1, 0, 0, 1), (1, 1, 8, 0, 1, 1)]


@settings(max_examples=40, **SETTINGS)
@given(seed=st.integers(0, 2 ** 31 - 1), n_o=st.integers(1, 120), n_a=st.integers(1, 8), n_k=st.integers(2, 40),
       moving=st.booleans(), cutoff=st.integers(0, 1), mixed=st.booleans(), tiling=st.sampled_from(POSE_TILINGS))
def test_random_pose_problems(ctx, seed, n_o, n_a, n_k, moving, cutoff, mixed, tiling):
    pb = scenes.tiny(seed, n_points=n_o, n_agents=n_a, n_steps=n_k, moving=moving, cutoff=cutoff)
    if mixed:                                   # every agent its own heuristic, r_d and k_f
        pb = _mix(pb, np.random.default_rng(seed + 3))
    rng = np.random.default_rng(seed)
    pa, pq = scenes.pose_agents(rng, n_a), scenes.pose_query(rng)
    print(f"seed {seed} N_O {n_o} N_a {n_a} N_k {n_k} moving {moving} cutoff {cutoff} mixed {mixed} tiling {tiling}",
          flush=True)
    ref = oracle.rollout_pose(pb, pa, pq)
    _compare(pb, _gpu(ctx, pb, pa, pq, tiling), ref)


@settings(max_examples=60, **SETTINGS)
@given(seed=st.integers(0, 2 ** 31 - 1), n=st.integers(0, 3000), voxel=st.sampled_from([0.001, 0.003, 0.01, 0.25]),
       lo=st.tuples(*[st.floats(-2.0, 2.0, width=32)] * 3), dims=st.tuples(*[st.integers(1, 300)] * 3),
       min_count=st.integers(1, 3), cap_frac=st.sampled_from([0.0, 0.5, 1.0, 2.0]), static=st.booleans())
def test_random_voxel_passes(ctx, seed, n, voxel, lo, dims, min_count, cap_frac, static):
    import torch
    rng = np.random.default_rng(seed)
    lo = np.array(lo, np.float32)
    dims = np.array(dims, np.int32)
    s = np.float32(voxel)
    ext = dims.astype(np.float64) * float(s)
    # points in the box and a margin around it, a third of them snapped to faces (one FP32
    # step either side included), a few duplicates and non-finite coordinates
    P = (lo.astype(np.float64) - 0.1 * ext + rng.uniform(0.0, 1.2, (n, 3)) * ext).astype(np.float32)
    if n:
        k = n // 3
        f = rng.integers(0, dims + 1, (k, 3)).astype(np.float64)
        face = (lo.astype(np.float64) + f * float(s)).astype(np.float32)
        step = rng.integers(-1, 2, (k, 3))
        face = np.where(step > 0, np.nextafter(face, np.float32(np.inf)),
                        np.where(step < 0, np.nextafter(face, np.float32(-np.inf)), face)).astype(np.float32)
        ax = rng.integers(0, 3, k)
        P[np.arange(k), ax] = face[np.arange(k), ax]
        d = min(n // 10, n - k)
        P[k:k + d] = P[:d]
        P[rng.integers(0, n, max(n // 50, 1)), rng.integers(0, 3, max(n // 50, 1))] = np.nan
    cells = op.voxel_cells(P[:, 0], P[:, 1], P[:, 2], s, lo, dims, min_count)
    cap = int(len(cells) * cap_frac)
    print(f"seed {seed} n {n} voxel {voxel} lo {lo} dims {dims} min_count {min_count} cells {len(cells)} "
          f"capacity {cap} static {static}", flush=True)
    t = [torch.as_tensor(np.ascontiguousarray(P[:, a]), device="cuda") for a in range(3)]
    buf = [torch.full((cap + 8,), -7.0, dtype=torch.float32, device="cuda") for _ in range(3)]
    m = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = (buf[0][:cap], buf[1][:cap], buf[2][:cap], m)
    if static and int(np.prod(dims.astype(np.int64))) <= 1 << 21:
        ctx.voxel_downsample_noalloc(*t, s, lo, dims, min_count=min_count, out=out)
    else:
        ctx.voxel_downsample(*t, s, lo, dims, min_count=min_count, capacity=cap, out=out)
    torch.cuda.synchronize()
    assert int(m.item()) == len(cells), (int(m.item()), len(cells))
    k = min(cap, len(cells))
    C = op.voxel_centres(cells[:k], s, lo, dims).astype(np.float32)
    G = np.stack([buf[a][:k].cpu().numpy() for a in range(3)], 1)
    assert np.array_equal(G, C)
    for a in range(3):                            # nothing written past the count or the capacity
        assert (buf[a][k:].cpu().numpy() == -7.0).all()
