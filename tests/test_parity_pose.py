"""GPU parity of 6-D pose agents (gmapp_rollout_pose: Eqs. 6-11 on Spin(3) x| R^3)
against the FP64 oracle, through the C ABI, in several kernel tilings."""
import copy

import numpy as np
import pytest

import oracle
from paper_2606_12579_amd import scenes
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

ROT_TOL = 1e-4          # rotor components (about 2e-4 rad of orientation)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2606_12579_amd import gmapp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = gmapp.Context(0)
    yield c
    c.close()


def _log(msg):
    print(msg, flush=True)


def _gpu(ctx, pb, pa, pq, tiling=None):
    import torch
    from paper_2606_12579_amd import gmapp
    if tiling is not None:
        ctx.set_tiling(*tiling)
    else:
        ctx.clear_tiling()
    sc, ag = gmapp.scene_to_device(pb.scene), gmapp.agents_to_device(pb.agents)
    out = ctx.rollout_pose(sc, ag, gmapp.pose_agents_to_device(pa), pb.query, pq, pb.params)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    res["best"] = int(res["best"][0])
    return res


def _smooth_bound(pb, ref):
    """C_smooth bound: the device takes the jerk from FP32 position increments d_k
    (|d| ~ dt |v|), each component off by up to 4 roundings of max |d|, and the
    error enters sum |j|^2 as 2 |j| e + 3 e^2 per step."""
    N = pb.params.n_steps
    d = np.diff(ref.traj[:, :N], axis=1)                                  # [N_a, N-1, 3]
    j = d[:, 2:] - 2 * d[:, 1:-1] + d[:, :-2]                             # [N_a, N-3, 3]
    e = 4 * 2.0 ** -24 * np.abs(d).max(axis=(1, 2))[:, None] * np.sqrt(3)
    err = (2 * np.linalg.norm(j, axis=2) * e + 3 * e * e).sum(axis=1)
    dt = float(np.float32(pb.params.dt))
    return err / (N * dt ** 4 * float(np.float32(pb.params.a_max)) ** 2)


def _compare(pb, gpu, ref, sampled=False):
    pos_err = float(np.abs(gpu["traj"].astype(np.float64) - ref.traj).max())
    assert pos_err <= gu.POS_TOL, f"position error {pos_err:.3e} m"
    r = gpu["rot"].astype(np.float64)
    r = r * np.where(r[..., :1] < 0, -1.0, 1.0)
    rot_err = float(np.abs(r - ref.rot).max())
    assert rot_err <= ROT_TOL, f"rotor error {rot_err:.3e}"
    mc = gpu["min_clear"].astype(np.float64)
    fin = np.isfinite(ref.min_clear)
    assert np.array_equal(np.isfinite(mc), fin)
    if fin.any():
        assert np.abs(mc[fin] - ref.min_clear[fin]).max() <= pos_err + 1e-6 + 1e-5 * ref.min_clear[fin].max()
    tol = gu.cost_tolerances(pb, pos_err)
    d = np.abs(gpu["cost"].astype(np.float64) - ref.cost)
    for k in range(3):
        assert (d[:, k] <= tol[k]).all(), (k, d[:, k].max(), tol[k])
    sm = tol[3] * np.maximum(np.abs(ref.cost[:, 3]), 1e-3) + _smooth_bound(pb, ref)
    assert (d[:, 3] <= sm).all(), ("C_smooth", d[:, 3].max(), sm.min())
    if not sampled:
        gu.check_selection(gpu["best"], ref.cost, gpu["cost"])
    return pos_err, rot_err


def _case(name):
    rng = np.random.default_rng(12)
    if name == "config1":
        pb = scenes.config1()
    elif name == "moving_multi":
        pb = scenes.tiny(8, n_points=200, n_agents=9, n_steps=50, moving=True)
        pb.agents = scenes.multi_agents(np.random.default_rng(11), 9)
    elif name == "taper":
        pb = scenes.tiny(9, n_points=150, n_agents=6, n_steps=50, cutoff=1)
    elif name == "objects":
        pb = scenes.config2(n_agents=24, n_steps=150, n_points=5000)
    else:
        raise KeyError(name)
    return pb, scenes.pose_agents(rng, pb.agents.n), scenes.pose_query(rng)


@pytest.mark.parametrize("case", ["config1", "moving_multi", "taper", "objects"])
def test_pose_rollout(ctx, case):
    pb, pa, pq = _case(case)
    ref = oracle.rollout_pose(pb, pa, pq)
    for tiling in (None, (1, 8, 4, 0, 0, 2), (2, 8, 4, 0, 0, 2), (2, 1, 2, 0, 1, 1), (8, 4, 1, 256, 2, 1),
                   (4, 4, 4, 0, 0, 1)):
        gpu = _gpu(ctx, pb, pa, pq, tiling)
        pe, re = _compare(pb, gpu, ref)
        _log(f"pose {case} tiling {tiling}: pos err {pe:.2e} rotor err {re:.2e} best {gpu['best']}/{ref.best}")


def test_pose_identity_rotors_match_point_mass(ctx):
    """With identity start and goal rotors and no angular velocity the pose path
    gives the point-mass rollout's trajectories (the same oracle, both within tolerance)."""
    pb = scenes.config1()
    pa = scenes.pose_agents(np.random.default_rng(2), pb.agents.n)
    pq = scenes.PoseQuery(np.array([1, 0, 0, 0], np.float32), np.zeros(3, np.float32),
                          np.array([1, 0, 0, 0], np.float32))
    ref = oracle.rollout(pb)
    gpu = _gpu(ctx, pb, pa, pq)
    assert np.abs(gpu["traj"].astype(np.float64) - ref.traj).max() <= gu.POS_TOL
    assert np.abs(gpu["rot"][..., 0] - 1.0).max() == 0.0


def test_pose_validation(ctx):
    import torch
    from paper_2606_12579_amd import gmapp
    pb, pa, pq = _case("taper")
    sc, ag = gmapp.scene_to_device(pb.scene), gmapp.agents_to_device(pb.agents)
    dpa = gmapp.pose_agents_to_device(pa)
    bad = copy.deepcopy(pq)
    bad.q0 = np.zeros(4, np.float32)
    with pytest.raises(gmapp.GmappError) as ei:
        ctx.rollout_pose(sc, ag, dpa, pb.query, bad, pb.params)
    assert ei.value.status == gmapp.EINVAL
    bad = copy.deepcopy(pq)
    bad.w0 = np.array([np.nan, 0, 0], np.float32)
    with pytest.raises(gmapp.GmappError) as ei:
        ctx.rollout_pose(sc, ag, dpa, pb.query, bad, pb.params)
    assert ei.value.status == gmapp.EINVAL
    torch.cuda.synchronize()


def test_pose_full_size_sampled(ctx):
    """The benchmark's pose workload at full size (config-2 scene, 50,000 moving
    points, 64 pose agents, 500 steps, the built-in tiling): eight sampled agents
    against the oracle run on those agents alone."""
    pb = scenes.config2()
    rng = np.random.default_rng(21)
    pa, pq = scenes.pose_agents(rng, pb.agents.n), scenes.pose_query(rng)
    idx = [0, 9, 18, 27, 36, 45, 54, 63]
    gpu = _gpu(ctx, pb, pa, pq)
    sub = copy.deepcopy(pb)
    sub.agents = pb.agents.subset(idx)
    ref = oracle.rollout_pose(sub, pa.subset(idx), pq)
    g = {k: (v[idx] if isinstance(v, np.ndarray) and v.ndim and v.shape[0] == pb.agents.n else v)
         for k, v in gpu.items()}
    pe, re = _compare(sub, g, ref, sampled=True)
    _log(f"pose full size: sampled pos err {pe:.2e} rotor err {re:.2e}")
