"""CPU checks of the tolerance helpers the GPU parity tests rely on (tests/gpu_util.py):
the C_path bound really bounds the cost change that a trajectory error causes, and the
nearest-sphere tie detector finds ties, agrees between its static (k-d tree) and moving
(brute force) paths, and ignores spheres beyond r_c."""
import copy

import numpy as np

import oracle
from paper_2606_12579_amd import scenes
from tests import gpu_util as gu


def _c_path(pb, traj):
    """C_path (Eq. 19) of trajectories [N_a, >= N_k, 3] through the oracle's cost function."""
    n = pb.params.n_steps
    rmin = np.full(n, 1.0)
    return np.array([oracle.costs(t[:n], rmin, pb.query.goal.astype(np.float64), pb.params)[2] for t in traj])


def test_path_tolerance_bounds_the_cost_change():
    """For smooth drifts, random jitter and a single kink of the position error, of 1e-7 to 1e-4 m, the C_path
    recomputed on the perturbed trajectory moves by no more than the bound (with no floor)."""
    rng = np.random.default_rng(5)
    for pb in (scenes.config1(), scenes.tiny(3, n_points=40, n_agents=5, n_steps=30, moving=True)):
        ref = oracle.rollout(pb)
        base = _c_path(pb, ref.traj)
        n = ref.traj.shape[1]
        for size in (1e-7, 1e-5, 1e-4):
            drift = size * np.linspace(0.0, 1.0, n)[None, :, None] * rng.standard_normal((1, 1, 3))
            jitter = size * rng.standard_normal(ref.traj.shape)
            kink = size * np.abs(np.arange(n) - n // 2)[None, :, None] / n * rng.standard_normal((1, 1, 3))
            for err in (drift, jitter, kink):
                err = err.copy()
                err[:, 0] = 0.0                          # both start at p^(1)
                moved = ref.traj + err
                bound = gu.path_tolerance(pb, moved, ref.traj, 0.0)
                change = np.abs(_c_path(pb, moved) - base)
                assert (change <= bound).all(), (pb.name, size, change, bound)


def test_path_tolerance_floor():
    pb = scenes.config1()
    ref = oracle.rollout(pb)
    assert np.all(gu.path_tolerance(pb, ref.traj, ref.traj, 1e-4) == 1e-4)


def test_nearest_sphere_gap_finds_a_tie():
    """An agent held on the perpendicular bisector of two spheres has gap 0; off it, the gap is the difference of
    the two distances; with both spheres beyond r_c the pair does not count."""
    pb = scenes.tiny(1, n_points=2, n_agents=1, n_steps=3)
    pb.scene = scenes.Scene(np.array([0.0, 0.0], np.float32), np.array([-0.02, 0.02], np.float32),
                            np.zeros(2, np.float32))
    on = np.zeros((1, 4, 3))
    on[0, :, 0] = [0.01, 0.011, 0.012, 0.013]
    assert gu.nearest_sphere_gap(pb, on)[0] == 0.0
    off = on.copy()
    off[0, :, 1] = 0.005
    d = lambda p, q: np.linalg.norm(p - q)
    expect = min(abs(d(off[0, k], [0, 0.02, 0]) - d(off[0, k], [0, -0.02, 0])) for k in range(3))
    assert np.isclose(gu.nearest_sphere_gap(pb, off)[0], expect, rtol=1e-12)
    far = on + np.array([1.0, 0.0, 0.0])
    assert gu.nearest_sphere_gap(pb, far)[0] == np.inf


def test_nearest_sphere_gap_static_equals_moving_path():
    """The k-d tree path (static scene) and the brute-force path (a moving scene whose segments do not move)
    give the same gaps."""
    pb = scenes.tiny(7, n_points=60, n_agents=6, n_steps=25)
    ref = oracle.rollout(pb)
    moving = copy.deepcopy(pb)
    moving.scene.seg_begin = np.array([0, 30, 60], np.int32)
    moving.scene.seg_vel = np.zeros((2, 3), np.float32)
    a = gu.nearest_sphere_gap(pb, ref.traj)
    b = gu.nearest_sphere_gap(moving, ref.traj)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-15)
    assert np.isfinite(a).any()
