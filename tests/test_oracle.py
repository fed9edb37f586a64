"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these checks re-types the oracle's own formulas: each compares it with a
hand-derived closed form, a physical invariant of the method, an independent
library routine (matrix powers, k-d tree nearest neighbours, ODE exponentials) or
a symmetry.  Together they are meant to fail on a dropped term, a wrong sign,
a wrong index or a transposed operand anywhere in the oracle.
"""
import copy
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.spatial

import oracle
from paper_2606_12579_amd import scenes

KF = 0.01


def _problem_from_points(P, agents, p0, goal, v0=(0, 0, 0), n_steps=50, seg_begin=None, seg_vel=None,
                         r_obs=scenes.R_OBS, cutoff=0):
    P = np.asarray(P, np.float32).reshape(-1, 3)
    sc = scenes.Scene(P[:, 0].copy(), P[:, 1].copy(), P[:, 2].copy(), r_obs, seg_begin, seg_vel)
    q = scenes.Query(np.asarray(p0, np.float32), np.asarray(v0, np.float32), np.asarray(goal, np.float32))
    return scenes.Problem(sc, agents, q, scenes.Params(n_steps=n_steps, cutoff=cutoff))


def _agents(n, **kw):
    rng = np.random.default_rng(123)
    ag = scenes.default_agents(rng, n)
    for k, v in kw.items():
        setattr(ag, k, np.full_like(getattr(ag, k), v) if np.isscalar(v) else np.asarray(v, np.float32))
    return ag


# --------------------------------------------------------------------------- Eq. (2)/(3), one pair
def test_pair_worked_example_perpendicular_current():
    # p = 0, w = (1,0,0), sphere centre (0, 0.1, 0), omega = (0,0,1), R = 0:
    # d = (0,-0.1,0), n = (0,-1,0), c = omega (already orthogonal to n),
    # c x w = (0,1,0), (w/|w|) x (c x w) = (0,0,1), rho = 0.1  =>  f = (k_f/0.1) (0,0,1).
    f, rho = oracle.pair_force([0, 0, 0], [1, 0, 0], [0, 0.1, 0], [0, 0, 1], KF, 0.2, 0.0, 1e-3)
    assert rho == pytest.approx(0.1, abs=1e-15)
    np.testing.assert_allclose(f, [0, 0, 10 * KF], atol=1e-15)


def test_pair_worked_example_projection_and_speed():
    # sphere straight below the agent: d = (0,0,0.05), n = (0,0,1); omega = (1,0,1)/sqrt2
    # => c = omega - n(n.omega) = (1/sqrt2, 0, 0); w = (0,2,0): c x w = (0,0,2/sqrt2),
    # (w/|w|) x (c x w) = (2/sqrt2, 0, 0); R = 0.005 => rho = 0.045.
    s2 = math.sqrt(2.0)
    f, rho = oracle.pair_force([0, 0, 0], [0, 2, 0], [0, 0, -0.05], [1 / s2, 0, 1 / s2], KF, 0.1, 0.005, 1e-3)
    assert rho == pytest.approx(0.045, rel=1e-14)
    np.testing.assert_allclose(f, [KF / 0.045 * 2 / s2, 0, 0], rtol=1e-13, atol=1e-16)
    # omega parallel to n: the current vanishes, so does the force
    f, _ = oracle.pair_force([0, 0, 0], [0, 2, 0], [0, 0, -0.05], [0, 0, 1], KF, 0.1, 0.005, 1e-3)
    np.testing.assert_allclose(f, 0, atol=1e-18)


def test_pair_clamp_cutoff_and_degenerate_cases():
    # inside the inflated sphere: rho clamps to eps (Alg. 1's max(., eps))
    f, rho = oracle.pair_force([0, 0, 0], [1, 0, 0], [0, 0.003, 0], [0, 0, 1], KF, 0.1, 0.005, 1e-3)
    assert rho == 1e-3
    np.testing.assert_allclose(f, [0, 0, KF / 1e-3], rtol=1e-14)
    # hard cut-off keeps rho <= r_d and drops rho > r_d
    f_in, rho = oracle.pair_force([0, 0, 0], [1, 0, 0], [0, 0.125, 0], [0, 0, 1], KF, 0.125, 0.0, 1e-3)
    assert rho == 0.125 and f_in[2] > 0
    f_out, _ = oracle.pair_force([0, 0, 0], [1, 0, 0], [0, 0.125, 0], [0, 0, 1], KF, 0.12499999, 0.0, 1e-3)
    np.testing.assert_array_equal(f_out, 0)
    # zero relative velocity: no force;  agent on the centre: n = 0, c = omega
    f, _ = oracle.pair_force([0, 0, 0], [0, 0, 0], [0, 0.05, 0], [0, 0, 1], KF, 0.1, 0.0, 1e-3)
    np.testing.assert_array_equal(f, 0)
    f, rho = oracle.pair_force([0.3, 0, 0], [0, 1, 0], [0.3, 0, 0], [0, 0, 1], KF, 0.1, 0.0, 1e-3)
    assert rho == 1e-3
    # c = omega = (0,0,1), w = (0,1,0): c x w = (-1,0,0), (w/|w|) x (c x w) = (0,0,1), rho = eps
    np.testing.assert_allclose(f, [0, 0, KF / 1e-3], rtol=1e-14)


def test_taper_closed_form():
    # C1 smoothstep s^2 (3 - 2 s), s = (r_d - rho)/(band r_d): value 1/2 at mid-band, 1 inside, 0 at r_d
    r_d, band = 0.1, 0.1
    for rho, sig in [(0.095, 0.5), (0.09, 1.0), (0.05, 1.0), (0.1, 0.0), (0.0975, 0.15625)]:
        f, r = oracle.pair_force([0, 0, 0], [1, 0, 0], [0, rho, 0], [0, 0, 1], KF, r_d, 0.0, 1e-3, cutoff=1,
                                 band=band)
        assert f[2] == pytest.approx(sig * KF / rho, rel=1e-12, abs=1e-18)


def test_pair_invariants_random():
    """f . w = 0 (no work), |f| <= k_f |w| |omega| / rho, evenness in d and in w."""
    rng = np.random.default_rng(7)
    for _ in range(200):
        p, q = rng.normal(size=3) * 0.05, rng.normal(size=3) * 0.05
        w, om = rng.normal(size=3), rng.normal(size=3)
        f, rho = oracle.pair_force(p, w, q, om, KF, 1.0, 0.005, 1e-3)
        assert abs(np.dot(f, w)) <= 1e-12 * np.linalg.norm(f) * np.linalg.norm(w) + 1e-300
        assert np.linalg.norm(f) <= KF * np.linalg.norm(w) * np.linalg.norm(om) / rho * (1 + 1e-12)
        f2, _ = oracle.pair_force(p, -w, q, om, KF, 1.0, 0.005, 1e-3)
        f3, _ = oracle.pair_force(p, w, 2 * p - q, om, KF, 1.0, 0.005, 1e-3)   # d -> -d
        np.testing.assert_allclose(f2, f, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(f3, f, rtol=1e-12, atol=1e-15)
        # the force is orthogonal to w and depends on omega only through its part
        # orthogonal to n: adding a multiple of n to omega changes nothing
        d = p - q
        n = d / np.linalg.norm(d)
        f4, _ = oracle.pair_force(p, w, q, om + 3.7 * n, KF, 1.0, 0.005, 1e-3)
        np.testing.assert_allclose(f4, f, rtol=1e-10, atol=1e-13)


# --------------------------------------------------------------------------- Alg. 1 sums
def test_repulsion_linear_in_points():
    """Duplicating every sphere doubles the force and keeps rho_min."""
    pb = scenes.tiny(3, n_points=16, n_agents=4)
    rng = np.random.default_rng(0)
    p = rng.uniform(-0.02, 0.06, (4, 3))
    v = rng.normal(size=(4, 3))
    r1 = oracle.repulsion(pb, p, v, 0.0)
    sc = pb.scene
    pb2 = _problem_from_points(np.concatenate([np.stack([sc.x, sc.y, sc.z], 1)] * 2), pb.agents, [0, 0, 0],
                               [1, 0, 0])
    r2 = oracle.repulsion(pb2, p, v, 0.0)
    np.testing.assert_allclose(r2.force, 2 * r1.force, rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(r2.rho_min, r1.rho_min)


def test_force_tolerance_terms_hand_placed():
    """The two diagnostics that enter the per-step force tolerance, pinned on hand-placed
    spheres around an agent at the origin moving along x with omega = z (r_O = r_a = 0,
    so rho is the centre distance):
      sum_j |f_j| counts every kept pair once, with |f_j| = k_f / rho_j for a current
        perpendicular to w (and 0 where the current vanishes);
      the edge terms count the pairs within 1e-6 r_d of the hard cut-off, on both sides
        of it, with the force each would give if classified the other way;
      the term magnitudes give each kept pair s |w| (|omega| + |n . omega|), s = k_f / rho:
        k_f / rho where n is perpendicular to omega, 2 k_f / rho for the pair whose current
        vanishes (its two terms cancel), and never less than |f_j|;
    pairs farther from the cut-off, and the whole edge band under the taper, add nothing."""
    r_d = np.float32(0.1)
    up = lambda x, n: [x := np.nextafter(x, np.float32(1.0)) for _ in range(n)][-1]
    dn = lambda x, n: [x := np.nextafter(x, np.float32(0.0)) for _ in range(n)][-1]
    r5, r6, r7 = up(r_d, 7), up(r_d, 41), dn(r_d, 7)     # 5.2e-7, 3.1e-6, -3.7e-7 relative to r_d
    P = np.array([[0.0, 0.05, 0.0],        # inside, current perpendicular to w: |f| = k_f / rho
                  [0.0, 0.0, 0.08],        # inside, n parallel to omega: no current, f = 0
                  [0.0, -r_d, 0.0],        # exactly at rho = r_d: kept, in the edge band
                  [0.2, 0.0, 0.0],         # beyond r_d
                  [-r5, 0.0, 0.0],         # just beyond r_d, in the band (force 0, would be k_f / rho)
                  [0.0, r6, 0.0],          # beyond r_d, outside the band
                  [r7, 0.0, 0.0]],         # just inside r_d, in the band
                 np.float32)
    ag = _agents(1, k_f=KF, r_d=r_d, r_a=0.0, omega=[[0.0, 0.0, 1.0]])
    rho = lambda i: float(np.linalg.norm(P[i].astype(np.float64)))
    for cutoff in (0, 1):
        pb = _problem_from_points(P, ag, [0, 0, 0], [1, 0, 0], r_obs=0.0, cutoff=cutoff)
        r = oracle.repulsion(pb, [[0.0, 0.0, 0.0]], [[1.0, 0.0, 0.0]], 0.0)
        assert r.rho_min[0] == rho(0)
        kf = float(np.float32(KF))
        if cutoff == 0:
            kept = kf / rho(0) + kf / rho(2) + kf / rho(6)
            np.testing.assert_allclose(r.force[0], [0.0, 0.0, kept], rtol=1e-12, atol=1e-18)
            np.testing.assert_allclose(r.abs_sum[0], kept, rtol=1e-12)
            np.testing.assert_allclose(r.edge_sum[0], kf / rho(2) + kf / rho(4) + kf / rho(6), rtol=1e-12)
            assert r.edge_cnt[0] == 3
            np.testing.assert_allclose(r.term_sum[0], kept + 2 * kf / rho(1), rtol=1e-12)
        else:
            assert r.edge_sum[0] == 0.0 and r.edge_cnt[0] == 0
            assert r.abs_sum[0] >= abs(r.force[0, 2]) > 0.0
        assert r.term_sum[0] >= r.abs_sum[0]


def test_force_tolerance_terms_cancellation_and_frame():
    """The term magnitudes and the frame-rounding diagnostic of the force tolerance, by their
    properties rather than their formulas:
      every pair's term magnitude is at least its |f_j| (so the sum is at least sum_j |f_j|), with
      equality for none of the APF pairs (its two terms 1/rho and 1/r_d have the same sign);
      an APF sphere just inside the cut-off gives a vanishing force but a term magnitude that
      stays at its interior size, and one beyond the cut-off adds nothing;
      under the taper the magnitude exceeds |f_j| most where the weight is smallest;
      the frame diagnostic is zero for static spheres, at t = 0, and when p - t v_seg is an FP32
      number, and otherwise positive and within the force's own change over one FP32 step."""
    r_d = 0.1
    P = np.array([[0.03, 0.0, 0.0], [0.0, 0.05, 0.0], [0.0, 0.0, 0.099999], [0.0, -0.2, 0.0]], np.float32)
    for heur in (0, 1, 2):
        for cutoff in (0, 1):
            ag = _agents(1, k_f=KF if heur < 2 else scenes.K_F_APF, r_d=r_d, r_a=0.0, omega=[[0.0, 0.6, 0.8]])
            ag.heuristic = np.array([heur], np.int32)
            pb = _problem_from_points(P, ag, [0, 0, 0], [1, 0, 0], r_obs=0.0, cutoff=cutoff)
            r = oracle.repulsion(pb, [[0.0, 0.0, 0.0]], [[0.3, -0.2, 0.1]], 0.0)
            assert r.term_sum[0] >= r.abs_sum[0] > 0.0
            if heur == 2:
                assert r.term_sum[0] > 1.5 * r.abs_sum[0]
            assert r.shift_sum[0] == 0.0                     # static spheres
    # APF at the cut-off: the force of a sphere at rho -> r_d vanishes, its term magnitude does not
    ag = _agents(1, k_f=scenes.K_F_APF, r_d=r_d, r_a=0.0)
    ag.heuristic = np.array([2], np.int32)
    near = lambda x: oracle.repulsion(_problem_from_points([[x, 0, 0]], ag, [0, 0, 0], [1, 0, 0], r_obs=0.0),
                                      [[0.0, 0.0, 0.0]], [[0.3, 0.0, 0.0]], 0.0)
    inner, edge, out = near(0.05), near(float(np.nextafter(np.float32(r_d), np.float32(0)))), near(0.2)
    assert edge.abs_sum[0] < 1e-5 * inner.abs_sum[0]
    assert edge.term_sum[0] > 0.1 * inner.term_sum[0]
    assert out.term_sum[0] == 0.0 and out.abs_sum[0] == 0.0
    # taper: the ratio term / |f| grows towards the outer edge of the band
    ag = _agents(1, k_f=KF, r_d=r_d, r_a=0.0, omega=[[0.0, 0.0, 1.0]])
    ratios = []
    for x in (0.08, 0.092, 0.096, 0.099):
        pb = _problem_from_points([[0.0, x, 0.0]], ag, [0, 0, 0], [1, 0, 0], r_obs=0.0, cutoff=1)
        r = oracle.repulsion(pb, [[0.0, 0.0, 0.0]], [[1.0, 0.0, 0.0]], 0.0)
        ratios.append(r.term_sum[0] / r.abs_sum[0])
    assert ratios[0] == pytest.approx(1.0, rel=1e-12)           # on the plateau: the force is one term
    assert all(b > a for a, b in zip(ratios[1:], ratios[2:]))
    # frame rounding on a moving sphere
    ag = _agents(1, k_f=KF, r_d=r_d, r_a=0.0, omega=[[0.0, 0.0, 1.0]])
    seg = dict(seg_begin=np.array([0, 1], np.int32), seg_vel=np.array([[1.0, 0.0, 0.0]], np.float32))

    def frame(p, t):
        pb = _problem_from_points([[0.0, 0.004, 0.0]], ag, [0, 0, 0], [1, 0, 0], r_obs=0.0, **seg)
        return oracle.repulsion(pb, [p], [[0.0, 0.5, 0.0]], t)
    assert frame([0.5, 0.0, 0.0], 0.0).shift_sum[0] == 0.0        # t = 0
    assert frame([0.5, 0.0, 0.0], 0.25).shift_sum[0] == 0.0       # 0.5 - 0.25 is an FP32 number
    p = [float(np.float32(0.05)), float(np.float32(0.003)), 0.0]
    t = float(np.float32(0.001))                                   # 0.05 - 0.001 is not an FP32 number
    r = frame(p, t)
    assert r.shift_sum[0] > 0.0
    # within the change of f over one FP32 step of the relative position (2^-24 of |p|, per axis)
    step = 2.0 ** -24 * 0.1
    r_up = frame([p[0] + step, p[1], p[2]], t)
    assert r.shift_sum[0] <= 4 * np.linalg.norm(r_up.force[0] - r.force[0]) + 1e-12 * np.linalg.norm(r.force[0])


def test_repulsion_diagnostics_do_not_change_the_force():
    """The tolerance diagnostics are computed beside the force, never into it: with and without them the force
    and rho_min are identical, and without them the diagnostics read zero."""
    pb = scenes.tiny(9, n_points=50, n_agents=6, n_steps=5, moving=True)
    pb.agents = scenes.multi_agents(np.random.default_rng(2), 6)
    rng = np.random.default_rng(3)
    p = rng.uniform(-0.02, 0.06, (6, 3))
    v = rng.normal(size=(6, 3))
    a = oracle.repulsion(pb, p, v, 0.003)
    b = oracle.repulsion(pb, p, v, 0.003, diagnostics=False)
    assert np.array_equal(a.force, b.force) and np.array_equal(a.rho_min, b.rho_min)
    for f in ("abs_sum", "edge_sum", "edge_cnt", "term_sum", "shift_sum"):
        assert not np.any(getattr(b, f)), f
    assert (a.term_sum >= a.abs_sum).all() and (a.shift_sum > 0).any()


def test_min_distance_matches_kdtree():
    """rho_min^(k) = max(nearest-centre distance - (r_O + r_a), eps): checked with scipy's k-d tree."""
    pb = scenes.config1()
    pb.params.n_steps = 60
    res = oracle.rollout(pb)
    P = np.stack([pb.scene.x, pb.scene.y, pb.scene.z], 1).astype(np.float64)
    tree = scipy.spatial.cKDTree(P)
    R = float(np.float32(pb.scene.r_obs)) + pb.agents.r_a.astype(np.float64)[:, None]
    dist, _ = tree.query(res.traj[:, :-1].reshape(-1, 3))
    expect = np.maximum(dist.reshape(res.min_clear.shape) - R, np.float32(pb.params.eps))
    np.testing.assert_allclose(res.min_clear, expect, rtol=1e-13, atol=1e-16)


def test_min_distance_moving_segments_bruteforce():
    """Moving obstacles: sphere j sits at q_j + t_k v_seg(j), t_k = (k-1) dt."""
    pb = scenes.tiny(11, n_points=12, n_agents=3, n_steps=8, moving=True)
    res = oracle.rollout(pb)
    sc = pb.scene
    Q = np.stack([sc.x, sc.y, sc.z], 1).astype(np.float64)
    V = np.zeros_like(Q)
    for s in range(sc.n_seg):
        V[sc.seg_begin[s]:sc.seg_begin[s + 1]] = sc.seg_vel[s]
    dt = float(np.float32(pb.params.dt))
    for k in range(1, pb.params.n_steps + 1):
        tree = scipy.spatial.cKDTree(Q + (k - 1) * dt * V)
        dist, _ = tree.query(res.traj[:, k - 1])
        expect = np.maximum(dist - (float(np.float32(sc.r_obs)) + pb.agents.r_a), float(np.float32(1e-3)))
        np.testing.assert_allclose(res.min_clear[:, k - 1], expect, rtol=1e-13)


# --------------------------------------------------------------------------- Eqs. (6)-(11)
def _attractive_closed_form(pb):
    """Per axis, e_k = x_k - g and v_{k-1} follow s_{k+1} = M s_k with
    M = [[1 - dt^2 k/2m, dt (1 - dt d/2m)], [-dt k/2m, 1 - dt d/2m]]; powers of M by numpy."""
    prm = pb.params
    dt, invm = float(np.float32(prm.dt)), float(np.float32(prm.inv_mass))
    out = []
    for i in range(pb.agents.n):
        k, d = float(pb.agents.k_a[i]), float(pb.agents.d_a[i])
        h = 0.5 * dt * invm
        M = np.array([[1 - dt * h * k, dt * (1 - h * d)], [-h * k, 1 - h * d]])
        e0 = pb.query.p0.astype(np.float64) - pb.query.goal.astype(np.float64)
        s = np.stack([e0, pb.query.v0.astype(np.float64)])   # [2, 3]
        traj = [np.linalg.matrix_power(M, n) @ s for n in range(prm.n_steps + 1)]
        out.append(np.stack([t[0] for t in traj]) + pb.query.goal.astype(np.float64))
    return np.stack(out)


def test_attractive_only_matches_matrix_power():
    ag = _agents(3, k_a=[400.0, 100.0, 900.0], d_a=[56.5685, 5.0, 30.0])
    pb = _problem_from_points(np.zeros((0, 3)), ag, [0.1, -0.2, 0.3], [1.0, 0.5, -0.25], v0=[0.3, 0.0, -0.1],
                              n_steps=300)
    res = oracle.rollout(pb)
    np.testing.assert_allclose(res.traj, _attractive_closed_form(pb), rtol=0, atol=1e-12)
    # k_f = 0 with obstacles present is the same motion
    pb2 = scenes.config1()
    pb2.agents.k_f[:] = 0
    pb2.params.n_steps = 100
    res2 = oracle.rollout(pb2)
    np.testing.assert_allclose(res2.traj, _attractive_closed_form(pb2), rtol=0, atol=1e-12)


def test_attractive_converges_to_continuous_damped_oscillator():
    """The scheme integrates xdd = (k (g - x) - d xd) / (2m) (Eq. 10 keeps its 1/2);
    halving dt halves the error at a fixed time (first order)."""
    ag = _agents(1, k_a=400.0, d_a=20.0)
    T = 0.2
    errs = []
    for dt in (1e-3, 5e-4, 2.5e-4):
        pb = _problem_from_points(np.zeros((0, 3)), ag, [0, 0, 0], [1, 0, 0], n_steps=int(round(T / dt)))
        pb.params.dt = dt
        res = oracle.rollout(pb)
        dt32 = float(np.float32(dt))
        n = pb.params.n_steps
        A = np.array([[0, 1], [-400.0 / 2, -20.0 / 2]])
        e = scipy.linalg.expm(A * n * dt32) @ np.array([-1.0, 0.0])
        errs.append(abs(res.traj[0, n, 0] - (1.0 + e[0])))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.8 < r1 < 2.2 and 1.8 < r2 < 2.2, errs


def test_circular_field_does_no_work():
    """k_a = d_a = 0, static spheres: F is orthogonal to v^(k-1), so
    |v^(k)|^2 = |v^(k-1)|^2 + (dt/2m)^2 |F^(k)|^2 exactly (discrete energy identity)."""
    pb = scenes.config1()
    pb.agents.k_a[:] = 0
    pb.agents.d_a[:] = 0
    pb.query.v0[:] = [1.5, 0.1, -0.05]
    pb.params.n_steps = 400
    res = oracle.rollout(pb)
    h = 0.5 * float(np.float32(pb.params.dt)) * float(np.float32(pb.params.inv_mass))
    v2 = np.sum(res.vel ** 2, -1)
    lhs = v2[:, 1:] - v2[:, :-1]
    rhs = h * h * np.sum(res.ftot ** 2, -1)
    assert np.abs(res.force).max() > 10.0   # the field really acts
    np.testing.assert_allclose(lhs, rhs, rtol=1e-7, atol=1e-12 * v2.max())
    # per step the work term 2 h v^(k-1).F^(k) vanishes
    work = np.sum(res.vel[:, :-1] * res.ftot, -1)
    assert np.abs(work).max() <= 1e-11 * np.abs(res.ftot).max()


def test_jerk_identity():
    """Delta^3 p^(k) = (dt^2/2m)(F^(k-1) - F^(k-2)) under the explicit half-kick scheme."""
    pb = scenes.config1()
    res = oracle.rollout(pb)
    dt, invm = float(np.float32(pb.params.dt)), float(np.float32(pb.params.inv_mass))
    p = res.traj
    d3 = p[:, 3:-1] - 3 * p[:, 2:-2] + 3 * p[:, 1:-3] - p[:, :-4]            # k = 4..N
    ident = 0.5 * dt * dt * invm * (res.ftot[:, 2:-1] - res.ftot[:, 1:-2])  # F^(k-1) - F^(k-2)
    np.testing.assert_allclose(d3, ident, rtol=0, atol=1e-9 * np.abs(ident).max())


# --------------------------------------------------------------------------- Eqs. (16)-(20)
def test_costs_straight_constant_velocity():
    N, dt = 80, 1e-3
    prm = scenes.Params(n_steps=N, dt=dt)
    dt = float(np.float32(dt))
    u = np.array([0.6, 0.0, 0.8])
    p0 = np.array([0.1, 0.2, 0.3])
    pos = p0 + np.arange(N)[:, None] * dt * u
    goal = p0 + (N - 1) * dt * u
    c = oracle.costs(pos, np.full(N, 1.0), goal, prm)
    rc = float(np.float32(prm.r_cost))
    assert c[0] == pytest.approx(dt * (N - 1) / (2 * rc), rel=1e-12)   # sum of (N-k) dt / r_c
    assert c[1] == 0.0                                                  # no sphere within r_c
    assert abs(c[2]) < 1e-12                                            # L = d1
    assert c[3] < 1e-20                                                 # no jerk
    assert c[4] == pytest.approx(c.sum() - c[4], rel=1e-12)


def test_costs_cubic_and_degenerate():
    N, dt = 50, 1e-3
    prm = scenes.Params(n_steps=N, dt=dt, a_max=10.0)
    dt = float(np.float32(dt))
    cc = 1e-9
    k = np.arange(1, N + 1)
    pos = np.stack([cc * k ** 3, np.zeros(N), np.zeros(N)], 1)
    c = oracle.costs(pos, np.full(N, 0.0), [5.0, 0, 0], prm)
    J = (N - 3) * (6 * cc) ** 2
    a = float(np.float32(10.0))
    assert c[3] == pytest.approx(min(1.0, J / (N * dt ** 4 * a * a)), rel=1e-9)
    assert c[1] == pytest.approx(1.0)                                   # touching every step
    assert c[0] == 1.0                                                  # goal farther than r_c throughout
    L = cc * (N ** 3 - 1)
    d1 = 5.0 - cc
    assert c[2] == pytest.approx(1 - L / d1, rel=1e-12)                 # L < d1 branch
    still = np.tile([0.2, 0.0, 0.0], (N, 1))
    assert oracle.costs(still, np.full(N, 1.0), [0.7, 0, 0], prm)[2] == 1.0   # L = 0 < d1
    assert oracle.costs(still, np.full(N, 1.0), [0.2, 0, 0], prm)[2] == 0.0   # L = d1 = 0
    eps = float(np.float32(1e-3))
    c = oracle.costs(still, np.full(N, eps), [0.2, 0, 0], prm)
    assert c[1] == pytest.approx(1 - eps / float(np.float32(prm.r_cost)))
    # smooth cost saturates at 1
    big = np.stack([1e-3 * k ** 3, np.zeros(N), np.zeros(N)], 1)
    assert oracle.costs(big, np.full(N, 1.0), [0, 0, 0], prm)[3] == 1.0


def test_selection_rule():
    assert oracle.select([3.0, 1.0, 2.0, 1.0]) == 1                 # argmin, lowest index on ties
    assert oracle.select([np.nan, 2.0, np.nan]) == 1                  # NaN never wins
    # with an incumbent b: only C_i < alpha C_b can replace it
    assert oracle.select([1.0, 0.95, 0.85], incumbent=0, alpha=0.9) == 2
    assert oracle.select([1.0, 0.95, 0.91], incumbent=0, alpha=0.9) == 0
    assert oracle.select([1.0, 0.5, 0.5], incumbent=0, alpha=0.9) == 1
    assert oracle.select([], incumbent=-1) == -1


# --------------------------------------------------------------------------- symmetry / structure
def _rotation(rng):
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def test_rotation_and_translation_covariance():
    rng = np.random.default_rng(5)
    pb = scenes.tiny(2, n_points=40, n_agents=3, n_steps=40)
    base = oracle.rollout(pb)
    R = _rotation(rng)
    t = np.array([0.3, -0.2, 0.1])
    P = np.stack([pb.scene.x, pb.scene.y, pb.scene.z], 1).astype(np.float64)
    # rotate the float64 scene; the oracle takes float64 values as given
    import copy
    pb2 = copy.deepcopy(pb)
    sc = pb2.scene
    P2 = P @ R.T + t
    sc.x, sc.y, sc.z = P2[:, 0], P2[:, 1], P2[:, 2]
    pb2.agents.omega = pb.agents.omega.astype(np.float64) @ R.T   # proper rotation: omega rotates too
    pb2.query.p0 = pb.query.p0.astype(np.float64) @ R.T + t
    pb2.query.goal = pb.query.goal.astype(np.float64) @ R.T + t
    pb2.query.v0 = pb.query.v0.astype(np.float64) @ R.T
    res = oracle.rollout(pb2)
    np.testing.assert_allclose(res.traj, base.traj @ R.T + t, rtol=0, atol=1e-10)
    np.testing.assert_allclose(res.cost, base.cost, rtol=1e-8, atol=1e-10)
    assert res.best == base.best


def test_agents_are_independent_and_point_order_free():
    pb = scenes.config1()
    pb.params.n_steps = 30
    base = oracle.rollout(pb)
    import copy
    sub = copy.deepcopy(pb)
    sub.agents = pb.agents.subset([5, 2])
    r = oracle.rollout(sub)
    np.testing.assert_array_equal(r.traj, base.traj[[5, 2]])
    perm = np.random.default_rng(1).permutation(pb.scene.n)
    sh = copy.deepcopy(pb)
    sh.scene.x, sh.scene.y, sh.scene.z = pb.scene.x[perm], pb.scene.y[perm], pb.scene.z[perm]
    r = oracle.rollout(sh)
    np.testing.assert_allclose(r.traj, base.traj, rtol=0, atol=1e-12)


# --------------------------------------------------------------------------- gradients
def test_dual_gradient_matches_central_differences():
    pb = scenes.tiny(4, n_points=24, n_agents=2, n_steps=25, cutoff=1)
    pb.agents.k_f[:] = 0.02
    g = oracle.rollout_grad(pb)
    base = oracle.rollout(pb)
    np.testing.assert_allclose(g[:, 0], base.cost[:, 4], rtol=1e-13)
    import copy
    names = [("k_a", None), ("d_a", None), ("k_f", None), ("omega", 0), ("omega", 1), ("omega", 2)]
    for i in range(pb.agents.n):
        for col, (name, ax) in enumerate(names):
            theta = float(getattr(pb.agents, name)[i] if ax is None else pb.agents.omega[i, ax])
            errs = []
            for h in (1e-3, 5e-4):
                step = h * max(1.0, abs(theta))
                vals = []
                for sgn in (1, -1):
                    q = copy.deepcopy(pb)
                    for f in ("k_a", "d_a", "k_f", "r_d", "r_a", "omega"):
                        setattr(q.agents, f, getattr(q.agents, f).astype(np.float64))
                    if ax is None:
                        getattr(q.agents, name)[i] = theta + sgn * step
                    else:
                        q.agents.omega[i, ax] = theta + sgn * step
                    vals.append(oracle.rollout(q).cost[i, 4])
                fd = (vals[0] - vals[1]) / (2 * step)
                errs.append(abs(fd - g[i, 1 + col]))
            scale = max(abs(g[i, 1 + col]), 1e-6)
            assert errs[-1] <= 1e-4 * scale + 1e-9, (i, name, ax, errs, g[i, 1 + col])
            # second-order convergence (or already at rounding level)
            assert errs[1] <= 0.5 * errs[0] or errs[1] < 1e-9 * max(1.0, scale), (i, name, ax, errs)


def test_moving_obstacles_galilean_invariance():
    """Without attractor and damping (k_a = d_a = 0) the force depends only on the
    relative position and the relative velocity w = v - v_obj.  Moving every sphere
    with u and giving the agent v0 + u reproduces the static motion shifted by
    u t_k, t_k = (k-1) dt, with velocities shifted by u."""
    import copy
    pb = scenes.tiny(21, n_points=30, n_agents=3, n_steps=60)
    pb.agents.k_a[:] = 0
    pb.agents.d_a[:] = 0
    pb.agents.k_f[:] = 0.05
    base = oracle.rollout(pb)
    u = np.array([0.15, -0.1, 0.05])
    mv = copy.deepcopy(pb)
    mv.scene.seg_begin = np.array([0, pb.scene.n], np.int32)
    mv.scene.seg_vel = u.reshape(1, 3)
    mv.query.v0 = pb.query.v0.astype(np.float64) + u
    res = oracle.rollout(mv)
    dt = float(np.float32(pb.params.dt))
    shift = (np.arange(pb.params.n_steps + 1) * dt)[:, None] * u
    assert np.abs(base.force).max() > 1.0
    np.testing.assert_allclose(res.traj, base.traj + shift, rtol=0, atol=1e-12)
    np.testing.assert_allclose(res.vel, base.vel + u, rtol=0, atol=1e-12)
    np.testing.assert_allclose(res.min_clear, base.min_clear, rtol=1e-10)


# ---------------------------------------------------------------- other heuristics (Sec. III-A)

def _apf_potential(p, q, k_f, r_d, R):
    """U = (k_f / 2) (1/rho - 1/r_d)^2 inside the detection distance (Khatib's FIRAS
    potential), whose negative gradient is Eq. (1)'s force."""
    rho = np.linalg.norm(p - q) - R
    return 0.5 * k_f * (1.0 / rho - 1.0 / r_d) ** 2 if rho < r_d else 0.0


def test_apf_force_is_the_potential_gradient():
    """Eq. (1) (distance read as the surface distance rho) against central
    differences of its potential, at random points inside the detection shell;
    zero outside it and continuous at rho = r_d."""
    rng = np.random.default_rng(21)
    k_f, r_d, R, eps = 0.01, 0.1, 0.005, 1e-3
    for _ in range(40):
        q = rng.uniform(-1, 1, 3)
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        rho = rng.uniform(0.01, 0.095)
        p = q + (R + rho) * n
        f, rho_o = oracle.pair_force_heuristic(2, p, np.zeros(3), q, np.zeros(3), k_f, r_d, R, eps)
        assert rho_o == pytest.approx(rho, rel=1e-12)
        h = 1e-7
        g = np.array([(_apf_potential(p + h * e, q, k_f, r_d, R) - _apf_potential(p - h * e, q, k_f, r_d, R)) / (2 * h)
                      for e in np.eye(3)])
        np.testing.assert_allclose(f, -g, rtol=1e-6, atol=1e-9 * np.abs(g).max())
        assert f @ n > 0                                     # repulsive, along the outward normal
    q = np.zeros(3)
    far = np.array([R + 0.2, 0.0, 0.0])
    f, _ = oracle.pair_force_heuristic(2, far, np.zeros(3), q, np.zeros(3), k_f, r_d, R, eps)
    assert not f.any()
    edge = np.array([R + r_d * (1 - 1e-9), 0.0, 0.0])
    f, _ = oracle.pair_force_heuristic(2, edge, np.zeros(3), q, np.zeros(3), k_f, r_d, R, eps)
    assert np.linalg.norm(f) < 1e-6


def test_velocity_current_field_closed_form():
    """Eq. (2) with Eq. (3)'s current taken from the relative velocity w:
    f = -(k_f |w|^2 / rho) (n . w^) (n - w^ (w^ . n)) -- no work, zero when w is
    parallel or orthogonal to the normal, deflecting away while approaching."""
    rng = np.random.default_rng(22)
    k_f, r_d, R, eps = 0.01, 0.1, 0.005, 1e-3
    for _ in range(40):
        q = rng.uniform(-1, 1, 3)
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        rho = rng.uniform(0.01, 0.09)
        p = q + (R + rho) * n
        w = rng.standard_normal(3) * rng.uniform(0.1, 2.0)
        f, _ = oracle.pair_force_heuristic(1, p, w, q, rng.standard_normal(3), k_f, r_d, R, eps)
        wn = np.linalg.norm(w)
        u = w / wn
        want = -(k_f * wn * wn / rho) * (n @ u) * (n - u * (u @ n))
        np.testing.assert_allclose(f, want, rtol=1e-10, atol=1e-14)
        assert abs(f @ w) <= 1e-12 * np.linalg.norm(f) * wn
        if n @ w < 0:                                        # approaching: pushed outwards
            assert f @ n >= -1e-15
        for w_special in (2.0 * n, np.cross(n, rng.standard_normal(3))):
            f0, _ = oracle.pair_force_heuristic(1, p, w_special, q, np.zeros(3), k_f, r_d, R, eps)
            assert np.linalg.norm(f0) <= 1e-12 * k_f / rho


def test_velocity_current_field_does_no_work():
    """The velocity-current field is orthogonal to w as well, so the discrete energy
    identity of the rotation-vector field holds for it too (k_a = d_a = 0, static)."""
    pb = scenes.config1()
    pb.agents.k_a[:] = 0
    pb.agents.d_a[:] = 0
    pb.agents.heuristic = np.ones(pb.agents.n, np.int32)
    pb.query.v0[:] = [1.5, 0.3, -0.2]
    pb.params.n_steps = 300
    res = oracle.rollout(pb)
    h = 0.5 * float(np.float32(pb.params.dt)) * float(np.float32(pb.params.inv_mass))
    v2 = np.sum(res.vel ** 2, -1)
    assert np.abs(res.force).max() > 1.0
    np.testing.assert_allclose(v2[:, 1:] - v2[:, :-1], h * h * np.sum(res.ftot ** 2, -1), rtol=1e-7,
                               atol=1e-12 * v2.max())


def test_mixed_heuristics_are_independent():
    """In a heterogeneous ensemble every agent's rollout equals its rollout alone."""
    pb = scenes.tiny(23, n_points=60, n_agents=6, n_steps=40)
    pb.agents.heuristic = np.array([0, 1, 2, 2, 1, 0], np.int32)
    pb.agents.k_f = np.where(pb.agents.heuristic == 2, 1e-5, 0.02).astype(np.float32)
    full = oracle.rollout(pb)
    for i in range(pb.agents.n):
        sub = copy.deepcopy(pb)
        sub.agents = pb.agents.subset([i])
        one = oracle.rollout(sub)
        np.testing.assert_array_equal(one.traj[0], full.traj[i])


# ---------------------------------------------------------------- closed planning loop (Sec. V-B)

def test_loop_control_steps_reproduce_the_selected_rollout():
    """With the control period equal to dt and N_k control steps per cycle, the
    robot's control steps integrate exactly the selected agent's rollout, so each
    cycle ends at that agent's p^(N_k+1), v^(N_k) and records its clearances; the
    control integration (numpy) and the rollout (C) are separate codes."""
    pb = scenes.tiny(8, n_points=200, n_agents=5, n_steps=30, moving=True)
    N, C = pb.params.n_steps, 3
    res = oracle.plan_loop(pb, C, N, pb.params.dt)
    inc = pb.query.incumbent
    for c in range(C):
        sub = copy.deepcopy(pb)
        row = res.robot[c * N]
        sub.query.p0, sub.query.v0, sub.query.t0, sub.query.incumbent = row[:3], row[3:], res.t0[c], inc
        r = oracle.rollout(sub)
        i = r.best
        assert i == res.best[c]
        np.testing.assert_allclose(res.robot[(c + 1) * N, :3], r.traj[i, N], rtol=0, atol=1e-12)
        np.testing.assert_allclose(res.robot[(c + 1) * N, 3:], r.vel[i, N], rtol=0, atol=1e-10)
        np.testing.assert_allclose(res.robot_clear[c * N:(c + 1) * N], r.min_clear[i], rtol=1e-12, atol=0)
        inc = i


def test_loop_grouping_of_control_steps():
    """While i* stays the same, the robot's path is the same sequence of control
    steps however they are grouped into cycles (moving spheres, so each step's
    time matters), and cycle c starts at t0 + c ctrl_steps ctrl_dt."""
    pb = scenes.tiny(8, n_points=200, n_agents=5, n_steps=30, moving=True)
    pb.query.t0 = 0.0125
    a = oracle.plan_loop(pb, 2, 10, 0.005)
    b = oracle.plan_loop(pb, 4, 5, 0.005)
    assert len(set(a.best.tolist() + b.best.tolist())) == 1
    # each cycle's start time is rounded to FP32 (about 1e-9 s here, the spheres move 0.2 m/s)
    np.testing.assert_allclose(a.robot, b.robot, rtol=0, atol=1e-8)
    np.testing.assert_allclose(a.robot_clear, b.robot_clear, rtol=0, atol=1e-8)
    dt = float(np.float32(0.005))
    assert b.t0.tolist() == [float(np.float32(float(np.float32(0.0125)) + 5 * c * dt)) for c in range(4)]


def test_loop_without_obstacles_is_the_damped_oscillator():
    """No spheres: every agent has the same cost, so i* stays agent 0 and N_sw = 0,
    and the robot follows x_{n+1} = M x_n + b per axis, whose closed form is
    x_n = x* + M^n (x_0 - x*) with the fixed point x* = (goal, 0)."""
    pb = scenes.tiny(3, n_points=0, n_agents=4, n_steps=20)
    C, J, dtc = 5, 7, 0.004
    res = oracle.plan_loop(pb, C, J, dtc)
    assert res.best.tolist() == [0] * C and res.n_switches == 0
    dt = float(np.float32(dtc))
    ka, da = float(pb.agents.k_a[0]), float(pb.agents.d_a[0])
    h = 0.5 * dt * float(np.float32(pb.params.inv_mass))
    M = np.array([[1.0 - dt * h * ka, dt * (1.0 - h * da)], [-h * ka, 1.0 - h * da]])
    g = np.asarray(pb.query.goal, np.float64)
    x0 = np.stack([np.asarray(pb.query.p0, np.float64), np.asarray(pb.query.v0, np.float64)])   # [2, 3]
    for n in (1, 2, 13, C * J):
        Mn = np.linalg.matrix_power(M, n)
        want = np.stack([g, np.zeros(3)]) + Mn @ (x0 - np.stack([g, np.zeros(3)]))
        np.testing.assert_allclose(res.robot[n, :3], want[0], rtol=0, atol=1e-12)
        np.testing.assert_allclose(res.robot[n, 3:], want[1], rtol=0, atol=1e-10)
    assert np.all(np.isinf(res.robot_clear))


def brute_select(total, incumbent, alpha):
    """The selection rule written out: the lowest-cost agent among those below
    alpha times the incumbent's cost (all agents without an incumbent), lowest
    index on ties, NaN never chosen; the incumbent when no agent qualifies."""
    best = -1
    for i, c in enumerate(total):
        if c != c or (incumbent >= 0 and not c < alpha * total[incumbent]):
            continue
        if best < 0 or c < total[best]:
            best = i
    return best if best >= 0 else incumbent


def test_loop_selection_and_switch_count():
    """Every cycle's i* is the selection rule (brute-force pinned) applied to that
    cycle's costs with the previous i* as incumbent, and N_sw counts the changes;
    the object scene with a mixed ensemble and alpha = 0.99 switches twice."""
    pb = scenes.config2(seed=7, n_agents=24, n_steps=100, n_points=5000)
    pb.agents = scenes.multi_agents(np.random.default_rng(7), 24)
    pb.params.alpha = 0.99
    res = oracle.plan_loop(pb, 10, 10, 0.01)
    inc, sw = pb.query.incumbent, 0
    for c in range(10):
        assert res.best[c] == brute_select(res.cost[c][:, 4], inc, pb.params.alpha)
        sw += int(inc >= 0 and res.best[c] != inc)
        inc = res.best[c]
    assert res.n_switches == sw >= 2


def test_loop_translation_covariance():
    """Translating spheres, start and goal together translates the robot's path and
    leaves every selection unchanged."""
    pb = scenes.config1()
    shift = np.array([0.25, -0.5, 1.0])
    pt = copy.deepcopy(pb)
    pt.scene = scenes.Scene((pb.scene.x + shift[0]).astype(np.float32), (pb.scene.y + shift[1]).astype(np.float32),
                            (pb.scene.z + shift[2]).astype(np.float32), pb.scene.r_obs)
    pt.query.p0 = np.asarray(pb.query.p0, np.float64) + shift
    pt.query.goal = np.asarray(pb.query.goal, np.float64) + shift
    a, b = oracle.plan_loop(pb, 4, 8, 0.01), oracle.plan_loop(pt, 4, 8, 0.01)
    assert a.best.tolist() == b.best.tolist()
    # the FP32 rounding of the shifted points moves each sphere by up to 6e-8 m
    np.testing.assert_allclose(b.robot[:, :3] - shift, a.robot[:, :3], rtol=0, atol=1e-6)


# ---------------------------------------------------------------- 6-D pose agents (Eqs. 6-11 on Spin(3) x| R^3)

def _identity_pose_query():
    return scenes.PoseQuery(np.array([1, 0, 0, 0], np.float32), np.zeros(3, np.float32),
                            np.array([1, 0, 0, 0], np.float32))


def test_pose_agents_without_rotation_are_point_masses():
    """Identity start and goal rotors and no angular velocity: no torque ever acts,
    the log's translational part is p_g - p, and the pose rollout is the point-mass
    rollout (moving spheres, mixed heuristics)."""
    pb = scenes.tiny(8, n_points=200, n_agents=6, n_steps=40, moving=True)
    pb.agents = scenes.multi_agents(np.random.default_rng(4), 6)
    pa = scenes.pose_agents(np.random.default_rng(5), 6)
    a = oracle.rollout(pb)
    b = oracle.rollout_pose(pb, pa, _identity_pose_query())
    np.testing.assert_allclose(b.traj, a.traj, rtol=0, atol=1e-12)
    np.testing.assert_allclose(b.cost, a.cost, rtol=1e-10, atol=1e-12)
    assert b.best == a.best
    assert np.abs(b.rot - np.array([1.0, 0, 0, 0])).max() < 1e-15


def test_se3_exp_log():
    """exp against scipy's rotation-vector map and against numerical integration of
    the constant-twist motion (t(1) = integral of Rot(s phi) rho ds); log inverts exp."""
    from scipy.integrate import quad_vec
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(31)
    for _ in range(25):
        phi = scenes.unit_vectors(rng, 1)[0].astype(np.float64) * rng.uniform(0.0, 3.0)
        rho = rng.uniform(-1, 1, 3)
        q, t = oracle.se3_exp(phi, rho)
        x, y, z, w = Rotation.from_rotvec(phi).as_quat()
        want = np.array([w, x, y, z]) * (1 if w >= 0 else -1)
        np.testing.assert_allclose(q, want, rtol=0, atol=1e-12)
        ti, _ = quad_vec(lambda s: Rotation.from_rotvec(s * phi).apply(rho), 0.0, 1.0, epsabs=1e-13)
        np.testing.assert_allclose(t, ti, rtol=0, atol=1e-10)
        phi2, rho2 = oracle.se3_log(q, t)
        np.testing.assert_allclose(phi2, phi, rtol=0, atol=1e-10)
        np.testing.assert_allclose(rho2, rho, rtol=0, atol=1e-10)
    q, t = oracle.se3_exp(np.zeros(3), np.array([0.1, -0.2, 0.3]))       # pure translation
    np.testing.assert_allclose(q, [1, 0, 0, 0], atol=0)
    np.testing.assert_allclose(t, [0.1, -0.2, 0.3], atol=1e-15)


def test_pose_rotation_about_a_fixed_axis():
    """At the goal position with no spheres, a rotor error about a fixed axis n stays
    about n: theta follows w_k = w_{k-1} + h_r (-k_r theta_k - d_r w_{k-1}),
    theta_{k+1} = theta_k + dt w_k, whose closed form is a matrix power."""
    pb = scenes.tiny(3, n_points=0, n_agents=2, n_steps=60)
    pb.query.p0 = np.asarray(pb.query.goal, np.float32).copy()
    pb.query.v0 = np.zeros(3, np.float32)
    n = np.array([2.0, -1.0, 2.0]) / 3.0
    th0, w0 = 2.0, 1.5
    pq = scenes.PoseQuery(np.concatenate([[np.cos(th0 / 2)], np.sin(th0 / 2) * n]).astype(np.float32),
                          (w0 * n).astype(np.float32), np.array([1, 0, 0, 0], np.float32))
    pa = scenes.pose_agents(np.random.default_rng(6), 2)
    res = oracle.rollout_pose(pb, pa, pq)
    q0 = pq.q0.astype(np.float64)
    th = 2.0 * np.arctan2(np.linalg.norm(q0[1:]), q0[0])
    axis = q0[1:] / np.linalg.norm(q0[1:])
    om = float(np.dot(pq.w0.astype(np.float64), axis))
    dt = float(np.float32(pb.params.dt))
    for i in range(2):
        kr, dr, ir = (float(pa.k_r[i]), float(pa.d_r[i]), float(pa.inv_inertia_r[i]))
        h = 0.5 * dt * ir
        M = np.array([[1.0 - dt * h * kr, dt * (1.0 - h * dr)], [-h * kr, 1.0 - h * dr]])
        for k in (1, 7, 60):
            th_k, _ = np.linalg.matrix_power(M, k) @ np.array([th, om])
            want = np.concatenate([[np.cos(th_k / 2)], np.sin(th_k / 2) * axis])
            np.testing.assert_allclose(res.rot[i, k], want * np.sign(want[0]), rtol=0, atol=1e-12)
        np.testing.assert_allclose(res.traj[i], np.broadcast_to(pb.query.p0, res.traj[i].shape), atol=1e-15)


def test_pose_frame_covariance():
    """Rotating the world (spheres, start, goal, start velocity, field rotation
    vectors, start and goal rotors) rotates the trajectories and rotors and leaves
    the costs and the selection unchanged."""
    from scipy.spatial.transform import Rotation
    pb = scenes.config1()
    pa = scenes.pose_agents(np.random.default_rng(7), pb.agents.n)
    pq = scenes.pose_query(np.random.default_rng(8))
    Qr = Rotation.from_rotvec([0.3, -1.1, 0.7])
    Qm = Qr.as_matrix()
    pt = copy.deepcopy(pb)
    P = Qm @ np.stack([pb.scene.x, pb.scene.y, pb.scene.z]).astype(np.float64)
    pt.scene = scenes.Scene(*(P[a].astype(np.float32) for a in range(3)), pb.scene.r_obs)
    pt.query.p0 = Qm @ np.asarray(pb.query.p0, np.float64)
    pt.query.goal = Qm @ np.asarray(pb.query.goal, np.float64)
    pt.query.v0 = Qm @ np.asarray(pb.query.v0, np.float64)
    pt.agents.omega = (pb.agents.omega.astype(np.float64) @ Qm.T).astype(np.float32)
    qw = lambda q: np.array([q[3], q[0], q[1], q[2]])
    rq = lambda q: (Qr * Rotation.from_quat([q[1], q[2], q[3], q[0]])).as_quat()
    ptq = scenes.PoseQuery(qw(rq(pq.q0.astype(np.float64))), pq.w0, qw(rq(pq.qg.astype(np.float64))))
    a = oracle.rollout_pose(pb, pa, pq)
    b = oracle.rollout_pose(pt, pa, ptq)
    assert a.best == b.best
    # the FP32 rounding of the rotated spheres, field rotation vectors and rotors moves inputs by ~6e-8
    np.testing.assert_allclose(b.traj, a.traj @ Qm.T, rtol=0, atol=2e-6)
    np.testing.assert_allclose(b.cost, a.cost, rtol=0, atol=2e-5)
    for i in range(pb.agents.n):
        r = qw(rq(a.rot[i, -1]))
        assert min(np.abs(b.rot[i, -1] - r).max(), np.abs(b.rot[i, -1] + r).max()) < 2e-6


# ---------------------------------------------------------------- arm agents (Eqs. 12-14)

def test_arm_forward_kinematics_composition():
    """M(q) against the chain composed with scipy rotations: R = R_0 Rz(q_1) R_1 ...,
    p = sum of each link offset rotated by the rotation accumulated before it."""
    from scipy.spatial.transform import Rotation
    from oracle import arm as oa
    L = scenes.arm_links(base=(0.1, -0.2, 0.05)).astype(np.float64)
    rng = np.random.default_rng(41)
    rq = lambda r: Rotation.from_quat([r[1], r[2], r[3], r[0]])
    for _ in range(10):
        q = rng.uniform(-2.5, 2.5, 7)
        R = rq(L[0])
        p = L[0, 4:7].copy()
        for i in range(7):
            R = R * Rotation.from_rotvec([0.0, 0.0, q[i]])
            p = p + R.apply(L[i + 1, 4:7])
            R = R * rq(L[i + 1])
        T = oa.fk(L.astype(np.float32), q)
        np.testing.assert_allclose(T[:3, 3], p, rtol=0, atol=1e-12)
        np.testing.assert_allclose(T[:3, :3], R.as_matrix(), rtol=0, atol=1e-12)


def test_arm_jacobian_and_pseudo_inverse():
    """The world Jacobian against central differences of M(q) (position, and the
    rotation vector of R(q + h e_i) R(q)^T), and J J^+ = I for the undamped
    pseudo-inverse J^T (J J^T)^-1."""
    from scipy.spatial.transform import Rotation
    from oracle import arm as oa
    L = scenes.arm_links()
    rng = np.random.default_rng(42)
    for _ in range(5):
        q = scenes.ARM_Q0.astype(np.float64) + rng.uniform(-0.5, 0.5, 7)
        J = oa.jacobian(L, q)
        T = oa.fk(L, q)
        h = 1e-6
        for i in range(7):
            e = np.zeros(7); e[i] = h
            Tp, Tm = oa.fk(L, q + e), oa.fk(L, q - e)
            np.testing.assert_allclose((Tp[:3, 3] - Tm[:3, 3]) / (2 * h), J[3:, i], rtol=0, atol=1e-7)
            w = Rotation.from_matrix(Tp[:3, :3] @ Tm[:3, :3].T).as_rotvec() / (2 * h)
            np.testing.assert_allclose(w, J[:3, i], rtol=0, atol=1e-7)
        Jp = J.T @ np.linalg.inv(J @ J.T)
        np.testing.assert_allclose(J @ Jp, np.eye(6), rtol=0, atol=1e-10)
        assert T.shape == (4, 4)


def test_arm_follows_the_pose_agent():
    """Undamped, the joint step realises the commanded twist to first order in dt:
    one step of the arm's hand matches the 6-D pose agent started at the same pose
    to second order, and over a fixed horizon the gap is first order in dt (halving
    dt halves it), i.e. both integrate the same motion."""
    from oracle import arm as oa

    def gap(n_steps, dt):
        pb, pa, pq, L, q0 = scenes.arm_problem(n_steps=n_steps)
        pb.params.dt = dt
        ra = oa.rollout_arm(pb, pa, pq, L, q0, 0.0)
        T = oa.fk(L, q0)
        pp = copy.deepcopy(pb)
        pp.query.p0 = T[:3, 3]
        rp = oracle.rollout_pose(pp, pa, scenes.PoseQuery(oa._mat_quat(T[:3, :3]), pq.w0, pq.qg))
        assert np.abs(ra["traj"][:, 1:] - ra["traj"][:, :1]).max() > 1e-3      # the hands do move
        return np.abs(ra["traj"] - rp.traj).max(axis=(0, 2))

    g1 = gap(40, 1e-3)
    assert g1[1] < 1e-7
    g2 = gap(80, 5e-4)
    ratio = g1[-1] / g2[-1]
    assert 1.6 < ratio < 2.5, ratio
