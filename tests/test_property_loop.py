"""Property sweeps on the GPU for heterogeneous ensembles and the closed planning loop.

Heterogeneous ensembles (Sec. III-A's heuristics mixed in one launch): random tiny
problems in which every agent draws its own heuristic (rotation-vector circular field,
velocity-current field, APF), detection radius r_d and gain k_f, under random tilings,
against the FP64 oracle: trajectories and costs (each agent to the bar of its
conditioning), the selection rule, and the teacher-forced response of every heuristic
at the oracle's own states of the first and the last step.

Closed loop (Sec. V-B): random tiny scenes, ensembles (homogeneous or mixed), cycle
counts, control steps, control periods, start times, hysteresis factors and incumbents.
Every cycle is checked from the robot state the device itself carried into it (an FP32
value the oracle can start from exactly), so that one cycle's rounding does not
compound through the next cycles' chaotic dynamics:
  - the costs of every well-conditioned agent against the oracle's rollout from that
    state (positions known to 1e-4 m fix them to the bounds of the rollout tests);
  - i* is the selection rule applied to the device's own costs against the device's
    previous i*; with those costs within the bounds above, any i* the oracle's rule
    picks on a cost vector inside those bounds is correct, which covers near ties;
  - the robot's control steps under that i* against the oracle's loop run with that
    agent alone, from the same state: positions, velocities and clearances (steps that
    one FP32 ulp of the agent's rotation vector, or 1e-5 of its gain, moves by more than
    1e-4 m are held to twice that spread);
  - N_sw counts the changes of i* from a valid previous i*."""
import copy

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_2606_12579_amd import scenes
from tests import gpu_util as gu
from tests.test_property import TILINGS, _problem

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


def _mix(pb, rng):
    """Per-agent heuristic, detection radius U[0.02, 0.2] m and gain (the heuristic's default scaled by
    U[0.5, 2])."""
    n = pb.agents.n
    ag = pb.agents
    ag.heuristic = rng.integers(0, 3, n).astype(np.int32)
    ag.r_d = rng.uniform(0.02, 0.2, n).astype(np.float32)
    base = np.where(ag.heuristic == scenes.H_APF, scenes.K_F_APF, scenes.K_F)
    ag.k_f = (base * rng.uniform(0.5, 2.0, n)).astype(np.float32)
    return pb


@settings(max_examples=80, **SETTINGS)
@given(seed=st.integers(0, 2 ** 31 - 1), n_o=st.integers(0, 64), n_a=st.integers(1, 8), n_k=st.integers(1, 20),
       moving=st.booleans(), cutoff=st.integers(0, 1), coincide=st.booleans(), on_centre=st.booleans(),
       tiling=st.sampled_from(TILINGS))
def test_random_mixed_ensembles(ctx, seed, n_o, n_a, n_k, moving, cutoff, coincide, on_centre, tiling):
    import torch
    from paper_2606_12579_amd import gmapp
    pb = _mix(_problem(seed, n_o, n_a, n_k, moving, cutoff, coincide, on_centre), np.random.default_rng(seed + 1))
    print(f"seed {seed} N_O {n_o} N_a {n_a} N_k {n_k} moving {moving} cutoff {cutoff} coincide {coincide} "
          f"on_centre {on_centre} tiling {tiling} heuristics {pb.agents.heuristic.tolist()}", flush=True)
    gpu = gu.gpu_rollout(ctx, pb, tiling=tiling)
    worst, n_ill = gu.compare_conditioned(pb, gpu, np.arange(n_a), label=f"seed {seed}")
    ref = oracle.rollout(pb)
    gu.check_selection(gpu["best"], ref.cost, gpu["cost"])
    sc, ag = gmapp.scene_to_device(pb.scene), gmapp.agents_to_device(pb.agents)
    for k in sorted({1, n_k}):
        p32 = ref.traj[:, k - 1].astype(np.float32)
        v32 = ref.vel[:, k - 1].astype(np.float32)
        t32 = np.float32((k - 1) * np.float32(pb.params.dt))
        r = oracle.repulsion(pb, p32.astype(np.float64), v32.astype(np.float64), float(t32))
        f, rho = ctx.force_probe(sc, ag, torch.as_tensor(p32, device="cuda"), torch.as_tensor(v32, device="cuda"),
                                 float(t32), pb.params)
        torch.cuda.synchronize()
        d = np.linalg.norm(f.cpu().numpy().astype(np.float64) - r.force, axis=1)
        assert (d <= gu.force_bound(r) + 1e-30).all(), (k, d, gu.force_bound(r))
    print(f"  worst position error {worst:.2e} m, ill-conditioned agents {n_ill}", flush=True)


def _select(total, incumbent, alpha):
    """The selection rule of Sec. IV-A on FP32 costs: the cheapest agent whose cost is finite and, with a
    valid incumbent, below alpha times the incumbent's; else the incumbent."""
    t = np.asarray(total, np.float32)
    n = len(t)
    inc_ok = 0 <= incumbent < n
    bound = np.float32(np.float32(alpha) * t[incumbent]) if inc_ok else np.float32(np.inf)
    best = -1
    for i in range(n):
        if np.isnan(t[i]) or (inc_ok and not t[i] < bound):
            continue
        if best < 0 or t[i] < t[best]:
            best = i
    return incumbent if best < 0 and inc_ok else best


def _control_spread(one, J, ctrl_dt, ref):
    """Largest change of the robot's position and velocity at each control step when the one agent's rotation
    vector moves by one FP32 ulp either way or its gain k_f by 1e-5 relative (the perturbations of reading R24)."""
    ps, vs = np.zeros(J + 1), np.zeros(J + 1)
    for dw, kf in ((1, 1.0), (-1, 1.0), (0, 1.0 + 1e-5), (0, 1.0 - 1e-5)):
        q = copy.deepcopy(one)
        w = q.agents.omega.astype(np.float32)
        if dw:
            w = np.nextafter(w, np.float32(np.inf * dw))
        q.agents.omega = np.ascontiguousarray(w)
        q.agents.k_f = (q.agents.k_f.astype(np.float64) * kf).astype(np.float32)
        r = oracle.plan_loop(q, 1, J, ctrl_dt)
        ps = np.maximum(ps, np.abs(r.robot[:, :3] - ref.robot[:, :3]).max(1))
        vs = np.maximum(vs, np.abs(r.robot[:, 3:] - ref.robot[:, 3:]).max(1))
    return ps, vs


LOOP_TILINGS = [None, (1, 8, 4, 0, 0, 2), (2, 1, 2, 0, 1, 1), (4, 4, 1, 64, 2, 1), (8, 2, 2, 0, 0, 1),
                (1, 4, 8, 0, 1, 2)]


@settings(max_examples=40, **SETTINGS)
@given(seed=st.integers(0, 2 ** 31 - 1), n_o=st.integers(0, 64), n_a=st.integers(1, 8), n_k=st.integers(1, 20),
       moving=st.booleans(), cutoff=st.integers(0, 1), mixed=st.booleans(), n_cycles=st.integers(1, 6),
       ctrl_steps=st.integers(1, 8), ctrl_dt=st.sampled_from([0.001, 0.005, 0.01]),
       alpha=st.sampled_from([0.5, 0.9, 0.99, 1.0]), t0=st.floats(0.0, 0.05),
       incumbent=st.integers(-1, 7), tiling=st.sampled_from(LOOP_TILINGS))
def test_random_planning_loops(ctx, seed, n_o, n_a, n_k, moving, cutoff, mixed, n_cycles, ctrl_steps, ctrl_dt,
                               alpha, t0, incumbent, tiling):
    import torch
    from paper_2606_12579_amd import gmapp
    pb = scenes.tiny(seed, n_points=n_o, n_agents=n_a, n_steps=n_k, moving=moving and n_o > 0, cutoff=cutoff)
    if mixed:
        pb = _mix(pb, np.random.default_rng(seed + 2))
    pb.params.alpha = alpha
    t0 = float(np.float32(t0))
    pb.query.t0 = t0
    pb.query.incumbent = min(incumbent, n_a - 1)
    C, J = n_cycles, ctrl_steps
    print(f"seed {seed} N_O {n_o} N_a {n_a} N_k {n_k} moving {moving} cutoff {cutoff} mixed {mixed} C {C} J {J} "
          f"dt_c {ctrl_dt} alpha {alpha} t0 {t0} incumbent {pb.query.incumbent} tiling {tiling}", flush=True)
    if tiling is not None:
        ctx.set_tiling(*tiling)
    else:
        ctx.clear_tiling()
    sc, ag = gmapp.scene_to_device(pb.scene), gmapp.agents_to_device(pb.agents)
    out = ctx.plan_loop(sc, ag, pb.query, pb.params, C, J, ctrl_dt)
    torch.cuda.synchronize()
    gpu = {k: v.cpu().numpy() for k, v in out.items()}
    best, robot, clear, cost = gpu["best"].astype(np.int64), gpu["robot"], gpu["robot_clear"], gpu["cost"]
    assert np.array_equal(robot[0], np.concatenate([pb.query.p0, pb.query.v0]).astype(np.float32))
    dt_c = float(np.float32(ctrl_dt))
    inc, n_sw, n_ill = int(pb.query.incumbent), 0, 0
    tol = gu.cost_tolerances(pb, gu.POS_TOL)
    for c in range(C):
        g = int(best[c])
        assert 0 <= g < n_a, (c, g)
        # the selection rule on the device's own costs
        assert g == _select(cost[c, :, 4], inc, alpha), (c, g, cost[c, :, 4].tolist(), inc)
        if inc >= 0 and g != inc:
            n_sw += 1
        # the oracle from the state the device carried into this cycle
        pc = copy.deepcopy(pb)
        s = robot[c * J].astype(np.float32)
        pc.query.p0, pc.query.v0 = s[:3].copy(), s[3:].copy()
        pc.query.t0 = float(np.float32(float(np.float32(t0)) + float(c) * float(J) * dt_c))
        pc.query.incumbent = inc
        nom, env, _ = gu.conditioning(pc, np.arange(n_a))
        good = env <= gu.POS_TOL
        n_ill += int((~good).sum())
        d = np.abs(cost[c].astype(np.float64) - nom.cost)[good]
        ref_c = nom.cost[good]
        for k in range(3):
            assert (d[:, k] <= tol[k]).all(), (c, k, d[:, k].max(), tol[k])
        assert (d[:, 3] / np.maximum(np.abs(ref_c[:, 3]), 1e-3) <= tol[3]).all(), (c, "C_smooth")
        # the robot's control steps under the device's i*, that agent alone
        one = copy.deepcopy(pc)
        one.agents = pb.agents.subset([g])
        one.query.incumbent = 0
        ref = oracle.plan_loop(one, 1, J, ctrl_dt)
        assert int(ref.best[0]) == 0
        seg = robot[c * J:(c + 1) * J + 1].astype(np.float64)
        pe = np.abs(seg[:, :3] - ref.robot[:, :3]).max(1)
        ve = np.abs(seg[:, 3:] - ref.robot[:, 3:]).max(1)
        pos_err, vel_err = float(pe.max()), float(ve.max())
        p_spread, v_spread = _control_spread(one, J, ctrl_dt, ref)
        if p_spread.max() <= gu.POS_TOL:
            assert pos_err <= gu.POS_TOL, (c, pos_err)
            assert vel_err <= 10 * gu.POS_TOL, (c, vel_err)
        else:                          # ill-conditioned control steps (reading R24): the perturbed family's bar
            n_ill += 1
            assert (pe <= np.maximum(gu.POS_TOL, 2 * np.maximum.accumulate(p_spread))).all(), (c, pe, p_spread)
            assert (ve <= np.maximum(10 * gu.POS_TOL, 2 * np.maximum.accumulate(v_spread))).all(), (c, ve, v_spread)
        rc, rr = clear[c * J:(c + 1) * J].astype(np.float64), ref.robot_clear
        fin = np.isfinite(rr)
        assert np.array_equal(np.isfinite(rc), fin), (c, rc, rr)
        if fin.any():
            assert np.abs(rc[fin] - rr[fin]).max() <= pos_err + 1e-6 + 1e-5 * rr[fin].max()
        inc = g
    assert int(gpu["n_switches"][0]) == n_sw
    print(f"  i* {best.tolist()} N_sw {n_sw} ill-conditioned agent-cycles {n_ill}", flush=True)
