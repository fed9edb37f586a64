"""FP64 CPU oracle for the G-MAPP rollout -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg import
this package.  The HIP library never calls it and shares no code with it; the
only common module is the seeded input generator (paper_2606_12579_amd.scenes),
which holds none of the method's arithmetic.

  rollout(problem)          Eqs. (6)-(11), (15)-(20) and the selection rule, C code
  repulsion(problem, p, v, t)  Alg. 1's response for given agent states (teacher forcing)
  rollout_grad(problem)     dC_i/d(k_a, d_a, k_f, omega) by dual numbers (C code)
  costs(...)                Eqs. (16)-(20) on a given trajectory
  select(...)               the selection rule
  plan_loop(problem, ...)   the closed planning loop: rollouts, selection across cycles, control steps
  rollout_pose(...)         6-D pose agents in Spin(3) x| R^3 (C code); se3_exp / se3_log
  perception.*              back-projection and voxel-centre sphere world (numpy)
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

from . import build as _build

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(_build.ensure_built())
        lib.oracle_rollout.restype = ctypes.c_int
        lib.oracle_rollout.argtypes = [ctypes.c_long, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int, _ip, _dp,
                                       ctypes.c_int, _dp, _dp, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int,
                                       _dp, _dp, _dp, _dp, _dp, _dp, _ip]
        lib.oracle_repulsion.restype = ctypes.c_int
        lib.oracle_repulsion.argtypes = [ctypes.c_long, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int, _ip, _dp,
                                         ctypes.c_int, _dp, _dp, _dp, ctypes.c_double, _dp, ctypes.c_int, ctypes.c_int,
                                         _dp]
        lib.oracle_rollout_grad.restype = ctypes.c_int
        lib.oracle_rollout_grad.argtypes = [ctypes.c_long, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int, _ip, _dp,
                                            ctypes.c_int, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int, _dp]
        lib.oracle_costs.restype = None
        lib.oracle_costs.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        lib.oracle_select.restype = ctypes.c_int
        lib.oracle_select.argtypes = [ctypes.c_int, _dp, ctypes.c_int, ctypes.c_double]
        lib.oracle_pair_force.restype = None
        lib.oracle_pair_force.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_int, ctypes.c_double, _dp, _dp]
        lib.oracle_pair_force_h.restype = None
        lib.oracle_pair_force_h.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double, _dp, _dp]
        lib.oracle_rollout_pose.restype = ctypes.c_int
        lib.oracle_rollout_pose.argtypes = [ctypes.c_long, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int, _ip, _dp,
                                            ctypes.c_int, _dp, _dp, _dp, _dp, ctypes.c_int, _dp, ctypes.c_int,
                                            ctypes.c_int, _dp, _dp, _dp, _dp, _ip]
        lib.oracle_se3_exp.restype = None
        lib.oracle_se3_exp.argtypes = [_dp, _dp, _dp, _dp]
        lib.oracle_se3_log.restype = None
        lib.oracle_se3_log.argtypes = [_dp, _dp, _dp, _dp]
        _lib = lib
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


def _params_row(prm) -> np.ndarray:
    # widen the FP32 values the HIP path receives, so both sides see the same numbers
    f = lambda x: float(np.float32(x))
    return np.array([f(prm.dt), f(prm.inv_mass), f(prm.eps), f(prm.r_cost), f(prm.w[0]), f(prm.w[1]), f(prm.w[2]),
                     f(prm.w[3]), f(prm.a_max), f(prm.alpha), f(prm.taper_band)], np.float64)


def _agents_rows(ag) -> np.ndarray:
    if ag.n == 0:
        return np.zeros((0, 9))
    heur = getattr(ag, "heuristic", None)
    heur = np.zeros(ag.n) if heur is None else np.asarray(heur, np.float64)
    return np.stack([ag.k_a, ag.d_a, ag.k_f, ag.r_d, ag.r_a, ag.omega[:, 0], ag.omega[:, 1], ag.omega[:, 2], heur],
                    1).astype(np.float64)


def _scene_args(sc):
    keep = []
    x, px = _d(sc.x); y, py = _d(sc.y); z, pz = _d(sc.z)
    keep += [x, y, z]
    if sc.n_seg > 0:
        sb, psb = _i(sc.seg_begin); sv, psv = _d(sc.seg_vel)
        keep += [sb, sv]
    else:
        psb, psv = ctypes.cast(None, _ip), ctypes.cast(None, _dp)
    return keep, (ctypes.c_long(sc.n), px, py, pz, ctypes.c_double(float(np.float32(sc.r_obs))),
                  ctypes.c_int(sc.n_seg), psb, psv)


@dataclasses.dataclass
class RolloutResult:
    traj: np.ndarray       # [N_a, N_k + 1, 3]  p^(1..N_k+1)
    cost: np.ndarray       # [N_a, 5] goal, obs, path, smooth, total
    min_clear: np.ndarray  # [N_a, N_k]        rho_min^(k)
    force: np.ndarray      # [N_a, N_k, 3]     F_r^(k)
    vel: np.ndarray        # [N_a, N_k + 1, 3] v^(0..N_k)
    ftot: np.ndarray       # [N_a, N_k, 3]     F^(k)
    best: int


def rollout(problem) -> RolloutResult:
    lib = _load()
    sc, ag, q, prm = problem.scene, problem.agents, problem.query, problem.params
    N, na = int(prm.n_steps), ag.n
    keep, sargs = _scene_args(sc)
    A, pA = _d(_agents_rows(ag))
    Q, pQ = _d(np.concatenate([q.p0, q.v0, q.goal, [np.float32(q.t0)]]).astype(np.float64))
    P, pP = _d(_params_row(prm))
    traj = np.zeros((na, N + 1, 3)); cost = np.zeros((na, 5)); mc = np.zeros((na, N))
    force = np.zeros((na, N, 3)); vel = np.zeros((na, N + 1, 3)); ftot = np.zeros((na, N, 3))
    best = ctypes.c_int(-1)
    rc = lib.oracle_rollout(*sargs, na, pA, pQ, int(q.incumbent), pP, N, int(prm.cutoff),
                            traj.ctypes.data_as(_dp), cost.ctypes.data_as(_dp), mc.ctypes.data_as(_dp),
                            force.ctypes.data_as(_dp), vel.ctypes.data_as(_dp), ftot.ctypes.data_as(_dp),
                            ctypes.byref(best))
    if rc != 0:
        raise RuntimeError(f"oracle_rollout failed ({rc})")
    del keep
    return RolloutResult(traj, cost, mc, force, vel, ftot, best.value)


@dataclasses.dataclass
class RepulsionResult:
    force: np.ndarray      # [N_a, 3]
    rho_min: np.ndarray    # [N_a]
    abs_sum: np.ndarray    # [N_a] sum_j |f_j|
    edge_sum: np.ndarray   # [N_a] force magnitude of pairs at the hard cut-off (within 1e-6 r_d)
    edge_cnt: np.ndarray   # [N_a]
    term_sum: np.ndarray   # [N_a] sum over pairs of the magnitudes of the terms of each pair force
    shift_sum: np.ndarray  # [N_a] sum over moving pairs of |f_j| changes when p - t v_seg is rounded to FP32


def repulsion(problem, p, v, t, diagnostics=True) -> RepulsionResult:
    """Alg. 1's response for each agent at positions p [N_a,3], velocities v [N_a,3], time t; with
    diagnostics, the terms of the force tolerance too (zeros without)."""
    lib = _load()
    sc, ag, prm = problem.scene, problem.agents, problem.params
    keep, sargs = _scene_args(sc)
    A, pA = _d(_agents_rows(ag))
    pp, ppp = _d(np.asarray(p, np.float64).reshape(-1, 3))
    vv, pvv = _d(np.asarray(v, np.float64).reshape(-1, 3))
    P, pP = _d(_params_row(prm))
    out = np.zeros((ag.n, 9))
    lib.oracle_repulsion(*sargs, ag.n, pA, ppp, pvv, float(t), pP, int(prm.cutoff), int(bool(diagnostics)),
                         out.ctypes.data_as(_dp))
    del keep
    return RepulsionResult(out[:, :3].copy(), out[:, 3].copy(), out[:, 4].copy(), out[:, 5].copy(),
                           out[:, 6].astype(np.int64), out[:, 7].copy(), out[:, 8].copy())


def rollout_grad(problem) -> np.ndarray:
    """[N_a, 7]: C_i, then dC_i/d(k_a, d_a, k_f, omega_x, omega_y, omega_z)."""
    lib = _load()
    sc, ag, q, prm = problem.scene, problem.agents, problem.query, problem.params
    if getattr(ag, "heuristic", None) is not None and np.any(np.asarray(ag.heuristic) != 0):
        raise ValueError("the dual-number gradient covers the rotation-vector circular field only")
    keep, sargs = _scene_args(sc)
    A, pA = _d(_agents_rows(ag))
    Q, pQ = _d(np.concatenate([q.p0, q.v0, q.goal, [np.float32(q.t0)]]).astype(np.float64))
    P, pP = _d(_params_row(prm))
    out = np.zeros((ag.n, 7))
    rc = lib.oracle_rollout_grad(*sargs, ag.n, pA, pQ, pP, int(prm.n_steps), int(prm.cutoff),
                                 out.ctypes.data_as(_dp))
    if rc != 0:
        raise RuntimeError(f"oracle_rollout_grad failed ({rc})")
    del keep
    return out


def costs(pos, rmin, goal, params) -> np.ndarray:
    """Eqs. (16)-(20) for one trajectory pos [N,3] = p^(1..N), rmin [N]."""
    lib = _load()
    pos, ppos = _d(np.asarray(pos).reshape(-1, 3))
    rm, prm_ = _d(rmin)
    g, pg = _d(goal)
    P, pP = _d(_params_row(params))
    out = np.zeros(5)
    lib.oracle_costs(int(pos.shape[0]), ppos, prm_, pg, pP, out.ctypes.data_as(_dp))
    return out


def select(total, incumbent=-1, alpha=0.9) -> int:
    lib = _load()
    t, pt = _d(total)
    return int(lib.oracle_select(int(t.shape[0]), pt, int(incumbent), float(alpha)))


def pair_force(p, w, q, omega, k_f, r_d, R, eps, cutoff=0, band=0.1):
    lib = _load()
    arrs = [_d(a) for a in (p, w, q, omega)]
    f = np.zeros(3)
    rho = ctypes.c_double()
    lib.oracle_pair_force(*[a[1] for a in arrs], float(k_f), float(r_d), float(R), float(eps), int(cutoff),
                          float(band), f.ctypes.data_as(_dp), ctypes.byref(rho))
    return f, rho.value


def pair_force_heuristic(heur, p, w, q, omega, k_f, r_d, R, eps, cutoff=0, band=0.1):
    """One pair of Sec. III-A's heuristics: 0 rotation-vector circular field, 1 the
    field with the relative-velocity current (Eq. 3), 2 artificial potential field (Eq. 1)."""
    lib = _load()
    arrs = [_d(a) for a in (p, w, q, omega)]
    f = np.zeros(3)
    rho = ctypes.c_double()
    lib.oracle_pair_force_h(int(heur), *[a[1] for a in arrs], float(k_f), float(r_d), float(R), float(eps),
                            int(cutoff), float(band), f.ctypes.data_as(_dp), ctypes.byref(rho))
    return f, rho.value


@dataclasses.dataclass
class PoseResult:
    traj: np.ndarray       # [N_a, N_k + 1, 3]
    rot: np.ndarray        # [N_a, N_k + 1, 4] unit quaternions (w, x, y, z), w >= 0
    cost: np.ndarray       # [N_a, 5]
    min_clear: np.ndarray  # [N_a, N_k]
    best: int


def rollout_pose(problem, pose_agents, pose_query) -> PoseResult:
    """6-D pose agents (Eqs. 6-11 on Spin(3) x| R^3) for one planning cycle."""
    lib = _load()
    sc, ag, q, prm = problem.scene, problem.agents, problem.query, problem.params
    N, na = int(prm.n_steps), ag.n
    keep, sargs = _scene_args(sc)
    A, pA = _d(_agents_rows(ag))
    G, pG = _d(np.stack([pose_agents.k_r, pose_agents.d_r, pose_agents.inv_inertia_r], 1).reshape(-1, 3)
               if na else np.zeros((0, 3)))
    Q, pQ = _d(np.concatenate([q.p0, q.v0, q.goal, [np.float32(q.t0)]]).astype(np.float64))
    PQ, pPQ = _d(np.concatenate([pose_query.q0, pose_query.w0, pose_query.qg]).astype(np.float32))
    P, pP = _d(_params_row(prm))
    traj = np.zeros((na, N + 1, 3)); rot = np.zeros((na, N + 1, 4)); cost = np.zeros((na, 5))
    mc = np.zeros((na, N))
    best = ctypes.c_int(-1)
    rc = lib.oracle_rollout_pose(*sargs, na, pA, pG, pQ, pPQ, int(q.incumbent), pP, N, int(prm.cutoff),
                                 traj.ctypes.data_as(_dp), rot.ctypes.data_as(_dp), cost.ctypes.data_as(_dp),
                                 mc.ctypes.data_as(_dp), ctypes.byref(best))
    if rc != 0:
        raise RuntimeError(f"oracle_rollout_pose failed ({rc})")
    del keep
    return PoseResult(traj, rot, cost, mc, best.value)


def se3_exp(phi, rho):
    """SE(3) exponential: (unit quaternion with w >= 0, translation)."""
    lib = _load()
    (a, pa), (b, pb) = _d(phi), _d(rho)
    q, t = np.zeros(4), np.zeros(3)
    lib.oracle_se3_exp(pa, pb, q.ctypes.data_as(_dp), t.ctypes.data_as(_dp))
    return q, t


def se3_log(q, t):
    """SE(3) logarithm: (rotation vector of angle <= pi, J(phi)^-1 t)."""
    lib = _load()
    (a, pa), (b, pb) = _d(q), _d(t)
    phi, rho = np.zeros(3), np.zeros(3)
    lib.oracle_se3_log(pa, pb, phi.ctypes.data_as(_dp), rho.ctypes.data_as(_dp))
    return phi, rho


@dataclasses.dataclass
class LoopResult:
    robot: np.ndarray        # [n_cycles * ctrl_steps + 1, 6] p, v of the robot
    robot_clear: np.ndarray  # [n_cycles * ctrl_steps] rho_min at each control step
    best: np.ndarray         # [n_cycles] i* of each cycle
    cost: np.ndarray         # [n_cycles, N_a, 5]
    n_switches: int          # N_sw
    t0: np.ndarray           # [n_cycles] start time of each cycle (FP32 values)


def plan_loop(problem, n_cycles, ctrl_steps, ctrl_dt) -> LoopResult:
    """The closed planning loop (Sec. V-B) with a point-mass robot, in the order
    the paper describes it.  Each cycle c:
      1. takes the robot's current state as the start of every agent and rolls all
         agents out over N_k steps (rollout above: Eqs. 6-11 and 15-20), selecting
         i* with the rule of Sec. IV-A against the incumbent, the previous cycle's
         i* (the query's incumbent at c = 0); the cycle starts at
         t0_c = t0 + c ctrl_steps ctrl_dt, rounded to FP32 like every time input;
      2. counts an agent switch when i* differs from a valid previous i*;
      3. moves the robot ctrl_steps control steps under i*: at step j the repulsive
         force of i*'s own field at the robot's state and time t0_c + j ctrl_dt
         (repulsion above, for that agent alone), the attractor of Eq. (7) with
         i*'s gains, and the explicit integration of Eqs. 9-11 with dt = ctrl_dt.
    A negative i* (no agents) leaves the robot where it is for that cycle."""
    import copy
    pb = copy.deepcopy(problem)
    ag, q, prm = pb.agents, pb.query, pb.params
    dt_c = float(np.float32(ctrl_dt))
    h = 0.5 * dt_c * float(np.float32(prm.inv_mass))
    goal = np.asarray(q.goal, np.float64)
    p = np.asarray(q.p0, np.float64).copy()
    v = np.asarray(q.v0, np.float64).copy()
    inc = int(q.incumbent)
    t0 = float(np.float32(q.t0))
    robot = [np.concatenate([p, v])]
    clear, best, cost, t0s = [], [], [], []
    n_sw = 0
    for c in range(int(n_cycles)):
        t0c = float(np.float32(t0 + float(c) * float(ctrl_steps) * dt_c))
        t0s.append(t0c)
        q.p0, q.v0, q.t0, q.incumbent = p.copy(), v.copy(), t0c, inc
        r = rollout(pb)
        i = int(r.best)
        best.append(i)
        cost.append(r.cost)
        if inc >= 0 and i >= 0 and i != inc:
            n_sw += 1
        one = copy.deepcopy(pb)
        if 0 <= i < ag.n:
            one.agents = ag.subset([i])
            k_a, d_a = float(np.float32(ag.k_a[i])), float(np.float32(ag.d_a[i]))
        for j in range(int(ctrl_steps)):
            if not 0 <= i < ag.n:
                robot.append(robot[-1].copy())
                clear.append(np.nan)
                continue
            t = t0c + j * dt_c
            rep = repulsion(one, p[None], v[None], t, diagnostics=False)
            F = k_a * (goal - p) - d_a * v + rep.force[0]
            v = v + h * F
            p = p + dt_c * v
            robot.append(np.concatenate([p, v]))
            clear.append(float(rep.rho_min[0]))
        inc = i
    return LoopResult(np.array(robot), np.array(clear), np.array(best, np.int64), np.array(cost), n_sw,
                      np.array(t0s))


def interactions(problem) -> int:
    return problem.agents.n * problem.params.n_steps * problem.scene.n


def n_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
