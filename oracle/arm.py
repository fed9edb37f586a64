"""FP64 oracle for arm agents (Sec. IV-A, Eqs. 12-14) -- TEST INFRASTRUCTURE ONLY.

  fk(links, q)              end-effector pose of the serial chain
                            M(q) = L_0 Rz(q_1) L_1 ... Rz(q_n) L_n as a 4x4 matrix
  jacobian(links, q)        world ("hybrid") Jacobian [6, n]: column i is
                            (z_i, z_i x (p - o_i)) for joint i's axis z_i and origin o_i
  rollout_arm(...)          one planning cycle of arm agents: the wrench and twist of
                            the 6-D pose agents (Eqs. 6-10) at M(q), then
                            qdot = J_b^T (J_b J_b^T + lambda^2 I)^-1 v (Eq. 12, body
                            Jacobian J_b = diag(R^T, R^T) J), q += dt qdot (Eq. 13),
                            M = M(q) (Eq. 14); costs and selection as the rollout

Plain numpy with 4x4 homogeneous matrices; the repulsive force comes from the C
oracle (repulsion) and the SE(3) logarithm from se3_log.
"""
import copy

import numpy as np

from . import costs, repulsion, se3_log, select


def _quat_mat(q):
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(np.asarray(q, np.float64))
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _mat_quat(R):
    from scipy.spatial.transform import Rotation
    x, y, z, w = Rotation.from_matrix(R).as_quat()
    q = np.array([w, x, y, z])
    return q if q[0] >= 0 else -q


def _link(row):
    T = np.eye(4)
    T[:3, :3] = _quat_mat(row[:4])
    T[:3, 3] = np.asarray(row[4:7], np.float64)
    return T


def _rz(a):
    T = np.eye(4)
    c, s = np.cos(a), np.sin(a)
    T[:2, :2] = [[c, -s], [s, c]]
    return T


def frames(links, q):
    """Joint frames (before each joint's rotation) and the end-effector pose."""
    L = np.asarray(links, np.float32).astype(np.float64)
    T = _link(L[0])
    out = []
    for i, a in enumerate(np.asarray(q, np.float64)):
        out.append(T.copy())
        T = T @ _rz(a) @ _link(L[i + 1])
    return out, T


def fk(links, q):
    return frames(links, q)[1]


def jacobian(links, q):
    F, T = frames(links, q)
    p = T[:3, 3]
    cols = []
    for Fi in F:
        z, o = Fi[:3, 2], Fi[:3, 3]
        cols.append(np.concatenate([z, np.cross(z, p - o)]))
    return np.array(cols).T


def rollout_arm(problem, pose_agents, pose_query, links, q0, damping):
    """Arm agents for one planning cycle: traj [N_a, N_k+1, 3], rot [N_a, N_k+1, 4],
    joints [N_a, N_k+1, n], cost [N_a, 5], min_clear [N_a, N_k], best."""
    pb = problem
    ag, q, prm = pb.agents, pb.query, pb.params
    N, na = int(prm.n_steps), ag.n
    n = len(q0)
    dt = float(np.float32(prm.dt))
    invm = float(np.float32(prm.inv_mass))
    lam2 = float(np.float32(damping)) ** 2
    goal = np.asarray(q.goal, np.float32).astype(np.float64)
    Rg = _quat_mat(np.asarray(pose_query.qg, np.float32).astype(np.float64))
    t0 = float(np.float32(q.t0))
    traj = np.zeros((na, N + 1, 3)); rot = np.zeros((na, N + 1, 4)); jts = np.zeros((na, N + 1, n))
    mc = np.zeros((na, N)); cost = np.zeros((na, 5))
    for i in range(na):
        one = copy.deepcopy(pb)
        one.agents = ag.subset([i])
        ka, da = float(ag.k_a[i]), float(ag.d_a[i])
        kr, dr, ir = (float(pose_agents.k_r[i]), float(pose_agents.d_r[i]), float(pose_agents.inv_inertia_r[i]))
        qj = np.asarray(q0, np.float32).astype(np.float64)
        T = fk(links, qj)
        R, p = T[:3, :3], T[:3, 3].copy()
        om = np.asarray(pose_query.w0, np.float32).astype(np.float64)
        u = R.T @ np.asarray(q.v0, np.float32).astype(np.float64)
        traj[i, 0], rot[i, 0], jts[i, 0] = p, _mat_quat(R), qj
        for k in range(1, N + 1):
            r = repulsion(one, p[None], (R @ u)[None], t0 + (k - 1) * dt, diagnostics=False)
            mc[i, k - 1] = r.rho_min[0]
            phi, rho = se3_log(_mat_quat(R.T @ Rg), R.T @ (goal - p))           # e = log(M^-1 M_g)
            Fa = kr * phi - dr * om                                               # Eqs. (6), (7)
            Fl = ka * rho - da * u + R.T @ r.force[0]
            om = om + 0.5 * dt * ir * Fa                                          # Eqs. (9), (10)
            u = u + 0.5 * dt * invm * Fl
            J = jacobian(links, qj)                                               # Eq. (12)
            vh = np.concatenate([R @ om, R @ u])
            qd = J.T @ np.linalg.solve(J @ J.T + lam2 * np.eye(6), vh)
            qj = qj + dt * qd                                                     # Eq. (13)
            T = fk(links, qj)                                                     # Eq. (14)
            R, p = T[:3, :3], T[:3, 3].copy()
            traj[i, k], rot[i, k], jts[i, k] = p, _mat_quat(R), qj
        cost[i] = costs(traj[i, :N], mc[i], goal, prm)
    return dict(traj=traj, rot=rot, joints=jts, cost=cost, min_clear=mc,
                best=select(cost[:, 4], int(q.incumbent), float(np.float32(prm.alpha))))
