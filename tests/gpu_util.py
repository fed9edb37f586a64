"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI and
compare it with the FP64 oracle: position 1e-4 m over the horizon, 1e-5 relative
teacher-forced force, costs within the bounds a position error implies."""
import numpy as np

POS_TOL = 1e-4          # m, position error over the horizon
FORCE_REL = 1e-5        # teacher-forced repulsive force, relative
SEL_GAP = 1e-6          # selection: oracle cost gap below which either index is correct


def gpu_rollout(ctx, pb, device="cuda:0", tiling=None, stream=None):
    import torch
    from paper_2606_12579_amd import gmapp
    if tiling is not None:
        ctx.set_tiling(*tiling)
    else:
        ctx.clear_tiling()
    sc = gmapp.scene_to_device(pb.scene, device)
    ag = gmapp.agents_to_device(pb.agents, device)
    out = ctx.rollout(sc, ag, pb.query, pb.params, stream=stream)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    res["best"] = int(res["best"][0])
    if pb.agents.n > 0:
        assert 0 <= res["best"] < pb.agents.n, f"best = {res['best']} (negative = device error status)"
    return res


def cost_tolerances(pb, pos_err):
    """Bounds on the cost differences implied by a position error `pos_err`.

    C_goal and C_obs average terms that are 1/r_c-Lipschitz in position; C_path is
    a ratio of lengths with L accumulated over N_k steps (FP32 rounding of each
    dt |v| term, relative 2^-24, plus the position error at both ends); C_smooth
    is relative (FP32 force differences)."""
    rc = float(np.float32(pb.params.r_cost))
    e = pos_err + 1e-6
    return np.array([1.01 * e / rc + 1e-6, 1.01 * e / rc + 1e-6, 1e-4, 2e-3, 0.0])


def path_tolerance(pb, traj, ref_traj, floor):
    """Per-agent bound on |dC_path| (Eq. 19), from the two trajectories themselves: the path length L moves by at
    most the total variation of the position error along the path, sum_k |e_k - e_(k-1)|, plus the FP32 rounding of
    the steps it sums (the device sums dt |v|, which differs from the stored position increments by one rounding of
    each position); C_path = 1 - d1/L or 1 - L/d1 then moves by at most that over min(L, d1).  Never below `floor`."""
    n = pb.params.n_steps
    g, o = traj[:, :n].astype(np.float64), ref_traj[:, :n]
    tv = np.linalg.norm(np.diff(g - o, axis=1), axis=2).sum(axis=1)
    L = np.linalg.norm(np.diff(o, axis=1), axis=2).sum(axis=1)
    d1 = np.linalg.norm(pb.query.goal.astype(np.float64) - o[:, 0], axis=1)
    scale = np.abs(o).max(axis=(1, 2)) if o.size else np.zeros(len(o))
    dL = tv + 2 * n * 2.0 ** -24 * scale + 4 * 2.0 ** -24 * L
    return np.maximum(floor, dL / np.maximum(np.minimum(L, d1), 1e-12) + 1e-6)


def check_selection(best_gpu, cost_or, cost_gpu, incumbent=-1, alpha=0.9):
    """The GPU's i* must be the oracle's, unless the oracle's cost gap to the
    GPU's choice is within max(1e-6, 2 max_i |C_gpu - C_or|)."""
    tot = cost_or[:, 4]
    if best_gpu == int(np.nanargmin(tot)) or incumbent >= 0:
        return 0.0
    allow = max(SEL_GAP, 2 * float(np.nanmax(np.abs(cost_gpu[:, 4] - tot))))
    gap = float(tot[best_gpu] - np.nanmin(tot))
    assert gap <= allow, (best_gpu, int(np.nanargmin(tot)), gap, allow)
    return gap


def compare_rollout(pb, gpu, ref, agents=None, pos_tol=POS_TOL, cost_spread=None):
    """Element-wise comparison of a GPU rollout with the oracle's (optionally on a
    subset `agents` of the GPU's agents, ref computed on that subset).  cost_spread [n, 5]:
    how far one ulp of the inputs moves each cost (reading R24); each cost is held to at
    least twice that."""
    idx = np.arange(pb.agents.n) if agents is None else np.asarray(agents)
    traj = gpu["traj"][idx].astype(np.float64)
    pos_err = float(np.abs(traj - ref.traj).max()) if traj.size else 0.0
    assert pos_err <= pos_tol, f"position error {pos_err:.3e} m"
    if gpu.get("min_clear") is not None and ref.min_clear.size:
        mc = gpu["min_clear"][idx].astype(np.float64)
        fin = np.isfinite(ref.min_clear)
        assert np.array_equal(np.isfinite(mc), fin)
        if fin.any():
            assert np.abs(mc[fin] - ref.min_clear[fin]).max() <= pos_err + 1e-6 + 1e-5 * ref.min_clear[fin].max()
    cost = gpu["cost"][idx].astype(np.float64)
    tol = cost_tolerances(pb, pos_err)
    d = np.abs(cost - ref.cost)
    spread = np.zeros_like(d) if cost_spread is None else 2.0 * np.asarray(cost_spread)
    t_goal = np.maximum(tol[0], spread[:, 0])
    t_obs = np.maximum(tol[1], spread[:, 1])
    t_path = np.maximum(path_tolerance(pb, traj, ref.traj, tol[2]), spread[:, 2])
    t_smooth = np.maximum(tol[3] * np.maximum(np.abs(ref.cost[:, 3]), 1e-3), spread[:, 3])
    assert (d[:, 0] <= t_goal).all(), ("C_goal", d[:, 0].max(), tol[0])
    assert (d[:, 1] <= t_obs).all(), ("C_obs", d[:, 1].max(), tol[1])
    assert (d[:, 2] <= t_path).all(), ("C_path", d[:, 2].max(), t_path.min())
    assert (d[:, 3] <= t_smooth).all(), ("C_smooth", (d[:, 3] / t_smooth).max())
    tot_tol = np.maximum(t_goal * abs(pb.params.w[0]) + t_obs * abs(pb.params.w[1]) + t_path * abs(pb.params.w[2])
                         + t_smooth * abs(pb.params.w[3]) + 1e-6, spread[:, 4])
    assert (d[:, 4] <= tot_tol).all(), ("C_total", d[:, 4].max())
    return pos_err


TERM_ROUNDINGS = 16     # FP32 roundings charged to the magnitude of each pair force's terms


def force_bound(r):
    """Per-agent force bound: |dF| <= 1e-5 max(|F|, 1e-2 sum_j |f_j|), plus
      - the force of pairs sitting at the hard cut-off (where FP32 and FP64 may decide
        rho <= r_d differently);
      - 16 FP32 roundings of the magnitudes of the terms each pair force is made of (where terms
        cancel -- the velocity current for motion along or across the line to a sphere centre,
        the APF's 1/rho - 1/r_d at its cut-off, the taper's argument at its outer edge -- rounding
        leaves an error of the order of the terms, not of the small result);
      - the force change when the agent's position in a moving segment's frame is rounded to
        FP32 (near a sphere centre the direction n = d / |d| amplifies that rounding)."""
    F = np.linalg.norm(r.force, axis=1)
    return (FORCE_REL * np.maximum(F, 1e-2 * r.abs_sum) + r.edge_sum + TERM_ROUNDINGS * 2.0 ** -24 * r.term_sum
            + r.shift_sum)


def conditioning(pb, idx, with_costs=False):
    """Conditioning of the sampled agents idx (reading R24), from one oracle call that runs
    each agent five times: nominal; its rotation vector moved by one FP32 ulp up and down in
    every component; its circular-field gain k_f scaled by 1 +- 1e-5 (a repulsive force off
    by the stated 1e-5 relative force tolerance at every step); and two more calls with the
    start position moved by one FP32 ulp up and down in every component.
      env[i]:       largest position change over the horizon under any of the six
                    perturbations; above 1e-4 m the agent is ill-conditioned (the exact problem
                    does not fix its FP32 trajectory to the tolerance: one ulp of its inputs, or a
                    force within the per-step tolerance, moves it further);
      env_step[i, k]: largest change of p^(k) under all six perturbations: the spread of the
                    trajectories whose every step meets the force tolerance;
      cost_spread[i, c]: largest change of cost component c under the six perturbations (with_costs).
    Returns (nominal oracle rollout of idx, env [m], env_step [m, N_k + 1][, cost_spread [m, 5]])."""
    import copy

    import oracle
    idx = np.asarray(idx)
    m = len(idx)
    sub = copy.deepcopy(pb)
    ag = pb.agents.subset(np.concatenate([idx] * 5))
    w = ag.omega.astype(np.float32)
    w[m:2 * m] = np.nextafter(w[m:2 * m], np.float32(np.inf))
    w[2 * m:3 * m] = np.nextafter(w[2 * m:3 * m], np.float32(-np.inf))
    ag.omega = np.ascontiguousarray(w)
    kf = ag.k_f.astype(np.float64)
    kf[3 * m:4 * m] *= 1.0 + 1e-5
    kf[4 * m:] *= 1.0 - 1e-5
    ag.k_f = kf.astype(np.float32)
    sub.agents = ag
    r = oracle.rollout(sub)
    nom = copy.deepcopy(r)
    for f in ("traj", "cost", "min_clear", "force", "vel", "ftot"):
        setattr(nom, f, getattr(r, f)[:m])
    dev = [np.abs(r.traj[q * m:(q + 1) * m] - r.traj[:m]).max(2) for q in range(1, 5)]
    cdev = [np.abs(r.cost[q * m:(q + 1) * m] - r.cost[:m]) for q in range(1, 5)]
    for direction in (np.inf, -np.inf):             # the start position, one FP32 ulp off
        moved = copy.deepcopy(pb)
        moved.agents = pb.agents.subset(idx)
        moved.query.p0 = np.nextafter(np.asarray(pb.query.p0, np.float32), np.float32(direction))
        rm = oracle.rollout(moved)
        dev.append(np.abs(rm.traj - r.traj[:m]).max(2))
        cdev.append(np.abs(rm.cost - r.cost[:m]))
    env_step = np.maximum.reduce(dev)
    env = env_step.max(1)
    if with_costs:
        return nom, env, env_step, np.maximum.reduce(cdev)
    return nom, env, env_step


def compare_conditioned(pb, gpu, idx, label=""):
    """Sampled agents idx of a GPU rollout against the oracle, each to its own bar: the
    well-conditioned ones (envelope <= 1e-4 m) element-wise as compare_rollout
    (positions 1e-4 m, costs); the ill-conditioned ones step by step within
    max(1e-4 m, twice the largest spread of the perturbed trajectories so far).  Returns
    (worst error of the well-conditioned agents, number of ill-conditioned agents)."""
    nom, env, env_step, cost_spread = conditioning(pb, idx, with_costs=True)
    idx = np.asarray(idx)
    err = np.abs(gpu["traj"][idx].astype(np.float64) - nom.traj).max(2)
    ill = env > POS_TOL
    # the GPU trajectory is one more member of the family the perturbations sample; past the
    # onset of divergence the members' spread saturates at the size of the region the agent
    # wanders in, so the bar is twice the running maximum of the sampled spread
    bar = np.maximum(POS_TOL, 2.0 * np.maximum.accumulate(env_step, axis=1))
    for i in np.nonzero(ill)[0]:
        k = int(np.argmax(err[i] - bar[i]))
        assert err[i, k] <= bar[i, k], (label, int(idx[i]), k, err[i, k], bar[i, k], env[i])
    worst = 0.0
    if (~ill).any():
        import copy
        good = np.nonzero(~ill)[0]
        ref = copy.deepcopy(nom)
        for f in ("traj", "cost", "min_clear", "force", "vel", "ftot"):
            setattr(ref, f, getattr(nom, f)[good])
        worst = compare_rollout(pb, gpu, ref, agents=idx[good], cost_spread=cost_spread[good])
    return worst, int(ill.sum())


def nearest_sphere_gap(pb, traj):
    """Per agent, the smallest gap between the nearest and the second-nearest sphere centre over the steps at which
    the nearest sphere is within r_c (where C_obs = mean(1 - min(rho_min, r_c) / r_c) depends on it).  At a gap of
    zero the argmin in rho_min switches spheres: the cost has a kink there and its gradient two one-sided values.
    traj: positions [N_a, >= N_k, 3] (p^(1..N_k) first)."""
    sc, prm = pb.scene, pb.params
    n_k = prm.n_steps
    out = np.full(traj.shape[0], np.inf)
    if sc.n < 2:
        return out
    P = np.stack([sc.x, sc.y, sc.z], 1).astype(np.float64)
    V = np.zeros_like(P)
    if sc.seg_begin is not None:
        for s in range(sc.n_seg):
            V[sc.seg_begin[s]:sc.seg_begin[s + 1]] = sc.seg_vel[s]
    dt = float(np.float32(prm.dt))
    t0 = float(np.float32(pb.query.t0))
    R = float(np.float32(sc.r_obs)) + pb.agents.r_a.astype(np.float64)
    rc = float(np.float32(prm.r_cost))
    eps = float(np.float32(prm.eps))
    if sc.seg_begin is None:                     # static: one k-d tree for every step
        import scipy.spatial
        two, _ = scipy.spatial.cKDTree(P).query(traj[:, :n_k].reshape(-1, 3), k=2)
        two = two.reshape(traj.shape[0], n_k, 2)
        near = np.maximum(two[..., 0] - R[:, None], eps) < rc
        return np.where(near, two[..., 1] - two[..., 0], np.inf).min(axis=1)
    for k in range(n_k):
        Q = P + (t0 + k * dt) * V
        d = np.linalg.norm(traj[:, k, None, :] - Q[None], axis=2)
        two = np.partition(d, 1, axis=1)[:, :2]
        near = np.maximum(two[:, 0] - R, eps) < rc
        gap = np.where(near, two[:, 1] - two[:, 0], np.inf)
        out = np.minimum(out, gap)
    return out
