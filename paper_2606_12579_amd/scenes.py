"""Seeded synthetic inputs for the rollout, the perception pass and the tests.

This module draws random scenes and agent sets and holds default parameter
values.  It contains none of the planner's arithmetic: no force law, no
integration, no cost, no back-projection.  Both the HIP path and the FP64 oracle
consume what it returns, so it is the only code they share.

Every generator takes a seed and returns FP32 arrays (the precision the HIP path
computes in); the oracle widens them to FP64 exactly.

Workloads (the paper's scenes exist only as figures, so these stand in for them):
  config1  1,000 points uniform in a 0.2 m cube centred at (0.5, 0, 0); 8 agents,
           100 steps; start (0,0,0), goal (1,0,0).
  config2  10 spheres (r 2-10 cm) and 10 boxes (edges 4-20 cm) in the unit cube,
           50,000 surface points (allocated by area) with 5 mm Gaussian noise,
           each object translating at 0.2 m/s; 64 agents, 500 steps.
  config3  640x480 z-depth image of 20 random boxes on a plane, seen from 1 m
           above; the rollout uses 256 agents, 1,000 steps on its voxel centres.
  config4  5 noisy spheres, 20,000 static points; 128 agents with jittered gains,
           400 steps, C1 taper (for gradients).
  config5  512 config2-style scenes with uneven N_O / N_a / N_k and Poisson
           arrival times at 1 kHz.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

F32 = np.float32

# ---------------------------------------------------------------------------
# default parameters (the paper prints no values for these; chosen readings)
MASS = 1.0
K_A = 400.0
D_A = 2.0 * math.sqrt(2.0 * K_A * MASS)  # critical damping of the half-kick dynamics
K_F = 0.01
R_D = 0.10
R_OBS = 0.005        # half of the 1 cm voxel
EPS = 1e-3
A_MAX = 10.0
ALPHA = 0.9
DT = 1e-3
TAPER_BAND = 0.1     # fraction of r_d over which the C1 taper falls to zero


@dataclasses.dataclass
class Params:
    dt: float = DT
    inv_mass: float = 1.0 / MASS
    eps: float = EPS
    r_cost: float = R_D
    w: tuple = (1.0, 1.0, 1.0, 1.0)   # goal, obs, path, smooth
    a_max: float = A_MAX
    alpha: float = ALPHA
    n_steps: int = 100
    cutoff: int = 0                   # 0 = hard (Alg. 1), 1 = C1 taper
    taper_band: float = TAPER_BAND


@dataclasses.dataclass
class Agents:
    k_a: np.ndarray
    d_a: np.ndarray
    k_f: np.ndarray
    r_d: np.ndarray
    r_a: np.ndarray
    omega: np.ndarray  # [N_a, 3]
    heuristic: Optional[np.ndarray] = None   # int32 [N_a]: 0 rotation-vector field, 1 velocity current, 2 APF

    @property
    def n(self) -> int:
        return int(self.k_a.shape[0])

    def subset(self, idx) -> "Agents":
        idx = np.asarray(idx, dtype=np.int64)
        pick = lambda a: None if a is None else np.ascontiguousarray(a[idx])
        return Agents(*(pick(getattr(self, f.name)) for f in dataclasses.fields(self)))


@dataclasses.dataclass
class Scene:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    r_obs: float = R_OBS
    seg_begin: Optional[np.ndarray] = None   # int32 [n_seg + 1] or None (static)
    seg_vel: Optional[np.ndarray] = None     # float32 [n_seg, 3]

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_seg(self) -> int:
        return 0 if self.seg_begin is None else int(self.seg_begin.shape[0] - 1)


@dataclasses.dataclass
class Query:
    p0: np.ndarray
    v0: np.ndarray
    goal: np.ndarray
    incumbent: int = -1
    t0: float = 0.0        # time of step 1 (moving obstacles sit at p_j + t v_seg)


@dataclasses.dataclass
class Problem:
    scene: Scene
    agents: Agents
    query: Query
    params: Params
    name: str = ""


@dataclasses.dataclass
class DepthFrame:
    depth: np.ndarray     # float32 [h, w], z-depth in metres
    K: np.ndarray         # float32 [4] fx, fy, cx, cy
    T_wc: np.ndarray      # float32 [3, 4] camera-to-world rotation | translation
    box_lo: np.ndarray    # float32 [3] workspace box (voxel grid origin)
    dims: np.ndarray      # int32 [3] voxel grid dimensions
    voxel: float = 2 * R_OBS


# ---------------------------------------------------------------------------
def unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    """n directions uniform on the unit sphere (normalised Gaussian samples)."""
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def default_agents(rng: np.random.Generator, n: int, jitter: float = 0.0) -> Agents:
    """Homogeneous circular-field agents; rotation vectors uniform on S^2.

    jitter > 0 multiplies k_a, d_a, k_f by independent U[1 - jitter, 1 + jitter]."""
    omega = unit_vectors(rng, n)
    k_a = np.full(n, K_A)
    d_a = np.full(n, D_A)
    k_f = np.full(n, K_F)
    if jitter > 0:
        k_a = k_a * rng.uniform(1 - jitter, 1 + jitter, n)
        d_a = d_a * rng.uniform(1 - jitter, 1 + jitter, n)
        k_f = k_f * rng.uniform(1 - jitter, 1 + jitter, n)
    return Agents(k_a.astype(F32), d_a.astype(F32), k_f.astype(F32), np.full(n, R_D, F32), np.zeros(n, F32),
                  omega.astype(F32))


def _query(p0, goal, v0=(0.0, 0.0, 0.0)) -> Query:
    return Query(np.asarray(p0, F32), np.asarray(v0, F32), np.asarray(goal, F32), -1)


def _sphere_surface(rng, n, c, r):
    return np.asarray(c) + r * unit_vectors(rng, n)


def _box_surface(rng, n, c, e):
    """n points uniform on the surface of an axis-aligned box with edges e."""
    e = np.asarray(e, float)
    areas = np.array([e[1] * e[2], e[1] * e[2], e[0] * e[2], e[0] * e[2], e[0] * e[1], e[0] * e[1]])
    face = rng.choice(6, size=n, p=areas / areas.sum())
    u = rng.uniform(-0.5, 0.5, (n, 3)) * e
    ax = face // 2
    sign = np.where(face % 2 == 0, -0.5, 0.5)
    u[np.arange(n), ax] = sign * e[ax]
    return np.asarray(c) + u


def _allocate(n_total, weights):
    """Split n_total into integer counts proportional to weights (largest remainder)."""
    w = np.asarray(weights, float)
    raw = n_total * w / w.sum()
    cnt = np.floor(raw).astype(int)
    rem = n_total - cnt.sum()
    order = np.argsort(-(raw - cnt), kind="stable")
    cnt[order[:rem]] += 1
    return cnt


def objects_scene(rng, n_points, n_spheres=10, n_boxes=10, lo=0.15, hi=0.85, sphere_r=(0.02, 0.10),
                  box_e=(0.04, 0.20), noise=0.005, speed=0.2) -> Scene:
    """Surface samples of random spheres and boxes; one constant velocity per object.

    Points are stored grouped by object, so the objects are the segments of the
    scene's segment table."""
    objs = []
    for _ in range(n_spheres):
        c = rng.uniform(lo, hi, 3)
        r = rng.uniform(*sphere_r)
        objs.append(("s", c, r, 4 * math.pi * r * r))
    for _ in range(n_boxes):
        c = rng.uniform(lo, hi, 3)
        e = rng.uniform(box_e[0], box_e[1], 3)
        objs.append(("b", c, e, 2 * (e[0] * e[1] + e[1] * e[2] + e[0] * e[2])))
    counts = _allocate(n_points, [o[3] for o in objs])
    pts, begin, vel = [], [0], []
    for (kind, c, g, _), m in zip(objs, counts):
        p = _sphere_surface(rng, m, c, g) if kind == "s" else _box_surface(rng, m, c, g)
        p = p + rng.normal(0.0, noise, p.shape) if noise > 0 else p
        pts.append(p)
        begin.append(begin[-1] + m)
        vel.append(speed * unit_vectors(rng, 1)[0])
    P = np.concatenate(pts).astype(F32) if pts else np.zeros((0, 3), F32)
    seg_begin = np.asarray(begin, np.int32)
    seg_vel = np.asarray(vel, F32).reshape(-1, 3)
    if speed == 0:
        seg_begin, seg_vel = None, None
    return Scene(np.ascontiguousarray(P[:, 0]), np.ascontiguousarray(P[:, 1]), np.ascontiguousarray(P[:, 2]),
                 R_OBS, seg_begin, seg_vel)


# ---------------------------------------------------------------------------
def config1(seed: int = 0) -> Problem:
    rng = np.random.default_rng(seed)
    P = rng.uniform([0.4, -0.1, -0.1], [0.6, 0.1, 0.1], (1000, 3)).astype(F32)
    scene = Scene(P[:, 0].copy(), P[:, 1].copy(), P[:, 2].copy(), R_OBS)
    agents = default_agents(rng, 8)
    return Problem(scene, agents, _query((0, 0, 0), (1, 0, 0)), Params(n_steps=100), "config1")


def config2(seed: int = 1, n_points: int = 50_000, n_agents: int = 64, n_steps: int = 500) -> Problem:
    rng = np.random.default_rng(seed)
    scene = objects_scene(rng, n_points)
    agents = default_agents(rng, n_agents)
    return Problem(scene, agents, _query((0.02, 0.5, 0.5), (0.98, 0.5, 0.5)), Params(n_steps=n_steps), "config2")


def _ray_box_depth(dirs, origin, c, e, yaw):
    """Distance along each unit-z-normalised ray (camera z-depth) to an upright box
    rotated by yaw about the world z axis; inf where the ray misses."""
    cy, sy = math.cos(yaw), math.sin(yaw)
    R = np.array([[cy, -sy, 0], [sy, cy, 0], [0, 0, 1]])
    o = (origin - c) @ R           # into the box frame (R orthonormal: R^T x = x @ R)
    d = dirs @ R
    half = 0.5 * np.asarray(e)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (-half - o) / d
        t2 = (half - o) / d
    tmin = np.nanmax(np.minimum(t1, t2), axis=1)
    tmax = np.nanmin(np.maximum(t1, t2), axis=1)
    hit = (tmax >= tmin) & (tmax > 0)
    return np.where(hit, np.maximum(tmin, 0.0), np.inf)


def config3_frame(seed: int = 2, w: int = 640, h: int = 480, n_boxes: int = 20) -> DepthFrame:
    """Ray-cast z-depth image of random boxes on the plane z = 0, camera 1 m above
    looking straight down (camera x = world x, camera y = -world y)."""
    rng = np.random.default_rng(seed)
    fx = fy = 525.0
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    R_wc = np.diag([1.0, -1.0, -1.0])
    t_wc = np.array([0.0, 0.0, 1.0])
    u, v = np.meshgrid(np.arange(w, dtype=float), np.arange(h, dtype=float))
    rays_c = np.stack([(u - cx) / fx, (v - cy) / fy, np.ones_like(u)], -1).reshape(-1, 3)  # z-depth 1
    rays_w = rays_c @ R_wc.T
    depth = np.full(rays_w.shape[0], 1.0)          # plane z = 0 sits at depth 1
    half_w, half_h = 0.5 * w / fx, 0.5 * h / fy
    for _ in range(n_boxes):
        e = rng.uniform(0.05, 0.30, 3)
        yaw = rng.uniform(0, math.pi)
        c = np.array([rng.uniform(-half_w + 0.1, half_w - 0.1), rng.uniform(-half_h + 0.1, half_h - 0.1),
                      0.5 * e[2]])
        depth = np.minimum(depth, _ray_box_depth(rays_w, t_wc, c, e, yaw))
    T = np.concatenate([R_wc, t_wc[:, None]], 1)
    voxel = 2 * R_OBS
    box_lo = np.array([-0.645, -0.485, -0.015])
    dims = np.array([130, 98, 40], np.int32)
    return DepthFrame(depth.reshape(h, w).astype(F32), np.array([fx, fy, cx, cy], F32), T.astype(F32),
                      box_lo.astype(F32), dims, voxel)


def config3_agents(seed: int = 2, n_agents: int = 256, n_steps: int = 1000):
    rng = np.random.default_rng(seed + 1000)
    return default_agents(rng, n_agents), _query((-0.5, 0.0, 0.35), (0.5, 0.0, 0.35)), Params(n_steps=n_steps)


def config3_poses(n: int, seed: int = 5, shift: float = 0.05, yaw: float = 0.05) -> np.ndarray:
    """n camera-to-world poses [n, 3, 4] around the config-3 camera (1 m above the
    plane, looking down): yaw about the vertical by U[-yaw, yaw] rad and a horizontal
    shift by U[-shift, shift] m per axis; the first pose is the config-3 pose."""
    rng = np.random.default_rng(seed)
    base = np.diag([1.0, -1.0, -1.0])
    out = np.zeros((n, 3, 4))
    for i in range(n):
        a = 0.0 if i == 0 else rng.uniform(-yaw, yaw)
        t = np.zeros(2) if i == 0 else rng.uniform(-shift, shift, 2)
        Rz = np.array([[math.cos(a), -math.sin(a), 0.0], [math.sin(a), math.cos(a), 0.0], [0.0, 0.0, 1.0]])
        out[i, :, :3] = Rz @ base
        out[i, :, 3] = [t[0], t[1], 1.0]
    return out.astype(F32)


H_CF_OMEGA, H_MFI_VEL, H_APF = 0, 1, 2
K_F_APF = 2e-6       # APF gain: sums over point clouds with 1/rho^3 growth need a much smaller gain


def multi_agents(rng: np.random.Generator, n: int, r_small: float = 0.05, r_large: float = 0.15) -> Agents:
    """A heterogeneous ensemble like the paper's MULTI agents: agent i uses heuristic
    i % 3 (rotation-vector circular field, velocity-current field, APF) and, in turn,
    a small or a large detection radius."""
    ag = default_agents(rng, n)
    heur = (np.arange(n) % 3).astype(np.int32)
    ag.r_d = np.where((np.arange(n) // 3) % 2 == 0, r_small, r_large).astype(F32)
    ag.k_f = np.where(heur == H_APF, K_F_APF, K_F).astype(F32)
    ag.heuristic = heur
    return ag


def config4(seed: int = 3, n_points: int = 20_000, n_agents: int = 128, n_steps: int = 400) -> Problem:
    rng = np.random.default_rng(seed)
    objs = [(rng.uniform(0.3, 0.7, 3), rng.uniform(0.05, 0.15)) for _ in range(5)]
    counts = _allocate(n_points, [r * r for _, r in objs])
    P = np.concatenate([_sphere_surface(rng, m, c, r) for (c, r), m in zip(objs, counts)])
    P = (P + rng.normal(0.0, 0.005, P.shape)).astype(F32)
    scene = Scene(P[:, 0].copy(), P[:, 1].copy(), P[:, 2].copy(), R_OBS)
    agents = default_agents(rng, n_agents, jitter=0.2)
    return Problem(scene, agents, _query((0.05, 0.5, 0.5), (0.95, 0.5, 0.5)),
                   Params(n_steps=n_steps, cutoff=1), "config4")


@dataclasses.dataclass
class Request:
    problem: Problem
    arrival_s: float


def config5_shapes(seed: int = 4, n_scenes: int = 512, rate_hz: float = 1000.0, n_lo: int = 1000,
                   n_hi: int = 200_000, agent_choices=(16, 64, 256), k_lo: int = 100,
                   k_hi: int = 1000) -> List[Tuple[int, int, int, float]]:
    """(N_O, N_a, N_k, arrival time) of each request of the batched-serving workload."""
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    for _ in range(n_scenes):
        n_o = int(rng.integers(n_lo, n_hi + 1))
        n_a = int(rng.choice(agent_choices))
        n_k = int(rng.integers(k_lo, k_hi + 1))
        out.append((n_o, n_a, n_k, t))
        t += float(rng.exponential(1.0 / rate_hz))
    return out


def config5(seed: int = 4, n_scenes: int = 512, rate_hz: float = 1000.0, n_lo: int = 1000, n_hi: int = 200_000,
            agent_choices=(16, 64, 256), k_lo: int = 100, k_hi: int = 1000, only=None) -> List[Request]:
    """Uneven replanning requests with Poisson arrival times (exponential gaps);
    `only` builds just the requests with those indices (each request's scene and
    agents come from their own seed, so a subset equals the same requests of the
    whole workload)."""
    shapes = config5_shapes(seed, n_scenes, rate_hz, n_lo, n_hi, agent_choices, k_lo, k_hi)
    out = []
    for i in (range(n_scenes) if only is None else only):
        n_o, n_a, n_k, t = shapes[i]
        sub = np.random.default_rng([seed, i])
        scene = objects_scene(sub, n_o)
        agents = default_agents(sub, n_a)
        prob = Problem(scene, agents, _query((0.02, 0.5, 0.5), (0.98, 0.5, 0.5)), Params(n_steps=n_k), f"req{i}")
        out.append(Request(prob, t))
    return out


def config5_stratified(n: int = 16, seed: int = 4, n_scenes: int = 512) -> List[int]:
    """Indices of n requests of the batched-serving workload spread over its strata:
    for each agent count, requests evenly spaced in N_O order (the larger share to
    the last agent count when n is not a multiple)."""
    shapes = config5_shapes(seed, n_scenes)
    counts = sorted({a for _, a, _, _ in shapes})
    per = [n // len(counts)] * len(counts)
    per[-1] += n - sum(per)
    pick = []
    for a, m in zip(counts, per):
        idx = sorted((i for i, sh in enumerate(shapes) if sh[1] == a), key=lambda i: shapes[i][0])
        pos = np.linspace(0, len(idx) - 1, m).round().astype(int)
        pick += [idx[p] for p in pos]
    return sorted(pick)


def tiny(seed: int, n_points: int = 8, n_agents: int = 4, n_steps: int = 10, moving: bool = False,
         cutoff: int = 0) -> Problem:
    """Small random problem for brute-force checks: points near the straight
    start-goal line so that the cut-off is exercised."""
    rng = np.random.default_rng(seed)
    P = np.stack([rng.uniform(0.0, 0.05, n_points), rng.uniform(-0.06, 0.06, n_points),
                  rng.uniform(-0.06, 0.06, n_points)], 1).astype(F32)
    seg_begin = seg_vel = None
    if moving and n_points > 0:
        cut = np.sort(rng.integers(0, n_points + 1, 2))
        seg_begin = np.array([0, cut[0], cut[1], n_points], np.int32)
        seg_vel = (0.2 * unit_vectors(rng, 3)).astype(F32)
    scene = Scene(P[:, 0].copy(), P[:, 1].copy(), P[:, 2].copy(), R_OBS, seg_begin, seg_vel)
    agents = default_agents(rng, n_agents)
    q = _query((0.0, 0.0, 0.0), (0.1, 0.0, 0.0), v0=(0.3, 0.0, 0.0))
    return Problem(scene, agents, q, Params(n_steps=n_steps, cutoff=cutoff), f"tiny{seed}")


# ---------------------------------------------------------------- 6-D pose agents
K_R = 10.0           # rotational stiffness [N m / rad]
I_R = 10.0           # inverse rotational inertia [1 / (kg m^2)]


@dataclasses.dataclass
class PoseAgents:
    k_r: np.ndarray            # float32 [N_a] rotational stiffness
    d_r: np.ndarray            # float32 [N_a] rotational damping
    inv_inertia_r: np.ndarray  # float32 [N_a] inverse rotational inertia

    def subset(self, idx) -> "PoseAgents":
        idx = np.asarray(idx, dtype=np.int64)
        return PoseAgents(*(np.ascontiguousarray(getattr(self, f.name)[idx]) for f in dataclasses.fields(self)))


@dataclasses.dataclass
class PoseQuery:
    q0: np.ndarray   # float32 [4] start rotor (w, x, y, z)
    w0: np.ndarray   # float32 [3] start angular velocity, body frame
    qg: np.ndarray   # float32 [4] goal rotor


def unit_rotors(rng: np.random.Generator, n: int) -> np.ndarray:
    """n rotors uniform on S^3 (normalised 4-D Gaussian samples), w >= 0."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1
    return q.astype(F32)


def pose_agents(rng: np.random.Generator, n: int, jitter: float = 0.2) -> PoseAgents:
    """Rotational gains around K_R, I_R (factors U[1 - jitter, 1 + jitter]), each
    agent critically damped: d_r = 2 sqrt(k_r / i_r)."""
    k_r = K_R * rng.uniform(1 - jitter, 1 + jitter, n)
    i_r = I_R * rng.uniform(1 - jitter, 1 + jitter, n)
    return PoseAgents(k_r.astype(F32), (2.0 * np.sqrt(k_r / i_r)).astype(F32), i_r.astype(F32))


def pose_query(rng: np.random.Generator, max_w: float = 1.0) -> PoseQuery:
    """Random start and goal rotors and a start angular velocity of up to max_w rad/s."""
    q = unit_rotors(rng, 2)
    return PoseQuery(q[0], (rng.uniform(-1, 1, 3) * max_w / np.sqrt(3)).astype(F32), q[1])


def robot_spheres(rng: np.random.Generator, n: int = 8, base=(-0.35, -0.05, 0.0), tip=(0.15, 0.1, 0.35),
                  r=(0.04, 0.08)) -> np.ndarray:
    """Bounding spheres of a synthetic arm, float32 [n, 4] (centre, radius): n
    spheres spaced along a bent polyline from base to tip (a stand-in for the FK
    of a robot's sphere set), radii U[r0, r1], shrinking towards the tip."""
    base, tip = np.asarray(base, np.float64), np.asarray(tip, np.float64)
    elbow = 0.5 * (base + tip) + np.array([0.0, 0.15, 0.1])
    s = np.linspace(0.0, 1.0, n)
    pts = np.where(s[:, None] < 0.5, base + (elbow - base) * (2 * s[:, None]),
                   elbow + (tip - elbow) * (2 * s[:, None] - 1))
    rad = rng.uniform(r[0], r[1], n) * np.linspace(1.0, 0.6, n)
    return np.concatenate([pts, rad[:, None]], 1).astype(F32)


# ---------------------------------------------------------------- arm agents
def arm_links(base=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Link transforms [8, 7] (rotor w, x, y, z; offset) of a synthetic 7-joint arm:
    joint axes alternate by +-90 degree turns about x, with 0.33 / 0.316 / 0.384 /
    0.107 m offsets (proportions of a common 7-DoF arm).  Row 0 places the base."""
    h = np.sqrt(0.5)
    rx_m = (h, -h, 0.0, 0.0)          # rotation by -90 degrees about x
    rx_p = (h, h, 0.0, 0.0)           # rotation by +90 degrees about x
    rows = [(1.0, 0.0, 0.0, 0.0, base[0], base[1], base[2] + 0.333),
            (*rx_m, 0.0, 0.0, 0.0),
            (*rx_p, 0.0, -0.316, 0.0),
            (*rx_p, 0.0825, 0.0, 0.0),
            (*rx_m, -0.0825, 0.384, 0.0),
            (*rx_p, 0.0, 0.0, 0.0),
            (*rx_p, 0.088, 0.0, 0.0),
            (1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.107)]
    return np.array(rows, F32)


ARM_Q0 = np.array([0.0, -0.3, 0.0, -2.2, 0.0, 2.0, 0.8], F32)


def arm_problem(seed: int = 13, n_agents: int = 8, n_points: int = 600, n_steps: int = 80, moving: bool = False):
    """Arm agents on a small scene: the synthetic arm at ARM_Q0 (its hand starts near
    (0.47, 0, 0.52)), a goal 0.3 m away, and spheres in an 8 cm box beside the way.
    Returns (Problem, PoseAgents, PoseQuery, links [8, 7], q0 [7])."""
    rng = np.random.default_rng(seed)
    goal = np.array([0.55, 0.25, 0.35], F32)
    P = rng.uniform([0.47, 0.08, 0.42], [0.55, 0.16, 0.50], (n_points, 3)).astype(F32)
    seg_begin = seg_vel = None
    if moving and n_points > 0:
        cut = np.sort(rng.integers(0, n_points + 1, 2))
        seg_begin = np.array([0, cut[0], cut[1], n_points], np.int32)
        seg_vel = (0.2 * unit_vectors(rng, 3)).astype(F32)
    scene = Scene(P[:, 0].copy(), P[:, 1].copy(), P[:, 2].copy(), R_OBS, seg_begin, seg_vel)
    agents = default_agents(rng, n_agents)
    pb = Problem(scene, agents, _query((0.0, 0.0, 0.0), tuple(goal)), Params(n_steps=n_steps), name=f"arm{seed}")
    pa = pose_agents(rng, n_agents)
    pq = PoseQuery(np.array([1, 0, 0, 0], F32), np.zeros(3, F32), unit_rotors(rng, 1)[0])
    return pb, pa, pq, arm_links(), ARM_Q0.copy()
