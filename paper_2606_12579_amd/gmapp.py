"""Python binding of the gmapp C ABI (include/gmapp.h): argument marshalling only.

Every step of the rollout runs in the HIP library libgmapp.so; this module turns
torch tensors (device memory) and the current HIP stream into the C structs and
raises GmappError on a non-zero status.  There is no fallback: if the library
is missing the calls raise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmapp.so")

OK, EINVAL, ENOMEM, EDEVICE, ECAPACITY, ETIMEOUT, ECANCELLED = 0, -1, -2, -3, -4, -5, -6
_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ECAPACITY: "ECAPACITY", ETIMEOUT: "ETIMEOUT",
          ECANCELLED: "ECANCELLED"}


class GmappError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


_fp = ctypes.POINTER(ctypes.c_float)
_ip32 = ctypes.POINTER(ctypes.c_int32)
_ip64 = ctypes.POINTER(ctypes.c_int64)


class Scene(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p), ("n_points", ctypes.c_int64),
                ("n_points_dev", ctypes.c_void_p), ("r_obs", ctypes.c_float), ("n_seg", ctypes.c_int32),
                ("seg_begin", ctypes.c_void_p), ("seg_vel", ctypes.c_void_p)]


class Agents(ctypes.Structure):
    _fields_ = [("k_a", ctypes.c_void_p), ("d_a", ctypes.c_void_p), ("k_f", ctypes.c_void_p), ("r_d", ctypes.c_void_p),
                ("r_a", ctypes.c_void_p), ("omega", ctypes.c_void_p), ("n_agents", ctypes.c_int32),
                ("heuristic", ctypes.c_void_p)]

H_CF_OMEGA, H_MFI_VEL, H_APF = 0, 1, 2


class PoseAgents(ctypes.Structure):
    _fields_ = [("k_r", ctypes.c_void_p), ("d_r", ctypes.c_void_p), ("inv_inertia_r", ctypes.c_void_p)]


class PoseQuery(ctypes.Structure):
    _fields_ = [("q0", ctypes.c_float * 4), ("w0", ctypes.c_float * 3), ("qg", ctypes.c_float * 4)]


class Arm(ctypes.Structure):
    _fields_ = [("n_joints", ctypes.c_int32), ("links", ctypes.c_void_p), ("q0", ctypes.c_void_p),
                ("damping", ctypes.c_float)]


class LoopConfig(ctypes.Structure):
    _fields_ = [("n_cycles", ctypes.c_int32), ("ctrl_steps", ctypes.c_int32), ("ctrl_dt", ctypes.c_float)]


class LoopOutputs(ctypes.Structure):
    _fields_ = [("robot", ctypes.c_void_p), ("robot_clear", ctypes.c_void_p), ("best", ctypes.c_void_p),
                ("cost", ctypes.c_void_p), ("n_switches", ctypes.c_void_p)]


class Query(ctypes.Structure):
    _fields_ = [("p0", ctypes.c_float * 3), ("v0", ctypes.c_float * 3), ("goal", ctypes.c_float * 3),
                ("incumbent", ctypes.c_int32), ("t0", ctypes.c_float)]


class Params(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_float), ("inv_mass", ctypes.c_float), ("eps", ctypes.c_float),
                ("r_cost", ctypes.c_float), ("w_goal", ctypes.c_float), ("w_obs", ctypes.c_float),
                ("w_path", ctypes.c_float), ("w_smooth", ctypes.c_float), ("a_max", ctypes.c_float),
                ("alpha", ctypes.c_float), ("taper_band", ctypes.c_float), ("n_steps", ctypes.c_int32),
                ("cutoff", ctypes.c_int32)]


class Outputs(ctypes.Structure):
    _fields_ = [("traj", ctypes.c_void_p), ("cost", ctypes.c_void_p), ("min_clear", ctypes.c_void_p),
                ("best", ctypes.c_void_p)]


class Tiling(ctypes.Structure):
    _fields_ = [("agents", ctypes.c_int32), ("waves", ctypes.c_int32), ("shards", ctypes.c_int32),
                ("tile_points", ctypes.c_int32), ("layout", ctypes.c_int32), ("group", ctypes.c_int32)]

    def as_tuple(self):
        return (self.agents, self.waves, self.shards, self.tile_points, self.layout, self.group)


class Job(ctypes.Structure):
    _fields_ = [("scene", Scene), ("agents", Agents), ("query", Query), ("params", Params), ("out", Outputs),
                ("state", ctypes.c_void_p), ("k_begin", ctypes.c_int32), ("k_end", ctypes.c_int32),
                ("cancel", ctypes.c_void_p)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("tile_points", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32), ("balance", ctypes.c_int32),
                ("item_shape", ctypes.c_int32)]

    def as_tuple(self):
        return (self.tile_points, self.wg_per_cu, self.balance, self.item_shape)


STATE_FLOATS = 28


class ServerConfig(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_uint64), ("max_active", ctypes.c_int32),
                ("quantum_steps", ctypes.c_int32), ("max_queue", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p), ("n_points", ctypes.c_int64),
                ("r_obs", ctypes.c_float), ("n_seg", ctypes.c_int32), ("seg_begin", ctypes.c_void_p),
                ("seg_vel", ctypes.c_void_p), ("k_a", ctypes.c_void_p), ("d_a", ctypes.c_void_p),
                ("k_f", ctypes.c_void_p), ("r_d", ctypes.c_void_p), ("r_a", ctypes.c_void_p),
                ("omega", ctypes.c_void_p), ("n_agents", ctypes.c_int32), ("query", Query), ("params", Params),
                ("deadline_s", ctypes.c_double), ("cost", ctypes.c_void_p), ("traj", ctypes.c_void_p)]


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("best", ctypes.c_int32),
                ("queue_s", ctypes.c_double), ("latency_s", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("expired", ctypes.c_int64), ("cancelled", ctypes.c_int64), ("cycles", ctypes.c_int64),
                ("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double), ("max_s", ctypes.c_double),
                ("mean_s", ctypes.c_double), ("busy_s", ctypes.c_double), ("interactions_per_s", ctypes.c_double),
                ("cycle_mean_s", ctypes.c_double), ("max_active_seen", ctypes.c_int32),
                ("peak_bytes", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgmapp.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise GmappError(EDEVICE, f"{path} is not built; run __graft_entry__.build() or paper_2606_12579_amd/build.py")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    sigs = {
        "gmapp_create": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_size_t, P(vp)]),
        "gmapp_destroy": (None, [vp]),
        "gmapp_last_error": (ctypes.c_char_p, [vp]),
        "gmapp_version": (ctypes.c_char_p, []),
        "gmapp_rollout": (ctypes.c_int32, [vp, P(Scene), P(Agents), P(Query), P(Params), P(Outputs), vp]),
        "gmapp_force_probe": (ctypes.c_int32, [vp, P(Scene), P(Agents), vp, vp, ctypes.c_float, P(Params), vp, vp,
                                               vp]),
        "gmapp_set_tiling": (ctypes.c_int32, [vp, P(Tiling)]),
        "gmapp_rollout_pose": (ctypes.c_int32, [vp, P(Scene), P(Agents), P(PoseAgents), P(Query), P(PoseQuery),
                                                P(Params), P(Outputs), vp, vp]),
        "gmapp_rollout_arm": (ctypes.c_int32, [vp, P(Scene), P(Agents), P(PoseAgents), P(Arm), P(Query),
                                               P(PoseQuery), P(Params), P(Outputs), vp, vp, vp]),
        "gmapp_plan_loop": (ctypes.c_int32, [vp, P(Scene), P(Agents), P(Query), P(Params), P(LoopConfig),
                                             P(LoopOutputs), vp]),
        "gmapp_control_force": (ctypes.c_int32, [vp, P(Scene), P(Agents), vp, vp, ctypes.c_float, P(Params), vp, vp,
                                                 vp]),
        "gmapp_rollout_backward": (ctypes.c_int32, [vp, P(Scene), P(Agents), P(Query), P(Params), vp, ctypes.c_int32,
                                                    vp, vp, vp, vp, vp]),
        "gmapp_depth_to_points": (ctypes.c_int32, [vp, vp, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_float),
                                                   P(ctypes.c_float), vp, vp, vp, vp]),
        "gmapp_voxel_downsample": (ctypes.c_int32, [vp, vp, vp, vp, ctypes.c_int64, ctypes.c_float, P(ctypes.c_float),
                                                    P(ctypes.c_int32), ctypes.c_int32, vp, vp, vp, ctypes.c_int64, vp,
                                                    vp]),
        "gmapp_voxel_downsample_filtered": (ctypes.c_int32, [vp, vp, vp, vp, ctypes.c_int64, ctypes.c_float,
                                                             P(ctypes.c_float), P(ctypes.c_int32), ctypes.c_int32,
                                                             vp, ctypes.c_int32, vp, vp, vp, ctypes.c_int64, vp,
                                                             vp]),
        "gmapp_depth_to_points_batch": (ctypes.c_int32, [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                         P(ctypes.c_float), vp, vp, vp, vp, vp]),
        "gmapp_voxel_downsample_noalloc": (ctypes.c_int32, [vp, vp, vp, vp, ctypes.c_int64, ctypes.c_float,
                                                            P(ctypes.c_float), P(ctypes.c_int32), ctypes.c_int32,
                                                            vp, vp, vp, ctypes.c_int64, vp, vp]),
        "gmapp_depth_to_voxels": (ctypes.c_int32, [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                   P(ctypes.c_float), vp, ctypes.c_float, P(ctypes.c_float),
                                                   P(ctypes.c_int32), ctypes.c_int32, vp, ctypes.c_int32, vp, vp, vp,
                                                   ctypes.c_int64, vp, vp]),
        "gmapp_set_watchdog": (ctypes.c_int32, [vp, ctypes.c_double]),
        "gmapp_abort": (ctypes.c_int32, [vp, ctypes.c_int32]),
        "gmapp_wait": (ctypes.c_int32, [vp, vp, ctypes.c_double]),
        "gmapp_get_tiling": (ctypes.c_int32, [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32, P(Tiling)]),
        "gmapp_rollout_batch": (ctypes.c_int32, [vp, P(Job), ctypes.c_int32, vp]),
        "gmapp_set_batch_tuning": (ctypes.c_int32, [vp, P(BatchTuning)]),
        "gmapp_get_batch_tuning": (ctypes.c_int32, [vp, P(BatchTuning)]),
        "gmapp_batch_create": (ctypes.c_int32, [vp, ctypes.c_int32, P(vp)]),
        "gmapp_batch_set_jobs": (ctypes.c_int32, [vp, P(Job), ctypes.c_int32]),
        "gmapp_batch_launch": (ctypes.c_int32, [vp, vp]),
        "gmapp_batch_destroy": (None, [vp]),
        "gmapp_autotune_rollout": (ctypes.c_int32, [vp, P(Scene), P(Agents), P(Query), P(Params), ctypes.c_int32,
                                                    P(Tiling), P(ctypes.c_float), vp]),
        "gmapp_autotune_batch": (ctypes.c_int32, [vp, P(Job), ctypes.c_int32, ctypes.c_int32, P(BatchTuning),
                                                  P(ctypes.c_float), vp]),
        "gmapp_server_create": (ctypes.c_int32, [vp, P(ServerConfig), P(vp)]),
        "gmapp_server_submit": (ctypes.c_int32, [vp, P(Request), P(ctypes.c_int64)]),
        "gmapp_server_poll": (ctypes.c_int32, [vp, P(Completion), ctypes.c_int32, ctypes.c_int32]),
        "gmapp_server_cancel": (ctypes.c_int32, [vp, ctypes.c_int64]),
        "gmapp_server_drain": (ctypes.c_int32, [vp, ctypes.c_int32]),
        "gmapp_server_get_stats": (ctypes.c_int32, [vp, P(ServerStats)]),
        "gmapp_server_destroy": (None, [vp]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _check_tensor(t, name, numel=None, dtype=None, device=None):
    import torch
    if t is None:
        return
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if device is not None and t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")


@dataclasses.dataclass
class DeviceScene:
    x: object
    y: object
    z: object
    r_obs: float
    seg_begin: object = None
    seg_vel: object = None
    n_points_dev: object = None   # int64 [1] device count (voxelizer output)

    @property
    def n(self) -> int:
        return int(self.x.numel())


@dataclasses.dataclass
class DeviceAgents:
    k_a: object
    d_a: object
    k_f: object
    r_d: object
    r_a: object
    omega: object
    heuristic: object = None    # int32 [N_a] (H_*), None = all rotation-vector field

    @property
    def n(self) -> int:
        return int(self.k_a.numel())


@dataclasses.dataclass
class DevicePoseAgents:
    k_r: object
    d_r: object
    inv_inertia_r: object


def pose_agents_to_device(pose, device="cuda") -> DevicePoseAgents:
    import torch
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=device)
    return DevicePoseAgents(t(pose.k_r), t(pose.d_r), t(pose.inv_inertia_r))


def scene_to_device(scene, device="cuda") -> DeviceScene:
    import torch
    t = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
    sb = t(scene.seg_begin, torch.int32) if scene.n_seg > 0 else None
    sv = t(scene.seg_vel) if scene.n_seg > 0 else None
    return DeviceScene(t(scene.x), t(scene.y), t(scene.z), float(scene.r_obs), sb, sv)


def agents_to_device(agents, device="cuda") -> DeviceAgents:
    import torch
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=device)
    h = getattr(agents, "heuristic", None)
    h = None if h is None else torch.as_tensor(np.ascontiguousarray(h, dtype=np.int32), device=device)
    return DeviceAgents(t(agents.k_a), t(agents.d_a), t(agents.k_f), t(agents.r_d), t(agents.r_a), t(agents.omega), h)


def make_params(prm) -> Params:
    return Params(float(prm.dt), float(prm.inv_mass), float(prm.eps), float(prm.r_cost), float(prm.w[0]),
                  float(prm.w[1]), float(prm.w[2]), float(prm.w[3]), float(prm.a_max), float(prm.alpha),
                  float(prm.taper_band), int(prm.n_steps), int(prm.cutoff))


def make_query(q) -> Query:
    f3 = lambda a: (ctypes.c_float * 3)(*[float(x) for x in np.asarray(a, np.float32)])
    return Query(f3(q.p0), f3(q.v0), f3(q.goal), int(q.incumbent), float(getattr(q, 't0', 0.0)))


def _scene_struct(sc: DeviceScene, device) -> Scene:
    import torch
    n = sc.n
    for nm in ("x", "y", "z"):
        _check_tensor(getattr(sc, nm), f"scene.{nm}", n, torch.float32, device)
    n_seg = 0
    if sc.seg_begin is not None:
        n_seg = int(sc.seg_begin.numel()) - 1
        _check_tensor(sc.seg_begin, "scene.seg_begin", n_seg + 1, torch.int32, device)
        _check_tensor(sc.seg_vel, "scene.seg_vel", 3 * n_seg, torch.float32, device)
    if sc.n_points_dev is not None:
        _check_tensor(sc.n_points_dev, "scene.n_points_dev", 1, torch.int64, device)
    return Scene(_ptr(sc.x), _ptr(sc.y), _ptr(sc.z), n, _ptr(sc.n_points_dev), float(sc.r_obs), n_seg,
                 _ptr(sc.seg_begin), _ptr(sc.seg_vel))


def _agents_struct(ag: DeviceAgents, device) -> Agents:
    import torch
    n = ag.n
    for nm in ("k_a", "d_a", "k_f", "r_d", "r_a"):
        _check_tensor(getattr(ag, nm), f"agents.{nm}", n, torch.float32, device)
    _check_tensor(ag.omega, "agents.omega", 3 * n, torch.float32, device)
    h = getattr(ag, "heuristic", None)
    if h is not None:
        _check_tensor(h, "agents.heuristic", n, torch.int32, device)
    return Agents(_ptr(ag.k_a), _ptr(ag.d_a), _ptr(ag.k_f), _ptr(ag.r_d), _ptr(ag.r_a), _ptr(ag.omega), n,
                  None if h is None else _ptr(h))


@dataclasses.dataclass
class BatchJob:
    """One job of a batched launch: device scene and agents, host query and
    params, device outputs (dict as returned by Context.outputs), optional state
    tensor [N_a, STATE_FLOATS] and the step range [k_begin, k_end)."""
    scene: DeviceScene
    agents: DeviceAgents
    query: object
    params: object
    out: dict
    state: object = None
    k_begin: int = 1
    k_end: int = 0          # 0 = N_k + 1


def _outputs_check(out, na, nk, dev):
    import torch
    _check_tensor(out.get("traj"), "traj", na * (nk + 1) * 3, torch.float32, dev)
    _check_tensor(out["cost"], "cost", na * 5, torch.float32, dev)
    _check_tensor(out.get("min_clear"), "min_clear", na * nk, torch.float32, dev)
    _check_tensor(out["best"], "best", 1, torch.int32, dev)


def _job_struct(j: BatchJob, dev) -> Job:
    import torch
    na, nk = j.agents.n, int(j.params.n_steps)
    _outputs_check(j.out, na, nk, dev)
    _check_tensor(j.state, "state", na * STATE_FLOATS, torch.float32, dev)
    o = Outputs(_ptr(j.out.get("traj")), _ptr(j.out["cost"]), _ptr(j.out.get("min_clear")), _ptr(j.out["best"]))
    k_end = int(j.k_end) if j.k_end else nk + 1
    return Job(_scene_struct(j.scene, dev), _agents_struct(j.agents, dev), make_query(j.query),
               make_params(j.params), o, _ptr(j.state), int(j.k_begin), k_end)


def _jobs_array(jobs, dev):
    arr = (Job * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = _job_struct(j, dev)
    return arr


class Batch:
    """An instantiated control-cycle graph (gmapp_batch_*): set_jobs, then launch."""

    def __init__(self, ctx: "Context", max_jobs: int):
        self.ctx = ctx
        h = ctypes.c_void_p()
        ctx._raise(ctx.lib.gmapp_batch_create(ctx.handle, int(max_jobs), ctypes.byref(h)))
        self.handle = h
        self._keep = None

    def set_jobs(self, jobs):
        arr = _jobs_array(jobs, self.ctx.device)
        self.ctx._raise(self.ctx.lib.gmapp_batch_set_jobs(self.handle, arr, len(jobs)))
        self._keep = jobs

    def launch(self, stream=None):
        self.ctx._raise(self.ctx.lib.gmapp_batch_launch(self.handle, self.ctx._stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            self.ctx.lib.gmapp_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """gmapp_server_*: the replanning request loop.  submit() takes a scenes.Problem
    (host arrays), keeps its arrays alive until its completion is polled, and
    returns the request id; poll() returns completions with the host results."""

    def __init__(self, ctx: "Context", memory_budget=0, max_active=0, quantum_steps=0, max_queue=0):
        self.ctx = ctx
        cfg = ServerConfig(int(memory_budget), int(max_active), int(quantum_steps), int(max_queue))
        h = ctypes.c_void_p()
        ctx._raise(ctx.lib.gmapp_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self.live = {}

    def submit(self, problem, deadline_s=0.0, traj=False):
        sc, ag, prm = problem.scene, problem.agents, problem.params
        f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
        keep = {"x": f32(sc.x), "y": f32(sc.y), "z": f32(sc.z)}
        n_seg = int(sc.n_seg)
        if n_seg > 0:
            keep["seg_begin"] = np.ascontiguousarray(sc.seg_begin, dtype=np.int32)
            keep["seg_vel"] = f32(sc.seg_vel)
        for nm in ("k_a", "d_a", "k_f", "r_d", "r_a", "omega"):
            keep[nm] = f32(getattr(ag, nm))
        na, nk = int(ag.n), int(prm.n_steps)
        keep["cost"] = np.full((na, 5), np.nan, np.float32)
        keep["traj"] = np.zeros((na, nk + 1, 3), np.float32) if traj else None
        p = lambda k: None if keep.get(k) is None else keep[k].ctypes.data
        r = Request(p("x"), p("y"), p("z"), int(sc.n), float(sc.r_obs), n_seg, p("seg_begin"), p("seg_vel"),
                    p("k_a"), p("d_a"), p("k_f"), p("r_d"), p("r_a"), p("omega"), na, make_query(problem.query),
                    make_params(prm), float(deadline_s), p("cost"), p("traj"))
        rid = ctypes.c_int64()
        self.ctx._raise(self.ctx.lib.gmapp_server_submit(self.handle, ctypes.byref(r), ctypes.byref(rid)))
        self.live[rid.value] = keep
        return rid.value

    def poll(self, max_n=256, wait_ms=0):
        buf = (Completion * max_n)()
        n = self.ctx.lib.gmapp_server_poll(self.handle, buf, int(max_n), int(wait_ms))
        out = []
        for c in buf[:n]:
            keep = self.live.pop(c.id, {})
            out.append({"id": c.id, "status": c.status, "best": c.best, "queue_s": c.queue_s,
                        "latency_s": c.latency_s, "cost": keep.get("cost"), "traj": keep.get("traj")})
        return out

    def cancel(self, rid):
        self.ctx._raise(self.ctx.lib.gmapp_server_cancel(self.handle, int(rid)))

    def drain(self, timeout_ms=-1):
        return self.ctx.lib.gmapp_server_drain(self.handle, int(timeout_ms))

    def stats(self):
        st = ServerStats()
        rc = self.ctx.lib.gmapp_server_get_stats(self.handle, ctypes.byref(st))
        d = st.as_dict()
        d["fault"] = rc
        return d

    def close(self):
        if getattr(self, "handle", None):
            self.ctx.lib.gmapp_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """One library context (device arena + tiling policy) on one HIP device."""

    def __init__(self, device: int = 0, workspace_bytes: int = 0):
        import torch
        self.lib = load_library()
        self.device_index = int(device)
        self.device = torch.device("cuda", self.device_index)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = self.lib.gmapp_create(self.device_index, int(workspace_bytes), ctypes.byref(h))
        if st != OK:
            raise GmappError(st, "gmapp_create failed")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.gmapp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st):
        if st != OK:
            raise GmappError(st, self.lib.gmapp_last_error(self.handle).decode())

    def _stream(self, stream):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(s.cuda_stream)

    # ------------------------------------------------------------------ failure handling
    def set_watchdog(self, seconds=0.0):
        """gmapp_set_watchdog: longest stall of one exchange wait (0 = the default 4 s)."""
        self._raise(self.lib.gmapp_set_watchdog(self.handle, float(seconds)))

    def abort(self, raise_=True):
        """gmapp_abort: raise (or lower) the context's abort word."""
        self._raise(self.lib.gmapp_abort(self.handle, 1 if raise_ else 0))

    def wait(self, timeout_s, stream=None):
        """gmapp_wait: wait for the stream up to timeout_s, else abort its launches (GmappError ETIMEOUT)."""
        self._raise(self.lib.gmapp_wait(self.handle, self._stream(stream), float(timeout_s)))

    # ------------------------------------------------------------------ tiling
    def set_tiling(self, agents=0, waves=0, shards=0, tile_points=0, layout=0, group=0):
        """Force a tiling (zeros = choose): agents per group, waves per workgroup, shards,
        streamed tile points, layout (0 auto, 1 resident, 2 streamed), group (1 wave, 2 workgroup)."""
        t = Tiling(agents, waves, shards, tile_points, layout, group)
        self._raise(self.lib.gmapp_set_tiling(self.handle, ctypes.byref(t)))

    def clear_tiling(self):
        self._raise(self.lib.gmapp_set_tiling(self.handle, None))

    def get_tiling(self, n_points, n_agents, n_steps, n_seg=0, cutoff=0):
        t = Tiling()
        self._raise(self.lib.gmapp_get_tiling(self.handle, int(n_points), int(n_agents), int(n_steps), int(n_seg),
                                              int(cutoff), ctypes.byref(t)))
        return t.as_tuple()

    # ------------------------------------------------------------------ batched launches
    def outputs(self, n_agents, n_steps, traj=True, min_clear=True):
        """Freshly allocated output tensors for one problem."""
        import torch
        dev = self.device
        return {
            "traj": torch.empty((n_agents, n_steps + 1, 3), dtype=torch.float32, device=dev) if traj else None,
            "cost": torch.empty((n_agents, 5), dtype=torch.float32, device=dev),
            "min_clear": torch.empty((n_agents, n_steps), dtype=torch.float32, device=dev) if min_clear else None,
            "best": torch.empty(1, dtype=torch.int32, device=dev),
        }

    def rollout_batch(self, jobs, stream=None):
        """gmapp_rollout_batch over a list of BatchJob."""
        arr = _jobs_array(jobs, self.device)
        self._raise(self.lib.gmapp_rollout_batch(self.handle, arr, len(jobs), self._stream(stream)))

    def batch(self, max_jobs):
        return Batch(self, max_jobs)

    def server(self, memory_budget=0, max_active=0, quantum_steps=0, max_queue=0):
        return Server(self, memory_budget, max_active, quantum_steps, max_queue)

    def set_batch_tuning(self, tile_points=0, wg_per_cu=0, balance=0, item_shape=0):
        t = BatchTuning(tile_points, wg_per_cu, balance, item_shape)
        self._raise(self.lib.gmapp_set_batch_tuning(self.handle, ctypes.byref(t)))

    def clear_batch_tuning(self):
        self._raise(self.lib.gmapp_set_batch_tuning(self.handle, None))

    def get_batch_tuning(self):
        t = BatchTuning()
        self._raise(self.lib.gmapp_get_batch_tuning(self.handle, ctypes.byref(t)))
        return t.as_tuple()

    def autotune_rollout(self, scene: DeviceScene, agents: DeviceAgents, query, params, proxy_steps=32, stream=None):
        """gmapp_autotune_rollout: returns (tiling tuple, proxy ms) and caches the choice."""
        t, ms = Tiling(), ctypes.c_float()
        sc, ag = _scene_struct(scene, self.device), _agents_struct(agents, self.device)
        q, p = make_query(query), make_params(params)
        self._raise(self.lib.gmapp_autotune_rollout(self.handle, ctypes.byref(sc), ctypes.byref(ag), ctypes.byref(q),
                                                    ctypes.byref(p), int(proxy_steps), ctypes.byref(t),
                                                    ctypes.byref(ms), self._stream(stream)))
        return t.as_tuple(), float(ms.value)

    def autotune_batch(self, jobs, proxy_steps=16, stream=None):
        """gmapp_autotune_batch: returns (tuning tuple, proxy ms) and keeps the choice."""
        arr = _jobs_array(jobs, self.device)
        t, ms = BatchTuning(), ctypes.c_float()
        self._raise(self.lib.gmapp_autotune_batch(self.handle, arr, len(jobs), int(proxy_steps), ctypes.byref(t),
                                                  ctypes.byref(ms), self._stream(stream)))
        return t.as_tuple(), float(ms.value)

    # ------------------------------------------------------------------ rollout
    def rollout(self, scene: DeviceScene, agents: DeviceAgents, query, params, traj=True, min_clear=True,
                out=None, stream=None):
        """gmapp_rollout.  Returns dict(traj, cost, min_clear, best) of device tensors."""
        import torch
        na, nk = agents.n, int(params.n_steps)
        dev = self.device
        if out is None:
            out = {
                "traj": torch.empty((na, nk + 1, 3), dtype=torch.float32, device=dev) if traj else None,
                "cost": torch.empty((na, 5), dtype=torch.float32, device=dev),
                "min_clear": torch.empty((na, nk), dtype=torch.float32, device=dev) if min_clear else None,
                "best": torch.empty(1, dtype=torch.int32, device=dev),
            }
        _check_tensor(out.get("traj"), "traj", na * (nk + 1) * 3, torch.float32, dev)
        _check_tensor(out["cost"], "cost", na * 5, torch.float32, dev)
        _check_tensor(out.get("min_clear"), "min_clear", na * nk, torch.float32, dev)
        _check_tensor(out["best"], "best", 1, torch.int32, dev)
        sc, ag = _scene_struct(scene, dev), _agents_struct(agents, dev)
        q, p = make_query(query), make_params(params)
        o = Outputs(_ptr(out.get("traj")), _ptr(out["cost"]), _ptr(out.get("min_clear")), _ptr(out["best"]))
        st = self.lib.gmapp_rollout(self.handle, ctypes.byref(sc), ctypes.byref(ag), ctypes.byref(q),
                                    ctypes.byref(p), ctypes.byref(o), self._stream(stream))
        self._raise(st)
        return out

    def force_probe(self, scene: DeviceScene, agents: DeviceAgents, p, v, t, params, stream=None):
        """gmapp_force_probe: Alg. 1's response at given states. Returns (f_r [N_a,3], rho_min [N_a])."""
        import torch
        na, dev = agents.n, self.device
        _check_tensor(p, "p", 3 * na, torch.float32, dev)
        _check_tensor(v, "v", 3 * na, torch.float32, dev)
        f = torch.empty((na, 3), dtype=torch.float32, device=dev)
        r = torch.empty(na, dtype=torch.float32, device=dev)
        sc, ag = _scene_struct(scene, dev), _agents_struct(agents, dev)
        prm = make_params(params)
        st = self.lib.gmapp_force_probe(self.handle, ctypes.byref(sc), ctypes.byref(ag), _ptr(p), _ptr(v),
                                        float(t), ctypes.byref(prm), _ptr(f), _ptr(r), self._stream(stream))
        self._raise(st)
        return f, r

    def rollout_pose(self, scene: DeviceScene, agents: DeviceAgents, pose_agents, query, pose_query, params,
                     traj=True, min_clear=True, rot=True, out=None, stream=None):
        """gmapp_rollout_pose: 6-D pose agents. pose_agents: (k_r, d_r, inv_inertia_r) device float32 [N_a]
        tensors (DevicePoseAgents); pose_query: q0 [4], w0 [3], qg [4]. Returns the outputs of rollout plus
        rot [N_a, N_k + 1, 4]."""
        import torch
        na, nk, dev = agents.n, int(params.n_steps), self.device
        if out is None:
            out = {"traj": torch.empty((na, nk + 1, 3), dtype=torch.float32, device=dev) if traj else None,
                   "cost": torch.empty((na, 5), dtype=torch.float32, device=dev),
                   "min_clear": torch.empty((na, nk), dtype=torch.float32, device=dev) if min_clear else None,
                   "best": torch.empty(1, dtype=torch.int32, device=dev),
                   "rot": torch.empty((na, nk + 1, 4), dtype=torch.float32, device=dev) if rot else None}
        for nm in ("k_r", "d_r", "inv_inertia_r"):
            _check_tensor(getattr(pose_agents, nm), f"pose_agents.{nm}", na, torch.float32, dev)
        sc, ag = _scene_struct(scene, dev), _agents_struct(agents, dev)
        pa = PoseAgents(_ptr(pose_agents.k_r), _ptr(pose_agents.d_r), _ptr(pose_agents.inv_inertia_r))
        f = lambda a, n: (ctypes.c_float * n)(*[float(x) for x in np.asarray(a, np.float32).reshape(-1)])
        pq = PoseQuery(f(pose_query.q0, 4), f(pose_query.w0, 3), f(pose_query.qg, 4))
        q, p = make_query(query), make_params(params)
        o = Outputs(_ptr(out["traj"]), _ptr(out["cost"]), _ptr(out["min_clear"]), _ptr(out["best"]))
        st = self.lib.gmapp_rollout_pose(self.handle, ctypes.byref(sc), ctypes.byref(ag), ctypes.byref(pa),
                                         ctypes.byref(q), ctypes.byref(pq), ctypes.byref(p), ctypes.byref(o),
                                         _ptr(out.get("rot")), self._stream(stream))
        self._raise(st)
        return out

    def rollout_arm(self, scene: DeviceScene, agents: DeviceAgents, pose_agents, links, q0, damping, query,
                    pose_query, params, stream=None):
        """gmapp_rollout_arm: arm agents driving the serial chain `links` (device float32 [n + 1, 7]) from the
        joint angles q0 (device float32 [n]). Returns the outputs of rollout_pose plus joints [N_a, N_k + 1, n]."""
        import torch
        na, nk, dev = agents.n, int(params.n_steps), self.device
        nj = int(q0.numel())
        _check_tensor(links, "links", 7 * (nj + 1), torch.float32, dev)
        _check_tensor(q0, "q0", nj, torch.float32, dev)
        for nm in ("k_r", "d_r", "inv_inertia_r"):
            _check_tensor(getattr(pose_agents, nm), f"pose_agents.{nm}", na, torch.float32, dev)
        out = {"traj": torch.empty((na, nk + 1, 3), dtype=torch.float32, device=dev),
               "cost": torch.empty((na, 5), dtype=torch.float32, device=dev),
               "min_clear": torch.empty((na, nk), dtype=torch.float32, device=dev),
               "best": torch.empty(1, dtype=torch.int32, device=dev),
               "rot": torch.empty((na, nk + 1, 4), dtype=torch.float32, device=dev),
               "joints": torch.empty((na, nk + 1, max(nj, 1)), dtype=torch.float32, device=dev)}
        sc, ag = _scene_struct(scene, dev), _agents_struct(agents, dev)
        pa = PoseAgents(_ptr(pose_agents.k_r), _ptr(pose_agents.d_r), _ptr(pose_agents.inv_inertia_r))
        arm = Arm(nj, _ptr(links), _ptr(q0), float(damping))
        f = lambda a, n: (ctypes.c_float * n)(*[float(x) for x in np.asarray(a, np.float32).reshape(-1)])
        pq = PoseQuery(f(pose_query.q0, 4), f(pose_query.w0, 3), f(pose_query.qg, 4))
        q, p = make_query(query), make_params(params)
        o = Outputs(_ptr(out["traj"]), _ptr(out["cost"]), _ptr(out["min_clear"]), _ptr(out["best"]))
        st = self.lib.gmapp_rollout_arm(self.handle, ctypes.byref(sc), ctypes.byref(ag), ctypes.byref(pa),
                                        ctypes.byref(arm), ctypes.byref(q), ctypes.byref(pq), ctypes.byref(p),
                                        ctypes.byref(o), _ptr(out["rot"]), _ptr(out["joints"]), self._stream(stream))
        self._raise(st)
        return out

    def plan_loop(self, scene: DeviceScene, agents: DeviceAgents, query, params, n_cycles, ctrl_steps, ctrl_dt,
                  clear=True, stream=None):
        """gmapp_plan_loop: the closed planning loop. Returns robot [n_cycles*ctrl_steps + 1, 6] (p, v),
        robot_clear [n_cycles*ctrl_steps] (or None), best [n_cycles], cost [n_cycles, N_a, 5], n_switches [1]."""
        import torch
        na, dev = agents.n, self.device
        T = int(n_cycles) * int(ctrl_steps)
        out = {"robot": torch.empty((T + 1, 6), dtype=torch.float32, device=dev),
               "robot_clear": torch.empty(T, dtype=torch.float32, device=dev) if clear else None,
               "best": torch.empty(max(int(n_cycles), 0), dtype=torch.int32, device=dev),
               "cost": torch.empty((max(int(n_cycles), 0), na, 5), dtype=torch.float32, device=dev),
               "n_switches": torch.empty(1, dtype=torch.int32, device=dev)}
        sc, ag = _scene_struct(scene, dev), _agents_struct(agents, dev)
        q, p = make_query(query), make_params(params)
        cfg = LoopConfig(int(n_cycles), int(ctrl_steps), float(ctrl_dt))
        lo = LoopOutputs(_ptr(out["robot"]), _ptr(out["robot_clear"]), _ptr(out["best"]), _ptr(out["cost"]),
                         _ptr(out["n_switches"]))
        st = self.lib.gmapp_plan_loop(self.handle, ctypes.byref(sc), ctypes.byref(ag), ctypes.byref(q),
                                      ctypes.byref(p), ctypes.byref(cfg), ctypes.byref(lo), self._stream(stream))
        self._raise(st)
        return out

    def control_force(self, scene: DeviceScene, agents: DeviceAgents, agent, state, t, params, stream=None):
        """gmapp_control_force: f_r [3] and rho_min [1] of the agent whose index is the device int32 `agent` [1]
        at the device state [6] (p, v) and time t."""
        import torch
        dev = self.device
        _check_tensor(agent, "agent", 1, torch.int32, dev)
        _check_tensor(state, "state", 6, torch.float32, dev)
        f = torch.empty(3, dtype=torch.float32, device=dev)
        r = torch.empty(1, dtype=torch.float32, device=dev)
        sc, ag = _scene_struct(scene, dev), _agents_struct(agents, dev)
        prm = make_params(params)
        st = self.lib.gmapp_control_force(self.handle, ctypes.byref(sc), ctypes.byref(ag), _ptr(agent), _ptr(state),
                                          float(t), ctypes.byref(prm), _ptr(f), _ptr(r), self._stream(stream))
        self._raise(st)
        return f, r

    def rollout_backward(self, scene: DeviceScene, agents: DeviceAgents, query, params, grad_total, ckpt_every=50,
                         stream=None):
        """gmapp_rollout_backward: d(sum_i grad_total[i] C_i) / d(k_a, d_a, k_f, omega) per agent."""
        import torch
        na, dev = agents.n, self.device
        _check_tensor(grad_total, "grad_total", na, torch.float32, dev)
        g = {k: torch.empty(na, dtype=torch.float32, device=dev) for k in ("k_a", "d_a", "k_f")}
        g["omega"] = torch.empty((na, 3), dtype=torch.float32, device=dev)
        sc, ag = _scene_struct(scene, dev), _agents_struct(agents, dev)
        q, p = make_query(query), make_params(params)
        st = self.lib.gmapp_rollout_backward(self.handle, ctypes.byref(sc), ctypes.byref(ag), ctypes.byref(q),
                                             ctypes.byref(p), _ptr(grad_total), int(ckpt_every), _ptr(g["k_a"]),
                                             _ptr(g["d_a"]), _ptr(g["k_f"]), _ptr(g["omega"]), self._stream(stream))
        self._raise(st)
        return g

    # ------------------------------------------------------------------ perception
    def depth_to_points(self, depth, K, T_wc, out=None, stream=None):
        """gmapp_depth_to_points: depth [h, w] (device float32) -> x, y, z [h*w] (NaN for invalid pixels)."""
        import torch
        if depth.dim() != 2:
            raise ValueError("depth must be [h, w]")
        h, w = depth.shape
        _check_tensor(depth, "depth", h * w, torch.float32, self.device)
        if out is None:
            out = tuple(torch.empty(h * w, dtype=torch.float32, device=self.device) for _ in range(3))
        for i, t in enumerate(out):
            _check_tensor(t, f"out[{i}]", h * w, torch.float32, self.device)
        Kc = (ctypes.c_float * 4)(*[float(v) for v in np.asarray(K, np.float32).reshape(4)])
        Tc = (ctypes.c_float * 12)(*[float(v) for v in np.asarray(T_wc, np.float32).reshape(12)])
        st = self.lib.gmapp_depth_to_points(self.handle, _ptr(depth), int(w), int(h), Kc, Tc, _ptr(out[0]),
                                            _ptr(out[1]), _ptr(out[2]), self._stream(stream))
        self._raise(st)
        return out

    def depth_to_points_batch(self, depth, K, T_wc, out=None, stream=None):
        """gmapp_depth_to_points_batch: depth [B, h, w] and poses T_wc [B, 3, 4] (device float32)
        -> x, y, z [B*h*w]."""
        import torch
        if depth.dim() != 3:
            raise ValueError("depth must be [frames, h, w]")
        b, h, w = depth.shape
        n = b * h * w
        _check_tensor(depth, "depth", n, torch.float32, self.device)
        _check_tensor(T_wc, "T_wc", 12 * b, torch.float32, self.device)
        if out is None:
            out = tuple(torch.empty(n, dtype=torch.float32, device=self.device) for _ in range(3))
        for i, t in enumerate(out):
            _check_tensor(t, f"out[{i}]", n, torch.float32, self.device)
        Kc = (ctypes.c_float * 4)(*[float(v) for v in np.asarray(K, np.float32).reshape(4)])
        st = self.lib.gmapp_depth_to_points_batch(self.handle, _ptr(depth), int(b), int(w), int(h), Kc, _ptr(T_wc),
                                                  _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), self._stream(stream))
        self._raise(st)
        return out

    def voxel_downsample_noalloc(self, x, y, z, voxel, lo, dims, min_count=1, out=None, stream=None):
        """gmapp_voxel_downsample_noalloc: the voxel pass on the library's static per-device grid (the call
        allocates nothing; `out` = (ox, oy, oz, n_out) must be given, the capacity is ox's length)."""
        import torch
        n = int(x.numel())
        for nm, t in (("x", x), ("y", y), ("z", z)):
            _check_tensor(t, nm, n, torch.float32, self.device)
        if out is None or len(out) != 4:
            raise ValueError("out = (ox, oy, oz, n_out) is required: this call allocates nothing")
        capacity = int(out[0].numel())
        for i in range(3):
            _check_tensor(out[i], f"out[{i}]", capacity, torch.float32, self.device)
        _check_tensor(out[3], "n_out", 1, torch.int64, self.device)
        loc = (ctypes.c_float * 3)(*[float(v) for v in np.asarray(lo, np.float32).reshape(3)])
        dc = (ctypes.c_int32 * 3)(*[int(v) for v in np.asarray(dims).reshape(3)])
        st = self.lib.gmapp_voxel_downsample_noalloc(self.handle, _ptr(x), _ptr(y), _ptr(z), n, float(voxel), loc,
                                                     dc, int(min_count), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]),
                                                     capacity, _ptr(out[3]), self._stream(stream))
        self._raise(st)
        return out

    def voxel_downsample(self, x, y, z, voxel, lo, dims, min_count=1, capacity=None, out=None, stream=None,
                         robot_spheres=None):
        """gmapp_voxel_downsample (gmapp_voxel_downsample_filtered with robot_spheres, a device float32 [K, 4]
        tensor of the robot's bounding spheres): occupied voxel centres (sorted by cell) and the device count.

        Returns (ox, oy, oz, n_out) with n_out an int64 [1] device tensor."""
        import torch
        n = int(x.numel())
        for nm, t in (("x", x), ("y", y), ("z", z)):
            _check_tensor(t, nm, n, torch.float32, self.device)
        if capacity is None:
            capacity = n
        if out is None:
            out = tuple(torch.empty(max(capacity, 1), dtype=torch.float32, device=self.device) for _ in range(3)) + \
                (torch.zeros(1, dtype=torch.int64, device=self.device),)
        loc = (ctypes.c_float * 3)(*[float(v) for v in np.asarray(lo, np.float32).reshape(3)])
        dc = (ctypes.c_int32 * 3)(*[int(v) for v in np.asarray(dims).reshape(3)])
        if robot_spheres is not None:
            ns = int(robot_spheres.numel()) // 4
            _check_tensor(robot_spheres, "robot_spheres", 4 * ns, torch.float32, self.device)
            st = self.lib.gmapp_voxel_downsample_filtered(self.handle, _ptr(x), _ptr(y), _ptr(z), n, float(voxel),
                                                          loc, dc, int(min_count), _ptr(robot_spheres), ns,
                                                          _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), int(capacity),
                                                          _ptr(out[3]), self._stream(stream))
        else:
            st = self.lib.gmapp_voxel_downsample(self.handle, _ptr(x), _ptr(y), _ptr(z), n, float(voxel), loc, dc,
                                                 int(min_count), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]),
                                                 int(capacity), _ptr(out[3]), self._stream(stream))
        self._raise(st)
        return out

    def depth_to_voxels(self, depth, K, T_wc, voxel, lo, dims, min_count=1, capacity=None, out=None, stream=None,
                        robot_spheres=None):
        """gmapp_depth_to_voxels: depth [B, h, w] and poses T_wc [B, 3, 4] (device float32) straight to the
        occupied voxel centres (sorted by cell) and the device count.  robot_spheres: optional device float32
        [K, 4] bounding spheres of the self-filter.

        Returns (ox, oy, oz, n_out) with n_out an int64 [1] device tensor."""
        import torch
        if depth.dim() != 3:
            raise ValueError("depth must be [frames, h, w]")
        b, h, w = depth.shape
        n = b * h * w
        _check_tensor(depth, "depth", n, torch.float32, self.device)
        _check_tensor(T_wc, "T_wc", 12 * b, torch.float32, self.device)
        if capacity is None:
            capacity = n
        if out is None:
            out = tuple(torch.empty(max(capacity, 1), dtype=torch.float32, device=self.device) for _ in range(3)) + \
                (torch.zeros(1, dtype=torch.int64, device=self.device),)
        Kc = (ctypes.c_float * 4)(*[float(v) for v in np.asarray(K, np.float32).reshape(4)])
        loc = (ctypes.c_float * 3)(*[float(v) for v in np.asarray(lo, np.float32).reshape(3)])
        dc = (ctypes.c_int32 * 3)(*[int(v) for v in np.asarray(dims).reshape(3)])
        ns, rs = 0, None
        if robot_spheres is not None:
            ns = int(robot_spheres.numel()) // 4
            _check_tensor(robot_spheres, "robot_spheres", 4 * ns, torch.float32, self.device)
            rs = _ptr(robot_spheres)
        st = self.lib.gmapp_depth_to_voxels(self.handle, _ptr(depth), int(b), int(w), int(h), Kc, _ptr(T_wc),
                                            float(voxel), loc, dc, int(min_count), rs, ns, _ptr(out[0]),
                                            _ptr(out[1]), _ptr(out[2]), int(capacity), _ptr(out[3]),
                                            self._stream(stream))
        self._raise(st)
        return out


class _RolloutCost:
    """torch.autograd.Function: total costs C_i of the rollout as a differentiable
    function of the per-agent k_a, d_a, k_f and omega (forward: gmapp_rollout;
    backward: gmapp_rollout_backward with state checkpoints every `ckpt_every` steps)."""

    _fn = None

    @classmethod
    def get(cls):
        if cls._fn is None:
            import torch

            class Fn(torch.autograd.Function):
                @staticmethod
                def forward(fctx, gctx, scene, r_d, r_a, query, params, ckpt_every, k_a, d_a, k_f, omega):
                    agents = DeviceAgents(k_a.detach().contiguous(), d_a.detach().contiguous(),
                                          k_f.detach().contiguous(), r_d, r_a, omega.detach().contiguous())
                    out = gctx.rollout(scene, agents, query, params, traj=False, min_clear=False)
                    fctx.save_for_backward(k_a, d_a, k_f, omega)
                    fctx.meta = (gctx, scene, r_d, r_a, query, params, ckpt_every)
                    fctx.mark_non_differentiable(out["best"])
                    return out["cost"][:, 4].clone(), out["best"]

                @staticmethod
                def backward(fctx, g_total, g_best):
                    k_a, d_a, k_f, omega = fctx.saved_tensors
                    gctx, scene, r_d, r_a, query, params, ckpt_every = fctx.meta
                    agents = DeviceAgents(k_a.detach().contiguous(), d_a.detach().contiguous(),
                                          k_f.detach().contiguous(), r_d, r_a, omega.detach().contiguous())
                    g = gctx.rollout_backward(scene, agents, query, params, g_total.contiguous().float(), ckpt_every)
                    return (None, None, None, None, None, None, None, g["k_a"], g["d_a"], g["k_f"], g["omega"])

            cls._fn = Fn
        return cls._fn


def rollout_cost(gctx: Context, scene: DeviceScene, agents: DeviceAgents, query, params, ckpt_every=50):
    """Differentiable total costs [N_a] (and the selected agent) with respect to
    agents.k_a, agents.d_a, agents.k_f and agents.omega (tensors that may require grad).
    The adjoint covers the rotation-vector circular field only: agents.heuristic must be None."""
    if getattr(agents, "heuristic", None) is not None:
        raise GmappError(EINVAL, "rollout_cost: the adjoint runs the rotation-vector circular field only "
                                 "(agents.heuristic must be None)")
    Fn = _RolloutCost.get()
    return Fn.apply(gctx, scene, agents.r_d, agents.r_a, query, params, int(ckpt_every), agents.k_a, agents.d_a,
                    agents.k_f, agents.omega)
