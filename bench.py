"""Benchmark: agent-step-point interactions/s of the batched multi-agent rollout.

One step = one planning cycle of the whole hot path (gmapp_rollout: the N_k-step
rollout of all agents with the pairwise circular-field pass, integration, costs
and selection) over the 64-agent, 500-step, 50,000-point moving scene (inputs
resident in HBM before the timed region).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--replans R] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12          # MI355X FP32 vector peak, FLOP/s
FLOP_PER_INTERACTION = 25     # algorithmic FP32 work of one (agent, sphere, step) evaluation


def _percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if xs else None


def cpu_baseline(pb_full):
    """The FP64 oracle on a bounded sample of the same workload (all agents, the
    first 200 steps), timed on this host's cores."""
    import copy
    import oracle
    sub = copy.deepcopy(pb_full)
    sub.params.n_steps = min(200, pb_full.params.n_steps)
    t0 = time.perf_counter()
    oracle.rollout(sub)
    dt = time.perf_counter() - t0
    n = oracle.interactions(sub)
    return {"value": n / dt, "unit": "interactions/s", "cores": oracle.n_threads(), "kind": "oracle",
            "sample": f"FP64 oracle, all {sub.agents.n} agents x first {sub.params.n_steps} steps x "
                      f"{sub.scene.n} points ({n:.3g} interactions) in {dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--replans", type=int, default=2000, help="back-to-back replans for the latency percentiles")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU (oracle) baseline")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the rollout shards scenes and agents with no per-step traffic, "
              "so a multi-GPU figure is not produced here (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2606_12579_amd import gmapp, scenes

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    pb = scenes.config2()
    ctx = gmapp.Context(0)
    sc = gmapp.scene_to_device(pb.scene, dev)
    ag = gmapp.agents_to_device(pb.agents, dev)
    na, nk, no = pb.agents.n, pb.params.n_steps, pb.scene.n
    out = ctx.rollout(sc, ag, pb.query, pb.params)          # allocates the outputs once
    tiling = ctx.get_tiling(no, na, nk, pb.scene.n_seg, pb.params.cutoff)
    stream = torch.cuda.current_stream(dev)
    for _ in range(args.warmup):
        ctx.rollout(sc, ag, pb.query, pb.params, out=out, stream=stream)
    torch.cuda.synchronize()

    # ---- timed region: K rollouts back to back, HIP events around each launch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        ctx.rollout(sc, ag, pb.query, pb.params, out=out, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    ms_step = wall * 1e3 / args.steps
    inter = float(na) * nk * no
    value = inter / (wall / args.steps)
    avg_kernel_s = float(np.mean(kern_ms)) * 1e-3
    achieved = inter * FLOP_PER_INTERACTION / avg_kernel_s

    # ---- replan loop: the scene stays resident, obstacles advance 1 ms per cycle,
    # the start follows the selected agent; latency = launch to result on the host
    lat = []
    q = pb.query
    import copy
    q = copy.deepcopy(pb.query)
    pin = torch.empty(4, dtype=torch.float32, pin_memory=True)
    for r in range(args.replans):
        t_a = time.perf_counter()
        o = ctx.rollout(sc, ag, q, pb.params, out=out, stream=stream)
        b = o["best"].item()                                   # synchronises
        if 0 <= b < na:
            pin[:3].copy_(o["traj"][b, 1])
        t_b = time.perf_counter()
        lat.append(t_b - t_a)
        if 0 <= b < na:
            q.p0 = pin[:3].numpy().copy()
        q.t0 = float(np.float32((r + 1) * 1e-3))
        q.incumbent = b
    p50, p99 = _percentile(lat, 50) * 1e3, _percentile(lat, 99) * 1e3

    res = {
        "metric": "agent-step-point interactions/s + p99 replan latency at 1e-4 m pos err",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "moving 10-sphere/10-box scene, N_O=50000 points, N_a=64 agents, N_k=500 steps, "
                               "dt=1 ms (one planning cycle per step)",
                   "n_points": no, "n_agents": na, "n_steps": nk, "tiling": list(tiling)},
        "p50_replan_ms": p50,
        "p99_replan_ms": p99,
        "replans": args.replans,
        "kernel_ms_mean": avg_kernel_s * 1e3,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": None},
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(pb)
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
