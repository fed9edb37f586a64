"""GPU parity of the batched persistent launch (gmapp_rollout_batch, the graph of
one control cycle gmapp_batch_*, the autotuners) against the FP64 oracle, through
the C ABI: every job of a mixed batch matches its own oracle rollout, a job's
result is the same alone and in a mix, step ranges resumed from the device state
reproduce the whole-horizon launch bit for bit, and graph replays reproduce the
direct launch."""
import copy

import numpy as np
import pytest

import oracle
from paper_2606_12579_amd import scenes
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


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


def _mix():
    """Uneven small problems: static, moving, tapered, ragged agent counts, an
    empty world, one point, zero agents."""
    pbs = [scenes.config1(),
           scenes.tiny(11, n_points=300, n_agents=13, n_steps=25),
           scenes.tiny(12, n_points=200, n_agents=9, n_steps=50, moving=True),
           scenes.tiny(13, n_points=150, n_agents=5, n_steps=50, cutoff=1),
           scenes.tiny(14, n_points=1, n_agents=3, n_steps=30),
           scenes.config2(seed=3, n_points=3000, n_agents=40, n_steps=60),
           scenes.tiny(15, n_points=37, n_agents=70, n_steps=20, moving=True)]
    e = scenes.tiny(16, n_points=37, n_agents=6, n_steps=40)
    e.scene = scenes.Scene(np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.float32))
    pbs.append(e)
    z = scenes.tiny(17, n_points=20, n_agents=4, n_steps=10)
    z.agents = z.agents.subset([])
    pbs.append(z)
    return pbs


def _jobs(ctx, pbs, state=False):
    import torch
    from paper_2606_12579_amd import gmapp
    jobs = []
    for pb in pbs:
        st = torch.zeros((pb.agents.n, gmapp.STATE_FLOATS), dtype=torch.float32, device=ctx.device) if state else None
        jobs.append(gmapp.BatchJob(gmapp.scene_to_device(pb.scene, ctx.device),
                                   gmapp.agents_to_device(pb.agents, ctx.device), pb.query, pb.params,
                                   ctx.outputs(pb.agents.n, pb.params.n_steps), st))
    return jobs


def _host(job):
    import torch
    torch.cuda.synchronize()
    r = {k: (v.cpu().numpy() if v is not None else None) for k, v in job.out.items()}
    r["best"] = int(r["best"][0])
    return r


def _check(pb, res, ref):
    gu.compare_rollout(pb, res, ref)
    if pb.agents.n == 0:
        assert res["best"] == -1
    else:
        assert 0 <= res["best"] < pb.agents.n
        gu.check_selection(res["best"], ref.cost, res["cost"])


@pytest.fixture(scope="module")
def mix_refs():
    pbs = _mix()
    return pbs, [oracle.rollout(pb) for pb in pbs]


@pytest.mark.parametrize("tuning", [None, (0, 0, 0, 1), (0, 0, 0, 4), (0, 0, 0, 5), (0, 0, 0, 8), (64, 1, 0, 2),
                                    (256, 0, 4, 0), (512, 2, 0, 7), (12288, 1, 1, 3)])
def test_batch_mix_matches_oracle(ctx, mix_refs, tuning):
    """Every job of a mixed batch matches its own oracle rollout, for item shapes
    (wave / workgroup items, 1..8 agents per group), LDS-resident and streamed
    worlds (tiles of 64..12288 points), workgroups per CU and balance."""
    pbs, refs = mix_refs
    if tuning is None:
        ctx.clear_batch_tuning()
    else:
        ctx.set_batch_tuning(*tuning)
    _log(f"batch tuning {ctx.get_batch_tuning()}")
    jobs = _jobs(ctx, pbs)
    ctx.rollout_batch(jobs)
    for pb, j, ref in zip(pbs, jobs, refs):
        _check(pb, _host(j), ref)
    ctx.clear_batch_tuning()


@pytest.mark.parametrize("shape", [2, 6])
def test_step_ranges_resume_bit_exact(ctx, mix_refs, shape):
    """A horizon run in quanta of steps (state kept on the device between launches)
    gives bit-identical results to the whole-horizon launch with the same item shape."""
    pbs, refs = mix_refs
    ctx.set_batch_tuning(0, 0, 0, shape)
    whole = _jobs(ctx, pbs)
    ctx.rollout_batch(whole)
    parts = _jobs(ctx, pbs, state=True)
    q = 7
    k = {id(j): 1 for j in parts}
    while True:
        live = []
        for j in parts:
            b = k[id(j)]
            if b <= j.params.n_steps:
                jj = copy.copy(j)
                jj.k_begin, jj.k_end = b, min(b + q, j.params.n_steps + 1)
                k[id(j)] = jj.k_end
                live.append(jj)
        if not live:
            break
        ctx.rollout_batch(live)
        q += 3                                      # uneven quanta
    for pb, a, b, ref in zip(pbs, whole, parts, refs):
        ra, rb = _host(a), _host(b)
        for key in ("traj", "cost", "min_clear"):
            assert np.array_equal(ra[key], rb[key], equal_nan=True), (pb.name, key)
        assert ra["best"] == rb["best"]
        _check(pb, rb, ref)
    ctx.clear_batch_tuning()


def test_alone_equals_in_mix(ctx, mix_refs):
    """A job's result does not depend on the other jobs of the launch (same item shape)."""
    pbs, _ = mix_refs
    ctx.set_batch_tuning(0, 0, 0, 3)
    mix = _jobs(ctx, pbs)
    ctx.rollout_batch(mix)
    for i in (0, 2, 5):
        alone = _jobs(ctx, [pbs[i]])
        ctx.rollout_batch(alone)
        ra, rb = _host(alone[0]), _host(mix[i])
        for key in ("traj", "cost", "min_clear"):
            assert np.array_equal(ra[key], rb[key]), (pbs[i].name, key)
        assert ra["best"] == rb["best"]
    ctx.clear_batch_tuning()


def test_graph_replays_match_direct(ctx, mix_refs):
    """The instantiated control-cycle graph (table copy + kernel) reproduces the
    direct launch on every replay, with eager work between replays, and after the
    job set changes (smaller table)."""
    import torch
    pbs, refs = mix_refs
    ctx.set_batch_tuning(0, 0, 0, 1)
    direct = _jobs(ctx, pbs)
    ctx.rollout_batch(direct)
    want = [_host(j) for j in direct]
    b = ctx.batch(32)
    try:
        jobs = _jobs(ctx, pbs)
        b.set_jobs(jobs)
        for rep in range(3):
            for j in jobs:
                j.out["cost"].fill_(float("nan"))
                j.out["traj"].zero_()
            b.launch()
            torch.cuda.synchronize()
            x = torch.randn(1 << 20, device=ctx.device)      # eager work between replays
            (x * 2).sum().item()
            for pb, j, w in zip(pbs, jobs, want):
                r = _host(j)
                for key in ("traj", "cost", "min_clear"):
                    assert np.array_equal(r[key], w[key]), (rep, pb.name, key)
                assert r["best"] == w["best"]
        sub = [jobs[1], jobs[3]]
        b.set_jobs(sub)
        for j in sub:
            j.out["cost"].zero_()
        b.launch()
        for i, j in zip((1, 3), sub):
            r = _host(j)
            assert np.array_equal(r["cost"], want[i]["cost"])
            _check(pbs[i], r, refs[i])
    finally:
        b.close()
        ctx.clear_batch_tuning()


def test_config5_sampled(ctx):
    """16 requests of the batched-serving workload (N_O in [1k, 200k], N_a in {16, 64, 256},
    N_k in [100, 1000]) spread over its strata, in one launch.  The oracle runs the first,
    middle and last agent of each job; each sampled agent is held to 1e-4 m when its FP64
    envelope (one FP32 ulp of the rotation vector) is below that, and otherwise, step by
    step, to twice the spread of the perturbed exact trajectories (reading R24).
    The ill-conditioned agents are counted."""
    pick = scenes.config5_stratified(16)
    pbs = [r.problem for r in scenes.config5(only=pick)]
    ctx.clear_batch_tuning()
    jobs = _jobs(ctx, pbs)
    ctx.rollout_batch(jobs)
    worst, n_ill, n_all = 0.0, 0, 0
    for pb, j in zip(pbs, jobs):
        res = _host(j)
        idx = np.array(sorted({0, pb.agents.n // 2, pb.agents.n - 1}))
        w, ill = gu.compare_conditioned(pb, res, idx, pb.name)
        worst, n_ill, n_all = max(worst, w), n_ill + ill, n_all + len(idx)
        _log(f"{pb.name}: N_O={pb.scene.n} N_a={pb.agents.n} N_k={pb.params.n_steps} ok ({ill} ill-conditioned)")
    _log(f"config5 stratified: {n_all} sampled agents, {n_ill} ill-conditioned, "
         f"well-conditioned pos err {worst:.2e}")


def test_autotuners(ctx, mix_refs):
    """The autotuners return a valid choice, cache it, and later launches that use
    it still match the oracle."""
    from paper_2606_12579_amd import gmapp
    pbs, refs = mix_refs
    pb = pbs[0]
    sc, ag = gmapp.scene_to_device(pb.scene), gmapp.agents_to_device(pb.agents)
    ctx.clear_tiling()
    t, ms = ctx.autotune_rollout(sc, ag, pb.query, pb.params, proxy_steps=20)
    _log(f"autotuned rollout tiling {t} ({ms:.3f} ms proxy)")
    assert ms > 0 and ctx.get_tiling(pb.scene.n, pb.agents.n, pb.params.n_steps) == t
    gu.compare_rollout(pb, gu.gpu_rollout(ctx, pb), refs[0])
    jobs = _jobs(ctx, pbs)
    tu, ms = ctx.autotune_batch(jobs, proxy_steps=8)
    _log(f"autotuned batch {tu} ({ms:.3f} ms proxy)")
    assert ms > 0 and ctx.get_batch_tuning()[:3] == tu[:3]
    ctx.rollout_batch(jobs)
    for p, j, ref in zip(pbs, jobs, refs):
        _check(p, _host(j), ref)


def test_batch_validation(ctx, mix_refs):
    from paper_2606_12579_amd import gmapp
    pbs, _ = mix_refs
    jobs = _jobs(ctx, pbs[:2])
    bad = copy.copy(jobs[1])
    bad.k_begin, bad.k_end = 3, 5                   # partial range without state
    with pytest.raises(gmapp.GmappError) as ei:
        ctx.rollout_batch([jobs[0], bad])
    assert ei.value.status == gmapp.EINVAL and "job 1" in str(ei.value)
    bad.k_begin, bad.k_end = 0, 5
    with pytest.raises(gmapp.GmappError):
        ctx.rollout_batch([bad])
    with pytest.raises(gmapp.GmappError) as ei:
        ctx.rollout_batch([])
    assert ei.value.status == gmapp.EINVAL
    with pytest.raises(gmapp.GmappError) as ei:
        ctx.set_batch_tuning(5, 0, 0, 0)
    assert ei.value.status == gmapp.EINVAL
    many = scenes.tiny(18, n_points=200, n_agents=2, n_steps=5)
    n = 70
    cut = np.linspace(0, 200, n + 1).astype(np.int32)
    many.scene.seg_begin = cut
    many.scene.seg_vel = np.zeros((n, 3), np.float32)
    with pytest.raises(gmapp.GmappError) as ei:
        ctx.rollout_batch(_jobs(ctx, [many]))
    assert ei.value.status == gmapp.ECAPACITY


def test_config5_ill_conditioned_agent(ctx):
    """An agent that runs into an obstacle (clamped distance rho = eps) is
    ill-conditioned: moving its rotation vector by one FP32 ulp, or its force by the
    1e-5 relative tolerance, moves the exact (FP64) trajectory by more than the 1e-4 m
    tolerance.  Such an agent is held, step
    by step, to twice the spread of the exact trajectories perturbed by one ulp of its
    rotation vector or by the 1e-5 relative force tolerance (reading R24), and its
    divergence from the oracle starts only after the agent has reached the clamp."""
    pb = scenes.config5(only=[3])[0].problem                # N_O = 160,579, N_a = 256, N_k = 885
    agent = 102
    jobs = _jobs(ctx, [pb])
    ctx.clear_batch_tuning()
    ctx.rollout_batch(jobs)
    gpu = _host(jobs[0])
    nom, env, _ = gu.conditioning(pb, [agent])
    err_k = np.abs(gpu["traj"][agent].astype(np.float64) - nom.traj[0]).max(1)
    err = float(err_k.max())
    first_div = int(np.argmax(err_k > 1e-5)) if (err_k > 1e-5).any() else -1
    clamp_k = np.nonzero(nom.min_clear[0] <= float(np.float32(pb.params.eps)) * 1.0001)[0]
    first_clamp = int(clamp_k[0]) + 1 if clamp_k.size else -1
    _log(f"ill-conditioned agent: envelope {env[0]:.2e} m, GPU error {err:.2e} m, first step off by > 1e-5: "
         f"{first_div}, first clamped step: {first_clamp}")
    assert env[0] > 1e-4, "the agent is expected to be ill-conditioned"
    assert first_clamp > 0 and (first_div < 0 or first_div >= first_clamp)
    gu.compare_conditioned(pb, gpu, [agent], "req3")
