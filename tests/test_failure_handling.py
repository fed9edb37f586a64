"""Failure handling of the persistent launches on the GPU: the per-wait watchdog, the
host's abort word and the host time-out (gmapp_set_watchdog, gmapp_abort,
gmapp_wait).  Every failure is forced from the host -- a tiny limit on the
kernels' own bounded waits, or the abort word raised before or during a launch --
so every kernel still reaches its end."""
import time

import numpy as np
import pytest

from paper_2606_12579_amd import scenes

pytestmark = pytest.mark.gpu

ETIMEOUT, ECANCELLED = -5, -6


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2606_12579_amd import gmapp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = gmapp.Context(0)
    yield c
    c.abort(False)
    c.set_watchdog(0.0)
    c.close()


def _log(msg):
    print(msg, flush=True)


def _rollout(ctx, pb, traj=False):
    import torch
    from paper_2606_12579_amd import gmapp
    sc, ag = gmapp.scene_to_device(pb.scene), gmapp.agents_to_device(pb.agents)
    out = ctx.rollout(sc, ag, pb.query, pb.params, traj=traj, min_clear=False)
    torch.cuda.synchronize()
    return int(out["best"].item()), out["cost"].cpu().numpy()


def _long_config2(n_steps):
    """The config-2 scene and ensemble over a long horizon: a sharded launch (4 shards per
    agent) that exchanges partial sums every step."""
    return scenes.config2(n_steps=n_steps)


def test_watchdog_limit_is_per_wait(ctx):
    """A sharded rollout many times longer than a 20 ms watchdog limit returns its
    results, identical to the run under the default limit: the limit bounds one
    wait, not the launch."""
    pb = _long_config2(30000)
    ctx.clear_tiling()
    t = ctx.get_tiling(pb.scene.n, pb.agents.n, pb.params.n_steps, pb.scene.n_seg)
    assert t[2] > 1, t
    ctx.set_watchdog(0.0)
    best0, cost0 = _rollout(ctx, pb)
    ctx.set_watchdog(0.02)
    t0 = time.perf_counter()
    best1, cost1 = _rollout(ctx, pb)
    ms = 1e3 * (time.perf_counter() - t0)
    ctx.set_watchdog(0.0)
    _log(f"30,000-step sharded rollout under a 20 ms per-wait limit: {ms:.1f} ms, best {best1}")
    assert ms > 60.0
    assert best1 == best0 and best1 >= 0
    assert np.array_equal(cost1, cost0)


def test_watchdog_limit_is_per_wait_adjoint_and_control(ctx):
    """The same for the sharded adjoint (2,000 steps) and a control launch of 20,000
    steps: a 5 ms (adjoint) or 20 ms (control) limit far below the launch's length
    leaves the results equal to those under the default limit."""
    import torch
    from paper_2606_12579_amd import gmapp
    pb = scenes.config4(n_steps=2000)
    sc, ag = gmapp.scene_to_device(pb.scene), gmapp.agents_to_device(pb.agents)
    gt = torch.ones(pb.agents.n, dtype=torch.float32, device="cuda")
    ctx.set_watchdog(0.0)
    g0 = ctx.rollout_backward(sc, ag, pb.query, pb.params, gt)
    ctx.set_watchdog(0.005)
    t0 = time.perf_counter()
    g1 = ctx.rollout_backward(sc, ag, pb.query, pb.params, gt)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0)
    _log(f"2,000-step adjoint under a 5 ms per-wait limit: {ms:.1f} ms")
    assert ms > 15.0
    for k in g0:
        assert torch.isfinite(g1[k]).all() and torch.equal(g0[k], g1[k]), k

    p2 = scenes.config2()
    sc2, ag2 = gmapp.scene_to_device(p2.scene), gmapp.agents_to_device(p2.agents)
    prm = p2.params
    prm.n_steps = 20
    ctx.set_watchdog(0.0)
    a = ctx.plan_loop(sc2, ag2, p2.query, prm, n_cycles=1, ctrl_steps=20000, ctrl_dt=1e-4)
    torch.cuda.synchronize()
    ctx.set_watchdog(0.02)
    t0 = time.perf_counter()
    b = ctx.plan_loop(sc2, ag2, p2.query, prm, n_cycles=1, ctrl_steps=20000, ctrl_dt=1e-4)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0)
    ctx.set_watchdog(0.0)
    _log(f"20,000 control steps under a 20 ms per-wait limit: {ms:.1f} ms")
    assert ms > 40.0
    assert torch.isfinite(b["robot"]).all() and torch.equal(a["robot"], b["robot"])


def test_watchdog_fires_on_a_tiny_limit(ctx):
    """A limit of one clock tick ends the first wait whose first poll finds its words
    missing: the rollout reports GMAPP_ETIMEOUT, the adjoint NaN gradients; the next
    launches under the default limit are unaffected (the status word is cleared by
    the launch's last workgroup)."""
    import torch
    from paper_2606_12579_amd import gmapp
    pb = _long_config2(500)
    ref_best, ref_cost = _rollout(ctx, pb)
    ctx.set_watchdog(1e-8)
    best, _ = _rollout(ctx, pb)
    ctx.set_watchdog(0.0)
    assert best == ETIMEOUT, best
    again, cost = _rollout(ctx, pb)
    assert again == ref_best and np.array_equal(cost, ref_cost)

    p4 = scenes.config4()
    sc, ag = gmapp.scene_to_device(p4.scene), gmapp.agents_to_device(p4.agents)
    gt = torch.ones(p4.agents.n, dtype=torch.float32, device="cuda")
    ctx.set_watchdog(1e-8)
    g = ctx.rollout_backward(sc, ag, p4.query, p4.params, gt)
    torch.cuda.synchronize()
    ctx.set_watchdog(0.0)
    assert torch.isnan(g["k_a"]).all()
    g2 = ctx.rollout_backward(sc, ag, p4.query, p4.params, gt)
    torch.cuda.synchronize()
    assert torch.isfinite(g2["k_a"]).all()


def test_abort_word(ctx):
    """With the abort word raised before the launch (and a 0.5 ms limit, so that every
    unanswered poll checks), the sharded rollout's first wait that finds its words
    missing ends: GMAPP_ECANCELLED; lowered again, the next rollout is the reference."""
    pb = _long_config2(500)
    ref_best, ref_cost = _rollout(ctx, pb)
    ctx.abort(True)
    ctx.set_watchdog(0.0005)
    try:
        best, _ = _rollout(ctx, pb)
    finally:
        ctx.abort(False)
        ctx.set_watchdog(0.0)
    assert best == ECANCELLED, best
    again, cost = _rollout(ctx, pb)
    assert again == ref_best and np.array_equal(cost, ref_cost)


def test_wait_times_out_and_aborts_a_running_launch(ctx):
    """gmapp_wait with a 10 ms limit on a rollout of about 0.1 s: it raises the abort
    word, the running launch's waits end (best = GMAPP_ECANCELLED), the launch drains,
    the call returns GMAPP_ETIMEOUT, and later launches are unaffected."""
    import torch
    from paper_2606_12579_amd import gmapp
    pb = _long_config2(30000)
    sc, ag = gmapp.scene_to_device(pb.scene), gmapp.agents_to_device(pb.agents)
    ctx.set_watchdog(0.0005)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        out = ctx.rollout(sc, ag, pb.query, pb.params, traj=False, min_clear=False)
        with pytest.raises(gmapp.GmappError) as ei:
            ctx.wait(0.01)
    finally:
        ctx.set_watchdog(0.0)
    ms = 1e3 * (time.perf_counter() - t0)
    assert ei.value.status == ETIMEOUT
    best = int(out["best"].item())
    _log(f"host time-out after 10 ms: the 30,000-step launch drained after {ms:.1f} ms with best {best}")
    assert best == ECANCELLED, best
    p = _long_config2(500)
    ref = scenes.config2()
    b1, c1 = _rollout(ctx, p)
    b2, c2 = _rollout(ctx, ref)
    assert b1 == b2 and np.array_equal(c1, c2)


def test_abort_word_stops_a_batched_launch(ctx):
    """The batched kernel reads the abort word at every work item and every 64 steps:
    raised before the launch, every job reports GMAPP_ECANCELLED in a fraction of the
    launch's normal time; lowered again, the same jobs give their normal results."""
    import torch
    from paper_2606_12579_amd import gmapp
    pbs = [scenes.config2(seed=8 + i, n_points=50_000, n_agents=64, n_steps=1000) for i in range(4)]

    def jobs():
        return [gmapp.BatchJob(gmapp.scene_to_device(pb.scene), gmapp.agents_to_device(pb.agents), pb.query,
                               pb.params, ctx.outputs(pb.agents.n, pb.params.n_steps)) for pb in pbs]

    ref = jobs()
    ctx.rollout_batch(ref)                        # warm-up and reference
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.rollout_batch(ref)
    torch.cuda.synchronize()
    full = time.perf_counter() - t0
    ab = jobs()
    ctx.abort(True)
    try:
        t0 = time.perf_counter()
        ctx.rollout_batch(ab)
        torch.cuda.synchronize()
        stopped = time.perf_counter() - t0
    finally:
        ctx.abort(False)
    _log(f"batched launch: {full * 1e3:.1f} ms, aborted before it started: {stopped * 1e3:.1f} ms")
    assert all(int(j.out["best"].item()) == ECANCELLED for j in ab)
    assert stopped < 0.5 * full, (stopped, full)
    again = jobs()
    ctx.rollout_batch(again)
    torch.cuda.synchronize()
    for a, r in zip(again, ref):
        assert int(a.out["best"].item()) == int(r.out["best"].item())
        assert torch.equal(a.out["cost"], r.out["cost"])
