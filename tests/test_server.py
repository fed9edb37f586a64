"""GPU tests of the replanning server (gmapp_server_*): requests admitted by
memory and slots, advanced in quanta by control-cycle graph replays with their
state on the device, give the oracle's results; each result is identical alone
and in the mix; deadlines, cancellation and refusals are reported."""
import copy
import time

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


def _collect(srv, ids, timeout_s=120.0):
    got = {}
    t0 = time.time()
    while len(got) < len(ids):
        assert time.time() - t0 < timeout_s, f"server gave {len(got)} of {len(ids)} completions"
        for c in srv.poll(wait_ms=500):
            got[c["id"]] = c
    return [got[i] for i in ids]


def _problems():
    pbs = [scenes.config1(),
           scenes.tiny(21, n_points=300, n_agents=13, n_steps=45),
           scenes.tiny(22, n_points=200, n_agents=9, n_steps=80, moving=True),
           scenes.tiny(23, n_points=150, n_agents=5, n_steps=33, cutoff=1),
           scenes.config2(seed=5, n_points=4000, n_agents=24, n_steps=70),
           scenes.tiny(24, n_points=1, n_agents=3, n_steps=12)]
    z = scenes.tiny(25, n_points=20, n_agents=4, n_steps=10)
    z.agents = z.agents.subset([])
    pbs.append(z)
    return pbs


def _check_oracle(pb, c, ref):
    assert c["status"] == 0, c
    res = {"traj": c["traj"], "cost": c["cost"], "min_clear": None}
    gu.compare_rollout(pb, res, ref)
    if pb.agents.n == 0:
        assert c["best"] == -1
    else:
        gu.check_selection(c["best"], ref.cost, c["cost"])


def test_server_mix_matches_oracle_and_alone(ctx):
    pbs = _problems()
    refs = [oracle.rollout(pb) for pb in pbs]
    ctx.set_batch_tuning(0, 0, 0, 2)               # item shape fixed: results independent of the mix
    budget = 1 << 20                               # 1 MiB: not all requests fit at once
    srv = ctx.server(memory_budget=budget, max_active=3, quantum_steps=16)
    try:
        ids = [srv.submit(pb, traj=True) for pb in pbs]
        mix = _collect(srv, ids)
        st = srv.stats()
        _log(f"server stats {st}")
        assert st["fault"] == 0 and st["completed"] == len(pbs)
        assert st["max_active_seen"] <= 3 and st["peak_bytes"] <= budget
        assert st["p50_s"] <= st["p99_s"] <= st["max_s"]
        for pb, c, ref in zip(pbs, mix, refs):
            _check_oracle(pb, c, ref)
        # alone: one request at a time through the same loop
        for pb, c in zip(pbs, mix):
            (a,) = _collect(srv, [srv.submit(pb, traj=True)])
            assert a["best"] == c["best"], pb.name
            assert np.array_equal(a["cost"], c["cost"]), pb.name
            assert np.array_equal(a["traj"], c["traj"]), pb.name
    finally:
        srv.close()
        ctx.clear_batch_tuning()


def test_server_overlapping_arrivals(ctx):
    """Requests submitted while others run join at the next cycle (continuous
    batching), with the automatic per-job item shapes; results match the oracle."""
    pbs = _problems()[:5]
    refs = [oracle.rollout(pb) for pb in pbs]
    srv = ctx.server(memory_budget=64 << 20, max_active=8, quantum_steps=8)
    try:
        ids = []
        for pb in pbs:
            ids.append(srv.submit(pb, traj=True))
            time.sleep(0.002)
        res = _collect(srv, ids)
        for pb, c, ref in zip(pbs, res, refs):
            _check_oracle(pb, c, ref)
        st = srv.stats()
        assert st["completed"] == len(pbs) and st["cycles"] >= max(pb.params.n_steps for pb in pbs) // 8
    finally:
        srv.close()


def test_server_deadline_cancel_refuse(ctx):
    from paper_2606_12579_amd import gmapp
    srv = ctx.server(memory_budget=1 << 20, max_active=1, quantum_steps=4)
    try:
        long_pb = scenes.config2(seed=6, n_points=4000, n_agents=16, n_steps=400)
        a = srv.submit(long_pb, deadline_s=1e-4)            # cannot finish in 0.1 ms
        b = srv.submit(scenes.tiny(26, n_points=50, n_agents=4, n_steps=300))
        srv.cancel(b)
        big = copy.deepcopy(long_pb)
        big.scene = scenes.objects_scene(np.random.default_rng(1), 200_000)
        with pytest.raises(gmapp.GmappError) as ei:             # can never fit the budget
            srv.submit(big)
        assert ei.value.status == gmapp.EINVAL
        c = srv.submit(scenes.tiny(27, n_points=50, n_agents=4, n_steps=20))
        res = {r["id"]: r for r in _collect(srv, [a, b, c])}
        assert res[a]["status"] == gmapp.ETIMEOUT and res[a]["best"] == -1
        assert res[b]["status"] == gmapp.ECANCELLED
        assert res[c]["status"] == 0
        st = srv.stats()
        assert st["expired"] == 1 and st["cancelled"] == 1 and st["rejected"] == 1 and st["completed"] == 1
        with pytest.raises(gmapp.GmappError):
            srv.cancel(c)                                     # already finished
    finally:
        srv.close()


def test_server_cancel_stops_the_running_cycle(ctx):
    """Cancelling a request whose work is on the GPU stops it there: a one-cycle request
    (quantum = its horizon) completes with ECANCELLED well before its uncancelled time
    once cancelled mid-cycle, and the loop goes on unaffected (oracle parity on a small
    request afterwards)."""
    from paper_2606_12579_amd import gmapp
    long_pb = scenes.config2(seed=7, n_points=200_000, n_agents=128, n_steps=1000)
    srv = ctx.server(memory_budget=1 << 30, max_active=4, quantum_steps=1000)
    try:
        (w,) = _collect(srv, [srv.submit(long_pb)])        # first launch of the loop's kernels
        assert w["status"] == 0, w
        t0 = time.time()
        (ra,) = _collect(srv, [srv.submit(long_pb)])
        full = time.time() - t0
        assert ra["status"] == 0, ra
        _log(f"uncancelled one-cycle request: {full * 1e3:.1f} ms")
        assert full > 0.04, full                      # long enough to cancel mid-cycle
        b = srv.submit(long_pb)
        time.sleep(0.3 * full)                        # admitted, uploaded and running by now
        t1 = time.time()
        srv.cancel(b)
        (rb,) = _collect(srv, [b])
        stop = time.time() - t1
        _log(f"cancelled mid-cycle: completion {stop * 1e3:.1f} ms after the cancel, status {rb['status']}")
        assert rb["status"] == gmapp.ECANCELLED and rb["best"] == -1
        assert stop < 0.5 * full, (stop, full)
        small = scenes.tiny(28, n_points=80, n_agents=5, n_steps=60)
        c = srv.submit(small, traj=True)
        (rc,) = _collect(srv, [c])
        _check_oracle(small, rc, oracle.rollout(small))
    finally:
        srv.close()
