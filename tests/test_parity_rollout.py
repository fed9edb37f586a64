"""GPU parity of the forward rollout (gmapp_rollout) and the teacher-forced force
query (gmapp_force_probe) against the FP64 oracle, through the C ABI."""
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


def test_config1_rollout(ctx):
    pb = scenes.config1()
    _log(f"config1 tiling {ctx.get_tiling(pb.scene.n, pb.agents.n, pb.params.n_steps)}")
    gpu = gu.gpu_rollout(ctx, pb)
    ref = oracle.rollout(pb)
    err = gu.compare_rollout(pb, gpu, ref)
    gu.check_selection(gpu["best"], ref.cost, gpu["cost"])
    _log(f"config1 pos err {err:.2e}")


# (agents per group, waves per workgroup, shards, streamed tile points, layout, group: 1 wave / 2 workgroup)
TILINGS = [(1, 1, 1, 0, 0, 1), (2, 2, 1, 0, 1, 1), (8, 4, 1, 0, 0, 1), (8, 4, 1, 256, 2, 1), (64, 1, 1, 0, 1, 1),
           (4, 4, 4, 0, 0, 1), (8, 1, 8, 128, 2, 1), (16, 8, 2, 0, 1, 1), (1, 4, 16, 0, 1, 1), (32, 2, 1, 0, 0, 1),
           (64, 4, 1, 512, 2, 1), (2, 16, 4, 0, 1, 1), (4, 2, 2, 64, 2, 1), (1, 8, 64, 0, 0, 1),
           (1, 4, 1, 0, 1, 2), (2, 8, 4, 0, 1, 2), (8, 16, 2, 0, 0, 2), (4, 4, 8, 128, 2, 2), (1, 16, 16, 0, 1, 2)]


@pytest.mark.parametrize("tiling", TILINGS)
def test_tilings_config1(ctx, tiling):
    """Every tiling (agents per group, waves, shards, tile size, layout, grouping) gives the oracle's result."""
    pb = scenes.config1()
    _log(f"config1 tiling {tiling}")
    gpu = gu.gpu_rollout(ctx, pb, tiling=tiling)
    ref = oracle.rollout(pb)
    gu.compare_rollout(pb, gpu, ref)


def test_teacher_forced_force(ctx):
    """At the oracle's own states (rounded to FP32), the GPU's Alg. 1 response
    matches the oracle's within 1e-5 relative (cancellation floor and cut-off pairs aside)."""
    import torch
    from paper_2606_12579_amd import gmapp
    ctx.clear_tiling()
    for pb in (scenes.config1(), scenes.config2(n_agents=16, n_steps=60)):
        ref = oracle.rollout(pb)
        sc = gmapp.scene_to_device(pb.scene)
        ag = gmapp.agents_to_device(pb.agents)
        worst = 0.0
        for k in (1, 2, pb.params.n_steps // 2, pb.params.n_steps):
            p32 = ref.traj[:, k - 1].astype(np.float32)
            v32 = ref.vel[:, k - 1].astype(np.float32)
            t32 = np.float32((k - 1) * np.float32(pb.params.dt))
            r = oracle.repulsion(pb, p32.astype(np.float64), v32.astype(np.float64), float(t32))
            f, rho = ctx.force_probe(sc, ag, torch.as_tensor(p32, device="cuda"), torch.as_tensor(v32, device="cuda"),
                                     float(t32), pb.params)
            torch.cuda.synchronize()
            f = f.cpu().numpy().astype(np.float64)
            d = np.linalg.norm(f - r.force, axis=1)
            bound = gu.force_bound(r)
            ratio = d / np.maximum(bound, 1e-300)
            worst = max(worst, float(ratio.max()))
            assert (d <= bound).all(), (pb.name, k, ratio.max(), d.max())
            np.testing.assert_allclose(rho.cpu().numpy(), r.rho_min, rtol=2e-6, atol=1e-9)
        _log(f"{pb.name} teacher-forced force: worst |dF|/bound = {worst:.3f}")


@pytest.mark.parametrize("case", ["empty", "one", "dupes", "single_agent", "ragged_agents", "moving", "taper",
                                  "on_point", "far"])
def test_edge_cases(ctx, case):
    pb = scenes.tiny(5, n_points=37, n_agents=6, n_steps=40)
    if case == "empty":
        pb.scene = scenes.Scene(np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.float32))
    elif case == "one":
        pb = scenes.tiny(6, n_points=1, n_agents=3, n_steps=30)
    elif case == "dupes":
        sc = pb.scene
        pb.scene = scenes.Scene(np.repeat(sc.x, 3), np.repeat(sc.y, 3), np.repeat(sc.z, 3), sc.r_obs)
    elif case == "single_agent":
        pb.agents = pb.agents.subset([2])
    elif case == "ragged_agents":
        pb = scenes.tiny(7, n_points=300, n_agents=13, n_steps=25)
    elif case == "moving":
        pb = scenes.tiny(8, n_points=200, n_agents=9, n_steps=50, moving=True)
    elif case == "taper":
        pb = scenes.tiny(9, n_points=150, n_agents=5, n_steps=50, cutoff=1)
    elif case == "on_point":
        sc = pb.scene
        sc.x[0], sc.y[0], sc.z[0] = 0.0, 0.0, 0.0          # a sphere centre at the start
    elif case == "far":
        pb.scene = scenes.Scene(pb.scene.x + 5, pb.scene.y, pb.scene.z)   # nothing within r_d
    ref = oracle.rollout(pb)
    for tiling in (None, (2, 1, 2, 0, 1, 1), (8, 2, 1, 64, 2, 1), (4, 4, 4, 0, 2, 1), (1, 2, 8, 0, 1, 1),
                   (2, 4, 4, 0, 1, 2), (1, 8, 2, 64, 2, 2)):
        gpu = gu.gpu_rollout(ctx, pb, tiling=tiling)
        gu.compare_rollout(pb, gpu, ref)
        gu.check_selection(gpu["best"], ref.cost, gpu["cost"])


def test_incumbent_rule(ctx):
    pb = scenes.config1()
    ref = oracle.rollout(pb)
    for inc in range(pb.agents.n):
        q = copy.deepcopy(pb)
        q.query.incumbent = inc
        gpu = gu.gpu_rollout(ctx, q)
        # the GPU applies the rule exactly to its own costs
        assert gpu["best"] == oracle.select(gpu["cost"][:, 4].astype(np.float64), inc, float(np.float32(0.9)))
        # and agrees with the oracle's choice unless the costs sit within tolerance of alpha C_best
        exp = oracle.select(ref.cost[:, 4], inc, float(np.float32(0.9)))
        if gpu["best"] != exp:
            tol = 2 * np.abs(gpu["cost"][:, 4] - ref.cost[:, 4]).max() + gu.SEL_GAP
            b = 0.9 * ref.cost[inc, 4]
            assert abs(ref.cost[gpu["best"], 4] - b) <= tol or abs(ref.cost[exp, 4] - b) <= tol or \
                abs(ref.cost[gpu["best"], 4] - ref.cost[exp, 4]) <= tol


def test_n_agents_zero(ctx):
    pb = scenes.config1()
    pb.agents = pb.agents.subset([])
    gpu = gu.gpu_rollout(ctx, pb)
    assert gpu["best"] == -1


def test_deterministic(ctx):
    pb = scenes.config2(n_agents=16, n_steps=50)
    for t in ((1, 8, 4, 0, 0, 1), (2, 8, 4, 0, 0, 2)):
        a = gu.gpu_rollout(ctx, pb, tiling=t)
        b = gu.gpu_rollout(ctx, pb, tiling=t)
        for k in ("traj", "cost", "min_clear"):
            assert np.array_equal(a[k], b[k]), (t, k)


def test_config2_full_size(ctx):
    """N_a = 64, N_k = 500, N_O = 50,000 moving points at the default (benchmarked)
    tiling; the oracle runs a spread subset of the agents (agents are independent)."""
    pb = scenes.config2()
    _log(f"config2 tiling {ctx.get_tiling(pb.scene.n, pb.agents.n, pb.params.n_steps, pb.scene.n_seg)}")
    gpu = gu.gpu_rollout(ctx, pb)
    idx = np.arange(0, 64, 8)
    sub = copy.deepcopy(pb)
    sub.agents = pb.agents.subset(idx)
    ref = oracle.rollout(sub)
    err = gu.compare_rollout(pb, gpu, ref, agents=idx)
    _log(f"config2 pos err {err:.2e} (agents {list(idx)})")


def test_validation_errors(ctx):
    import torch
    from paper_2606_12579_amd import gmapp
    pb = scenes.config1()
    sc = gmapp.scene_to_device(pb.scene)
    ag = gmapp.agents_to_device(pb.agents)
    bad = []
    for field, val in (("n_steps", 0), ("eps", 0.0), ("dt", -1.0), ("cutoff", 2), ("r_cost", 0.0)):
        p = copy.deepcopy(pb.params)
        setattr(p, field, val)
        bad.append(p)
    for p in bad:
        with pytest.raises(gmapp.GmappError) as ei:
            ctx.rollout(sc, ag, pb.query, p)
        assert ei.value.status == gmapp.EINVAL
    q = copy.deepcopy(pb.query)
    q.p0 = np.array([np.nan, 0, 0], np.float32)
    with pytest.raises(gmapp.GmappError):
        ctx.rollout(sc, ag, q, pb.params)
    with pytest.raises(gmapp.GmappError) as ei:
        ctx.set_tiling(3, 4, 1)
        ctx.rollout(sc, ag, pb.query, pb.params)
    assert ei.value.status == gmapp.EINVAL
    ctx.clear_tiling()
    torch.cuda.synchronize()
