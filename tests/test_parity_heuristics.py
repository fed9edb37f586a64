"""GPU parity of heterogeneous ensembles (Sec. III-A): agents that mix the
rotation-vector circular field (Eq. 2), the velocity-current field (Eq. 3 with
the relative velocity as current) and the artificial potential field (Eq. 1),
with small and large detection distances, against the FP64 oracle through the
C ABI, in every kernel path (wave and workgroup groups, sharded, streamed)."""
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


def _multi(pb, seed=11):
    pb = copy.deepcopy(pb)
    pb.agents = scenes.multi_agents(np.random.default_rng(seed), pb.agents.n)
    return pb


# (agents per group, waves, shards, streamed tile points, layout, group: 1 wave / 2 workgroup)
TILINGS = [None, (1, 1, 1, 0, 0, 1), (8, 4, 1, 256, 2, 1), (4, 4, 4, 0, 0, 1), (8, 1, 8, 128, 2, 1),
           (1, 8, 4, 0, 0, 2), (2, 8, 4, 0, 1, 2), (4, 4, 8, 128, 2, 2), (1, 16, 16, 0, 1, 2)]


@pytest.fixture(scope="module")
def multi1():
    pb = _multi(scenes.config1())
    return pb, oracle.rollout(pb)


@pytest.mark.parametrize("tiling", TILINGS)
def test_multi_config1_tilings(ctx, multi1, tiling):
    pb, ref = multi1
    _log(f"multi config1 tiling {tiling}")
    gpu = gu.gpu_rollout(ctx, pb, tiling=tiling)
    err = gu.compare_rollout(pb, gpu, ref)
    gu.check_selection(gpu["best"], ref.cost, gpu["cost"])
    _log(f"  pos err {err:.2e}")


@pytest.mark.parametrize("case", ["moving", "taper", "ragged", "all_apf", "all_vel", "out_of_range"])
def test_multi_cases(ctx, case):
    if case == "moving":
        pb = _multi(scenes.tiny(8, n_points=200, n_agents=9, n_steps=50, moving=True))
    elif case == "taper":
        pb = _multi(scenes.tiny(9, n_points=150, n_agents=6, n_steps=50, cutoff=1))
    elif case == "ragged":
        pb = _multi(scenes.tiny(7, n_points=300, n_agents=13, n_steps=25))
    elif case in ("all_apf", "all_vel"):
        pb = _multi(scenes.tiny(5, n_points=37, n_agents=6, n_steps=40))
        h = scenes.H_APF if case == "all_apf" else scenes.H_MFI_VEL
        pb.agents.heuristic = np.full(pb.agents.n, h, np.int32)
        pb.agents.k_f = np.full(pb.agents.n, scenes.K_F_APF if h == scenes.H_APF else scenes.K_F, np.float32)
    else:
        # values other than 0, 1, 2 select the rotation-vector field, in the oracle as on the device
        pb = _multi(scenes.tiny(5, n_points=37, n_agents=6, n_steps=40))
        pb.agents.heuristic = np.array([7, 1, -3, 2, 0, 100], np.int32)
    _log(f"multi case {case}: heuristics {pb.agents.heuristic.tolist()}")
    ref = oracle.rollout(pb)
    for tiling in (None, (2, 1, 2, 0, 1, 1), (8, 2, 1, 64, 2, 1), (1, 8, 2, 64, 2, 2), (2, 4, 4, 0, 1, 2)):
        gpu = gu.gpu_rollout(ctx, pb, tiling=tiling)
        gu.compare_rollout(pb, gpu, ref)
        gu.check_selection(gpu["best"], ref.cost, gpu["cost"])


def test_multi_objects_scene(ctx):
    """A 24-agent mixed ensemble over 200 steps in a 5,000-point object scene
    (agents reach the eps clamp, where the APF is steepest)."""
    pb = _multi(scenes.config2(n_agents=24, n_steps=200, n_points=5000))
    ref = oracle.rollout(pb)
    for tiling in (None, (1, 8, 4, 0, 0, 2), (8, 4, 1, 256, 2, 1)):
        gpu = gu.gpu_rollout(ctx, pb, tiling=tiling)
        err = gu.compare_rollout(pb, gpu, ref)
        gu.check_selection(gpu["best"], ref.cost, gpu["cost"])
        _log(f"multi objects tiling {tiling}: pos err {err:.2e}")


def test_multi_teacher_forced_force(ctx):
    """At the oracle's own states (rounded to FP32) the device's response of each
    heuristic matches the oracle's within the teacher-forced bound."""
    import torch
    from paper_2606_12579_amd import gmapp
    ctx.clear_tiling()
    for pb in (_multi(scenes.config1()), _multi(scenes.config2(n_agents=24, n_steps=60, n_points=5000)),
               _multi(scenes.tiny(8, n_points=200, n_agents=9, n_steps=50, moving=True))):
        ref = oracle.rollout(pb)
        sc = gmapp.scene_to_device(pb.scene)
        ag = gmapp.agents_to_device(pb.agents)
        worst = np.zeros(3)
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
            assert (d <= bound).all(), (pb.name, k, (d / np.maximum(bound, 1e-300)).max())
            for h in range(3):
                sel = pb.agents.heuristic == h
                if sel.any():
                    worst[h] = max(worst[h], float((d[sel] / np.maximum(bound[sel], 1e-300)).max()))
            np.testing.assert_allclose(rho.cpu().numpy(), r.rho_min, rtol=2e-6, atol=1e-9)
        _log(f"{pb.name} teacher-forced |dF|/bound per heuristic (CF, velocity, APF): {np.round(worst, 3)}")


def test_zero_heuristics_match_null(ctx):
    """An all-zero heuristic array runs the rotation-vector field: bit-identical to NULL."""
    pb = scenes.config2(n_agents=16, n_steps=60, n_points=5000)
    a = gu.gpu_rollout(ctx, pb)
    pz = copy.deepcopy(pb)
    pz.agents.heuristic = np.zeros(pb.agents.n, np.int32)
    b = gu.gpu_rollout(ctx, pz)
    for k in ("traj", "cost", "min_clear"):
        assert np.array_equal(a[k], b[k]), k
    assert a["best"] == b["best"]


def test_heuristics_rejected_outside_rollout(ctx):
    """Batched, adjoint and served launches run the rotation-vector field only and
    reject a heuristic array with EINVAL."""
    import torch
    from paper_2606_12579_amd import gmapp
    pb = _multi(scenes.tiny(5, n_points=37, n_agents=6, n_steps=20))
    sc = gmapp.scene_to_device(pb.scene, ctx.device)
    ag = gmapp.agents_to_device(pb.agents, ctx.device)
    job = gmapp.BatchJob(sc, ag, pb.query, pb.params, ctx.outputs(pb.agents.n, pb.params.n_steps))
    with pytest.raises(gmapp.GmappError) as ei:
        ctx.rollout_batch([job])
    assert ei.value.status == gmapp.EINVAL and "heuristic" in str(ei.value)
    g = torch.ones(pb.agents.n, dtype=torch.float32, device=ctx.device)
    with pytest.raises(gmapp.GmappError) as ei:
        ctx.rollout_backward(sc, ag, pb.query, pb.params, g)
    assert ei.value.status == gmapp.EINVAL
    with pytest.raises(gmapp.GmappError) as ei:
        gmapp.rollout_cost(ctx, sc, ag, pb.query, pb.params)
    assert ei.value.status == gmapp.EINVAL


def test_multi_full_size_sampled(ctx):
    """The benchmark's mixed-ensemble workload at full size (config-2 scene, 50,000
    moving points, 64 agents, 500 steps, the built-in tiling): eight sampled agents
    against the oracle run on those agents alone (agents are independent)."""
    pb = _multi(scenes.config2())
    idx = [0, 9, 18, 27, 36, 45, 54, 63]
    gpu = gu.gpu_rollout(ctx, pb)
    sub = copy.deepcopy(pb)
    sub.agents = pb.agents.subset(idx)
    ref = oracle.rollout(sub)
    err = gu.compare_rollout(pb, gpu, ref, agents=idx)
    _log(f"mixed full size: sampled pos err {err:.2e}")
