"""GPU parity of the adjoint rollout (gmapp_rollout_backward) against the FP64
oracle's dual-number gradient, and the autograd wiring."""
import copy

import numpy as np
import pytest

import oracle
from paper_2606_12579_amd import scenes
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

NAMES = ("k_a", "d_a", "k_f", "omega_x", "omega_y", "omega_z")


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2606_12579_amd import gmapp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = gmapp.Context(0)
    yield c
    c.close()


def _gpu_grads(ctx, pb, w, ckpt=50):
    import torch
    from paper_2606_12579_amd import gmapp
    sc = gmapp.scene_to_device(pb.scene)
    ag = gmapp.agents_to_device(pb.agents)
    g = ctx.rollout_backward(sc, ag, pb.query, pb.params, torch.as_tensor(w, dtype=torch.float32, device="cuda"),
                             ckpt)
    torch.cuda.synchronize()
    return np.concatenate([g["k_a"].cpu().numpy()[:, None], g["d_a"].cpu().numpy()[:, None],
                           g["k_f"].cpu().numpy()[:, None], g["omega"].cpu().numpy()], 1).astype(np.float64)


def _check(pb, gpu, ref, w, rel=5e-3, label="", fwd=None):
    """Per parameter column: |g_gpu - g_or| <= rel * max(|g_or|, 1e-3 max_i |g_or_i|) + 16 * 2^-24 |w_i C_i| / theta:
    FP32 reverse-mode rounding grows with the horizon, the first floor covers near-zero entries, the second
    entries whose response to a relative change of the parameter theta (k_a, d_a, k_f; 1 for the unit vector
    omega) lies below 16 FP32 roundings of the weighted cost, which an FP32 evaluation of the cost cannot
    resolve.  fwd: the device's forward trajectories of the same agents, which place the kinks of C_obs."""
    exp = ref[:, 1:] * w[:, None]
    scale = np.abs(exp).max(0)
    err = np.abs(gpu - exp)
    theta = np.stack([pb.agents.k_a, pb.agents.d_a, pb.agents.k_f] + [np.ones(pb.agents.n)] * 3, 1)
    theta = np.abs(theta.astype(np.float64))
    resolve = 16 * 2.0 ** -24 * np.abs(w * ref[:, 0])[:, None] / np.maximum(theta, 1e-30)
    bound = rel * np.maximum(np.abs(exp), 1e-3 * scale[None, :]) + resolve + 1e-9
    # an agent whose nearest two spheres are tied, at some step, to within what separates the device's
    # trajectory from the oracle's sits on a kink of C_obs (the argmin of rho_min may switch there): its
    # gradient has two one-sided values and either trajectory may take either; such agents are counted,
    # not compared
    kink = np.zeros(pb.agents.n, bool)
    if fwd is not None:
        orc = oracle.rollout(pb).traj
        sep = np.abs(fwd.astype(np.float64) - orc).max(axis=(1, 2))
        kink = gu.nearest_sphere_gap(pb, orc) <= 2 * sep + 1e-8
    bound[kink] = np.inf
    worst = (err / bound).max(0)
    print(f"{label} adjoint worst err/bound per column " + ", ".join(f"{n} {v:.2e}" for n, v in zip(NAMES, worst))
          + f"; agents at a kink of C_obs: {int(kink.sum())} of {len(kink)}", flush=True)
    assert kink.sum() <= max(1, len(kink) // 4), ("agents at a kink", int(kink.sum()), len(kink))
    assert (err <= bound).all(), (label, worst)


@pytest.mark.parametrize("case", ["static", "moving", "ckpt7", "hard_cutoff_far", "sharded"])
def test_adjoint_small(ctx, case):
    """Small problems against the dual-number oracle; "sharded" has few agents and
    2,000 moving points, so the points are split over several workgroups that
    exchange every reduction."""
    pb = scenes.tiny(12, n_points=120, n_agents=6, n_steps=90, cutoff=1, moving=(case == "moving"))
    if case == "sharded":
        pb = scenes.tiny(14, n_points=2000, n_agents=8, n_steps=90, cutoff=1, moving=True)
    pb.agents.k_f[:] = 0.02
    ckpt = 7 if case == "ckpt7" else 50
    if case == "hard_cutoff_far":
        pb.params.cutoff = 0
        pb.scene = scenes.Scene(pb.scene.x + 3.0, pb.scene.y, pb.scene.z)   # no sphere within r_d: smooth
    w = np.random.default_rng(0).uniform(0.5, 1.5, pb.agents.n).astype(np.float32)
    gpu = _gpu_grads(ctx, pb, w, ckpt)
    ref = oracle.rollout_grad(pb)
    _check(pb, gpu, ref, w.astype(np.float64), label=case, fwd=gu.gpu_rollout(ctx, pb)["traj"])


def test_adjoint_config4_sampled(ctx):
    """128 agents, 400 steps, 20,000 noisy sphere points, C1 taper, checkpoints
    every 50 steps; the oracle's dual-number gradient on 33 agents spread over the
    ensemble (every fourth, and the last)."""
    pb = scenes.config4()
    w = np.ones(pb.agents.n, np.float32)
    gpu = _gpu_grads(ctx, pb, w, 50)
    idx = np.append(np.arange(0, pb.agents.n, 4), pb.agents.n - 1)
    sub = copy.deepcopy(pb)
    sub.agents = pb.agents.subset(idx)
    ref = oracle.rollout_grad(sub)
    _check(sub, gpu[idx], ref, w[idx].astype(np.float64), label="config4", fwd=gu.gpu_rollout(ctx, pb)["traj"][idx])


def test_autograd_function(ctx):
    import torch
    from paper_2606_12579_amd import gmapp
    pb = scenes.tiny(13, n_points=80, n_agents=5, n_steps=60, cutoff=1)
    sc = gmapp.scene_to_device(pb.scene)
    ag = gmapp.agents_to_device(pb.agents)
    for t in (ag.k_a, ag.d_a, ag.k_f, ag.omega):
        t.requires_grad_(True)
    total, best = gmapp.rollout_cost(ctx, sc, ag, pb.query, pb.params)
    w = torch.linspace(0.5, 1.5, pb.agents.n, device="cuda")
    (total * w).sum().backward()
    direct = _gpu_grads(ctx, pb, w.cpu().numpy())
    got = np.concatenate([ag.k_a.grad.cpu().numpy()[:, None], ag.d_a.grad.cpu().numpy()[:, None],
                          ag.k_f.grad.cpu().numpy()[:, None], ag.omega.grad.cpu().numpy()], 1)
    np.testing.assert_allclose(got, direct, rtol=1e-6, atol=1e-9)
    ref = oracle.rollout(pb)
    np.testing.assert_allclose(total.detach().cpu().numpy(), ref.cost[:, 4], rtol=1e-4, atol=1e-5)
