"""Property sweep of the adjoint rollout on the GPU: random tiny problems (N_O 1-150,
N_a 1-8, N_k 2-60, moving or static, C1 taper), random checkpoint spacing and random
weights of the agents' costs, against the FP64 dual-number oracle gradient with the
per-column bound of the fixed adjoint tests."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_2606_12579_amd import scenes
from tests import gpu_util as gu
from tests.test_parity_adjoint import _check, _gpu_grads

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


@settings(max_examples=40, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.function_scoped_fixture, HealthCheck.too_slow])
@given(seed=st.integers(0, 2 ** 31 - 1), n_o=st.integers(1, 150), n_a=st.integers(1, 8), n_k=st.integers(2, 60),
       moving=st.booleans(), ckpt=st.integers(1, 64), kf=st.sampled_from([0.005, 0.01, 0.02]))
def test_random_adjoint(ctx, seed, n_o, n_a, n_k, moving, ckpt, kf):
    pb = scenes.tiny(seed, n_points=n_o, n_agents=n_a, n_steps=n_k, moving=moving, cutoff=1)
    pb.agents.k_f[:] = kf
    w = np.random.default_rng(seed).uniform(0.5, 1.5, n_a).astype(np.float32)
    print(f"seed {seed} N_O {n_o} N_a {n_a} N_k {n_k} moving {moving} ckpt {ckpt} k_f {kf}", flush=True)
    gpu = _gpu_grads(ctx, pb, w, ckpt)
    ref = oracle.rollout_grad(pb)
    _check(pb, gpu, ref, w.astype(np.float64), label=f"seed {seed}", fwd=gu.gpu_rollout(ctx, pb)["traj"])
