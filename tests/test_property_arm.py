"""Property sweep on the GPU for arm agents (gmapp_rollout_arm: Eqs. 12-14, the end
effector of a serial chain moved through the damped pseudo-inverse of its Jacobian).

Random small problems: 1-8 agents, 0-200 spheres beside the way (static or moving),
2-40 steps, chains of 1 to 7 joints (the first joints of the synthetic arm), damping
0.01-0.1 or none (with at least 6 joints; a shorter undamped chain is refused), random
goals, homogeneous or mixed heuristics, under random tilings, against the FP64 oracle: hand positions, rotors, joint
angles, clearances, costs and the selection rule, with the bounds of the fixed arm
tests."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import arm as oa
from paper_2606_12579_amd import scenes
from tests.test_parity_arm import _check, _gpu
from tests.test_property_loop import _mix

pytestmark = pytest.mark.gpu

SETTINGS = dict(deadline=None, derandomize=True,
                suppress_health_check=[HealthCheck.function_scoped_fixture, HealthCheck.too_slow])


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2606_12579_amd import gmapp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = gmapp.Context(0)
    yield c
    c.clear_tiling()
    c.close()


ARM_TILINGS = [None, (1, 8, 4, 0, 0, 2), (2, 8, 4, 0, 0, 2), (2, 1, 2, 0, 1, 1), (8, 4, 1, 64, 2, 1),
               (4, 2, 2, 0, 1, 1), (1, 1, 1, 0, 0, 1)]


@settings(max_examples=40, **SETTINGS)
@given(seed=st.integers(0, 2 ** 31 - 1), n_a=st.integers(1, 8), n_o=st.integers(0, 200), n_k=st.integers(2, 40),
       moving=st.booleans(), joints=st.integers(1, 7), damping=st.sampled_from([0.0, 0.01, 0.1]),
       mixed=st.booleans(), tiling=st.sampled_from(ARM_TILINGS))
def test_random_arm_problems(ctx, seed, n_a, n_o, n_k, moving, joints, damping, mixed, tiling):
    pb, pa, pq, L, q0 = scenes.arm_problem(seed=seed, n_agents=n_a, n_points=n_o, n_steps=n_k, moving=moving)
    if mixed:                                   # every agent its own heuristic, r_d and k_f
        pb = _mix(pb, np.random.default_rng(seed + 4))
    rng = np.random.default_rng(seed)
    pb.query.goal = (pb.query.goal + rng.uniform(-0.1, 0.1, 3)).astype(np.float32)
    Ln, qn = np.ascontiguousarray(L[:joints + 1]), np.ascontiguousarray(q0[:joints])
    print(f"seed {seed} N_a {n_a} N_O {n_o} N_k {n_k} moving {moving} joints {joints} damping {damping} "
          f"mixed {mixed} tiling {tiling}", flush=True)
    if damping == 0.0 and joints < 6:          # J_b J_b^T (6 x 6) singular: refused before any launch
        from paper_2606_12579_amd import gmapp
        with pytest.raises(gmapp.GmappError) as ei:
            _gpu(ctx, pb, pa, pq, Ln, qn, damping, tiling)
        assert ei.value.status == gmapp.EINVAL
        return
    ref = oa.rollout_arm(pb, pa, pq, Ln, qn, damping)
    gpu = _gpu(ctx, pb, pa, pq, Ln, qn, damping, tiling)
    assert gpu["joints"].shape == ref["joints"].shape
    pos_err, rot_err, j_err = _check(pb, gpu, ref)
    print(f"  pos {pos_err:.2e} rotor {rot_err:.2e} joints {j_err:.2e}", flush=True)
