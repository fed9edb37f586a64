"""Property sweep of the batched persistent launch on the GPU: random mixes of 1-5
tiny jobs (N_O 0-200, N_a 0-24, N_k 1-40, moving or static, cut-off or taper) under
random tunings (tile size, workgroups per CU, balance, item shape), each job run
whole or in random quanta of steps resumed from the device state, every job against
its own FP64 oracle rollout (positions 1e-4 m, costs, the selection rule)."""
import copy

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_2606_12579_amd import scenes
from tests.test_parity_batch import _check, _host, _jobs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2606_12579_amd import gmapp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = gmapp.Context(0)
    yield c
    c.clear_batch_tuning()
    c.close()


job = st.tuples(st.integers(0, 2 ** 31 - 1), st.integers(0, 200), st.integers(0, 24), st.integers(1, 40),
                st.booleans(), st.integers(0, 1))
tuning = st.tuples(st.sampled_from([0, 64, 96, 256, 4096]), st.integers(0, 2), st.sampled_from([0, 1, 4, 16]),
                   st.integers(0, 8))


def _problem(seed, n_o, n_a, n_k, moving, cutoff):
    pb = scenes.tiny(seed, n_points=n_o, n_agents=max(n_a, 1), n_steps=n_k, moving=moving and n_o > 0,
                     cutoff=cutoff)
    if n_a == 0:
        pb.agents = pb.agents.subset([])
    return pb


@settings(max_examples=60, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.function_scoped_fixture, HealthCheck.too_slow])
@given(jobs=st.lists(job, min_size=1, max_size=5), tune=tuning, quantum=st.sampled_from([0, 1, 5, 13]))
def test_random_batches(ctx, jobs, tune, quantum):
    pbs = [_problem(*j) for j in jobs]
    print(f"jobs {[(p.scene.n, p.agents.n, p.params.n_steps) for p in pbs]} tuning {tune} quantum {quantum}",
          flush=True)
    ctx.set_batch_tuning(*tune)
    try:
        js = _jobs(ctx, pbs, state=quantum > 0)
        if quantum == 0:
            ctx.rollout_batch(js)
        else:                                   # the horizon in quanta, state kept on the device
            k = [1] * len(js)
            while True:
                live = []
                for i, j in enumerate(js):
                    if k[i] <= j.params.n_steps:
                        jj = copy.copy(j)
                        jj.k_begin, jj.k_end = k[i], min(k[i] + quantum, j.params.n_steps + 1)
                        k[i] = jj.k_end
                        live.append(jj)
                if not live:
                    break
                ctx.rollout_batch(live)
        for pb, j in zip(pbs, js):
            _check(pb, _host(j), oracle.rollout(pb))
    finally:
        ctx.clear_batch_tuning()
