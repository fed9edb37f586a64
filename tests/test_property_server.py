"""Property sweep on the GPU for the replanning server (gmapp_server_*): random mixes
of 1-6 small requests (empty worlds and empty ensembles included, moving or static,
cut-off or taper), random memory budgets, slot counts and step quanta, submitted
back to back or spread out, some cancelled at once.  Every completed request gives
the oracle's rollout (positions, costs, the selection rule); a cancelled one either
completed first (then it is held to the same bar) or reports ECANCELLED with no
agent; the counters add up and stay within the budget and the slots."""
import time

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_2606_12579_amd import scenes
from tests.test_server import _check_oracle, _collect

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
    c.close()


request = st.tuples(st.integers(0, 2 ** 31 - 1), st.integers(0, 200), st.integers(0, 12), st.integers(1, 60),
                    st.booleans(), st.integers(0, 1), st.booleans())


def _problem(seed, n_o, n_a, n_k, moving, cutoff):
    pb = scenes.tiny(seed, n_points=n_o, n_agents=max(n_a, 1), n_steps=n_k, moving=moving and n_o > 0,
                     cutoff=cutoff)
    if n_a == 0:
        pb.agents = pb.agents.subset([])
    return pb


@settings(max_examples=30, **SETTINGS)
@given(reqs=st.lists(request, min_size=1, max_size=6), budget=st.sampled_from([1 << 20, 64 << 20]),
       slots=st.integers(1, 4), quantum=st.integers(1, 32), spread=st.booleans())
def test_random_request_mixes(ctx, reqs, budget, slots, quantum, spread):
    from paper_2606_12579_amd import gmapp
    pbs = [_problem(*r[:6]) for r in reqs]
    cancel = [r[6] and i % 2 == 1 for i, r in enumerate(reqs)]
    print(f"requests {[(p.scene.n, p.agents.n, p.params.n_steps) for p in pbs]} cancel {cancel} budget {budget} "
          f"slots {slots} quantum {quantum} spread {spread}", flush=True)
    srv = ctx.server(memory_budget=budget, max_active=slots, quantum_steps=quantum)
    try:
        ids = []
        for pb, c in zip(pbs, cancel):
            ids.append(srv.submit(pb, traj=True))
            if c:
                try:
                    srv.cancel(ids[-1])
                except gmapp.GmappError:              # already finished
                    pass
            if spread:
                time.sleep(0.001)
        res = _collect(srv, ids)
        for pb, c, r in zip(pbs, cancel, res):
            if c and r["status"] == gmapp.ECANCELLED:
                assert r["best"] == -1
                continue
            _check_oracle(pb, r, oracle.rollout(pb))
        st = srv.stats()
        n_cancelled = sum(r["status"] == gmapp.ECANCELLED for r in res)
        assert st["fault"] == 0
        assert st["completed"] == len(pbs) - n_cancelled and st["cancelled"] == n_cancelled
        assert st["max_active_seen"] <= slots and st["peak_bytes"] <= budget
    finally:
        srv.close()
