"""The serving loop on the GPU: every served request's final state equals,
agent by agent (ids, species, position bits, and the last step's cell ids,
events and partners), the oracle's for the same model run alone, whether
the requests are served concurrently (several resident, on streams of their
own, in chunks of graph-replayed steps), one at a time, or with a budget
smaller than the requests that serialises admission; the library's state
digest of each result equals the digest computed from its export."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import assert_same, say, state_digest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_14603_amd as mabm
    mabm.lib()


def _requests():
    return W.c5_requests(6, seed=3, n_min=5_000, n_max=40_000, h_min=30, h_max=150)


def _oracle_state(m, grid):
    o = oracle.OracleSim(m, grid_n=grid)
    o.step(m.steps)
    c, t = o.counts()
    assert t == m.steps
    return c, o.export()


def check_served(res, models, where):
    by_name = {m.name: m for m in models}
    assert sorted(r.name for r in res) == sorted(by_name)
    for r in res:
        want_c, want_e = _oracle_state(by_name[r.name], r.grid)
        assert np.array_equal(r.counts, want_c), (r.name, where)
        assert_same(r.state, want_e, f"{r.name} {where}")
        assert r.digest == state_digest(r.state), (r.name, where)


def test_concurrent_fifo_and_budgeted_serving_match_the_oracle():
    from paper_2606_14603_amd import serve, arena_bytes
    models = _requests()
    arrivals = np.array([0.0, 0.0, 0.001, 0.002, 0.002, 0.004])
    for kw in (dict(max_active=4, chunk=32), dict(max_active=1, chunk=64),
               dict(max_active=8, chunk=16, budget_bytes=2 * max(arena_bytes(m) for m in models))):
        budget = kw.pop("budget_bytes", 1 << 34)
        res = serve.Server(budget, record=True, keep_state=True, **kw).run(models, arrivals)
        check_served(res, models, str(kw))
        for r in res:
            assert r.completed_s >= r.admitted_s >= r.arrival_s - 1e-3
        s = serve.summarize(res)
        say(f"[serve] {kw} p50={s['p50_s']:.4f}s p99={s['p99_s']:.4f}s")
