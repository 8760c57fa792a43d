"""The serving loop on the GPU: every request's result (its per-species
counts after its horizon) equals the oracle's for the same model run alone,
whether the requests are served concurrently (several resident, on streams
of their own, in chunks of graph-replayed steps) or one at a time; a budget
smaller than the requests serialises admission without changing results."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import say

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


def _oracle_counts(m):
    o = oracle.OracleSim(m)
    o.step(m.steps)
    c, t = o.counts()
    assert t == m.steps
    return c


def test_concurrent_and_fifo_serving_match_the_oracle():
    from paper_2606_14603_amd import serve, arena_bytes
    models = _requests()
    want = {m.name: _oracle_counts(m) for m in models}
    arrivals = np.array([0.0, 0.0, 0.001, 0.002, 0.002, 0.004])
    for kw in (dict(max_active=4, chunk=32), dict(max_active=1, chunk=64),
               dict(max_active=8, chunk=16, budget_bytes=2 * max(arena_bytes(m) for m in models))):
        budget = kw.pop("budget_bytes", 1 << 34)
        res = serve.Server(budget, **kw).run(models, arrivals)
        assert sorted(r.name for r in res) == sorted(want)
        for r in res:
            assert np.array_equal(r.counts, want[r.name]), (r.name, kw)
            assert r.completed_s >= r.admitted_s >= r.arrival_s - 1e-3
        s = serve.summarize(res)
        say(f"[serve] {kw} p50={s['p50_s']:.4f}s p99={s['p99_s']:.4f}s")
