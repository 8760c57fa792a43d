"""The static-arena entry point (mabm_create_sim_static), for callers that
cannot allocate device memory: a simulation created in the library's
static device arena gives, bit for bit, the results of the same model
created in a caller's arena (mabm_create_sim), on two simulations in a
row, the second smaller than the first, so that the arena's stale
contents from the first must not leak into the second.  Sizes beyond the
arena, and a second simulation while one holds it, are rejected."""
import ctypes

import numpy as np
import pytest

import workloads as W
from parity import assert_same, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_14603_amd as mabm
    mabm.lib()


def _same_run(model, steps):
    import paper_2606_14603_amd as mabm
    say(f"[static] {model.name} n={model.n_agents} steps={steps}")
    a = mabm.Sim(model, record=True, static_arena=True)
    b = mabm.Sim(model, record=True)
    assert a.arena is None
    assert a.grid() == b.grid()
    for k in (1, steps - 1):
        a.step(k)
        b.step(k)
        assert_same(a.export(), b.export(), f"{model.name} static vs caller's arena")
        ca, ta = a.counts()
        cb, tb = b.counts()
        assert ta == tb and np.array_equal(ca, cb)
    assert int(a.digest()[0]) == int(b.digest()[0])
    # direct launches only: the graph flag is forced off
    assert a.agent_updates() == b.agent_updates()
    live = a.size()[0]
    a.close()
    b.close()
    return live


def test_static_arena_matches_caller_arena_twice_second_smaller():
    # births, deaths, splits, translocations and contact rules, then a
    # smaller model of another kind in the same arena
    first = W.c3(40_000, seed=5, n_genes=400).with_(name="static_c3")
    second = W.c1(n_a=1200, n_b=1000, n_c=300, box_um=0.9, seed=9, unbind_p=0.02)
    second.name = "static_c1"
    assert second.n_agents < first.n_agents
    n1 = _same_run(first, 120)
    n2 = _same_run(second, 150)
    assert n1 > n2 > 0


def test_static_arena_rejects_oversize_and_a_second_holder():
    import paper_2606_14603_amd as mabm
    big = W.c2(2_000_000)
    with pytest.raises(mabm.MabmError) as e:
        mabm.Sim(big, static_arena=True)
    assert e.value.code == mabm.E_NOMEM and "static arena" in str(e.value)
    small = W.c1(n_a=500, n_b=500, box_um=0.5)
    a = mabm.Sim(small, static_arena=True)
    with pytest.raises(mabm.MabmError) as e:
        mabm.Sim(small, static_arena=True)
    assert e.value.code == mabm.E_STATE
    a.step(3)
    a.close()
    # released: the arena can be taken again
    b = mabm.Sim(small, static_arena=True)
    b.step(2)
    assert b.counts()[1] == 2
    b.close()
