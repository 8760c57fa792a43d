"""GPU tests of the library's call contract: error codes, sticky device
errors forced from the host, timing and agent-update counters."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mabm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_14603_amd as m
    m.lib()
    return m


def test_add_after_step_is_state_error(mabm):
    s = mabm.Sim(W.c1(n_a=10, n_b=10, box_um=0.5))
    s.step(1)
    with pytest.raises(mabm.MabmError) as e:
        s._chk(mabm.lib().mabm_add_species(s._h, b"late", 1.0, 1, 0, None))
    assert e.value.code == mabm.E_STATE


def test_invalid_rules_and_sums(mabm):
    m = W.c1(n_a=10, n_b=10, box_um=0.5)
    m.rules = [W.bimol(0, 9, 2, -1, 0.01, 0.5)]
    with pytest.raises(mabm.MabmError) as e:
        mabm.Sim(m)
    assert e.value.code == mabm.E_INVALID
    m.rules = [W.unimol(0, -1, 0.7), W.unimol(0, 1, 0.7)]
    s = mabm.Sim(m)
    with pytest.raises(mabm.MabmError) as e:
        s.step(1)
    assert e.value.code == mabm.E_INVALID


def test_arena_too_small(mabm):
    import torch
    m = W.c1(n_a=10, n_b=10, box_um=0.5)
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(mabm.MabmError) as e:
        mabm.Sim(m, arena=small)
    assert e.value.code == mabm.E_NOMEM


def test_capacity_overflow_is_sticky(mabm):
    m = W.Model("cap", W.SPHERE, 1e-6, 0, [W.Species("G", 0.0, 10), W.Species("M", 1.0, 0)],
                [W.unimol(0, -1, 1.0, placement=W.EMIT, p2=1, release=0.005)],
                outer_radius_um=1.0, capacity=25)
    s = mabm.Sim(m)
    s.step(1)
    assert s.counts()[0].tolist() == [10, 10]
    s.step(1)
    with pytest.raises(mabm.MabmError) as e:
        s.counts()
    assert e.value.code == mabm.E_CAPACITY
    with pytest.raises(mabm.MabmError):
        s.step(1)


def test_five_thousand_births_in_one_step_are_placed(mabm):
    # every gene emits in the first step: 5,000 children ranked by parent id
    # over twenty sorted runs, ids next_id.. in parent order
    import oracle
    from parity import assert_same
    m = W.Model("burst", W.SPHERE, 1e-6, 0, [W.Species("G", 0.0, 5000), W.Species("M", 1.0, 0)],
                [W.unimol(0, -1, 1.0, placement=W.EMIT, p2=1, release=0.005)],
                outer_radius_um=1.0, capacity=20000)
    s = mabm.Sim(m, record=True)
    G, _ = s.grid()
    o = oracle.OracleSim(m, grid_n=G)
    for k in range(3):
        s.step(1)
        o.step(1)
        assert_same(s.export(), o.export(), f"burst t={k + 1}")
    assert s.counts()[0].tolist() == [5000, 15000]


def test_agent_updates_and_profile(mabm):
    m = W.c2(20_000, seed=1)
    s = mabm.Sim(m)
    s.profile(True)
    s.step(10)
    prof = s.profile_read()
    assert prof["move"][0] == 10 and prof["move"][1] > 0
    assert s.agent_updates() >= 10 * 19_000
    n, _ = s.size()
    assert n <= 20_000


def test_import_validation(mabm):
    m = W.c1(n_a=10, n_b=10, box_um=0.5)
    ids = np.arange(4, dtype=np.uint32)
    sp = np.zeros(4, np.uint8)
    x = np.full(4, 0.1, np.float32)
    cases = [
        (np.array([0, 1, 1, 3], np.uint32), sp, x, 10, "duplicate"),
        (ids, sp, x, 3, "next_id"),
        (ids, np.array([0, 0, 9, 0], np.uint8), x, 10, "species"),
        (ids, sp, np.array([0.1, 0.1, 0.6, 0.1], np.float32), 10, "outside"),
    ]
    for i, s_, xx, nid, what in cases:
        s = mabm.Sim(m)
        with pytest.raises(mabm.MabmError) as e:
            s.import_state(i, s_, xx, x, x, next_id=nid)
        assert e.value.code == mabm.E_INVALID, what
        s.close()
    s = mabm.Sim(m)
    s.import_state(ids, sp, x, x, x, next_id=10)
    assert s.size() == (4, 10)
