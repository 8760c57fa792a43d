"""Births at scale and the capacity edge, on the GPU against the oracle.

Children of a step are ranked by (simulation, parent id) over sorted runs
of 256 birth records; tens of thousands of children per step, in a single
simulation and in a batch, must get the oracle's ids, positions and slots'
contents bit for bit, with steps that keep the binning refilling the holes
that removals leave.  The capacity (the most live agents at a step's end)
must fail exactly where the oracle fails, whatever the binning interval
(holes are not live agents)."""
import numpy as np
import pytest

import oracle
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


def turnover_model(n_gene: int, n_eater: int, seed: int = 0, emit_p: float = 0.9,
                   decay_p: float = 0.8, capacity: int = 0, eat_p: float = 0.5) -> W.Model:
    """Expressors G emit M at emit_p per step; M decays at decay_p; eaters X
    consume M on contact (10 nm): many children, unimolecular removals and
    pair removals every step, in a sphere at the cascade's density."""
    g, m_, x = 0, 1, 2
    sp = [W.Species("G", 1.0, n_gene), W.Species("M", 1.0, 0), W.Species("X", 0.5, n_eater)]
    rules = [W.unimol(g, -1, emit_p, placement=W.EMIT, p2=m_, release=0.005),
             W.unimol(m_, -1, decay_p),
             W.bimol(x, m_, x, -1, 0.010, eat_p)]
    n_mean = n_gene + n_eater + n_gene * emit_p / max(decay_p, 1e-9)
    radius = (3 * n_mean / (4 * np.pi * 3820.0)) ** (1.0 / 3.0)
    return W.Model(f"turnover_{n_gene}_{seed}", W.SPHERE, 1e-6, seed, sp, rules,
                   outer_radius_um=float(radius),
                   capacity=capacity or int(2 * n_mean) + 4096)


@pytest.mark.parametrize("bin_max", [0, 1])
def test_twenty_thousand_births_per_step_single(bin_max):
    import paper_2606_14603_amd as mabm
    m = turnover_model(25_000, 20_000, seed=4)
    g = mabm.Sim(m, record=True)
    g.set_param(mabm.PARAM_BIN_EVERY_MAX, bin_max)
    G, _ = g.grid()
    say(f"[births] {m.name} bin_every={g.get_param(mabm.PARAM_BIN_EVERY)} grid={G}")
    if bin_max == 0:
        assert g.get_param(mabm.PARAM_BIN_EVERY) > 1  # kept steps refill holes
    o = oracle.OracleSim(m, grid_n=G)
    done = 0
    for c in (1, 2, 3, 6, 12, 25):
        g.step(c - done)
        o.step(c - done)
        done = c
        assert_same(g.export(), o.export(), f"{m.name} t={c}")
        gc, _ = g.counts()
        oc, _ = o.counts()
        assert np.array_equal(gc, oc)
    # the last steps each had more than 20,000 children
    e = o.export()
    assert int((e["event"] == 0).sum()) > 20_000


def test_batch_births_beyond_the_old_limit():
    # five simulations whose children together exceed 4,096 per step many
    # times over, ids per simulation
    import paper_2606_14603_amd as mabm
    models = [turnover_model(n, n // 2, seed=10 + k) for k, n in
              enumerate([9000, 3000, 12000, 500, 7000])]
    b = mabm.Batch(models, record=True)
    orcs = [oracle.OracleSim(m, grid_n=b.grid(k)[0]) for k, m in enumerate(models)]
    done = 0
    for c in (1, 4, 15):
        b.step(c - done)
        for o in orcs:
            o.step(c - done)
        done = c
        for k, (m, o) in enumerate(zip(models, orcs)):
            assert_same(b.export(k), o.export(), f"{m.name} (simulation {k}) t={c}")
            assert b.size(k)[1] == o.size()[1]
    births = sum(int((o.export()["event"] == 0).sum()) for o in orcs)
    assert births > 4 * 4096


def _oracle_history(m, steps):
    """Live agents after each step, and the first step whose end exceeds
    the capacity (None if none does)."""
    o = oracle.OracleSim(m)
    live = []
    for t in range(1, steps + 1):
        try:
            o.step(1)
        except oracle.OracleError as e:
            assert e.code == -4
            return live, t
        live.append(o.size()[0])
    return live, None


@pytest.mark.parametrize("bin_max", [0, 1])
def test_capacity_edge_fails_where_the_oracle_fails(bin_max):
    import paper_2606_14603_amd as mabm
    base = turnover_model(600, 400, seed=7, emit_p=0.6, decay_p=0.2, eat_p=0.9)
    steps = 40
    live, _ = _oracle_history(base.with_(capacity=100_000), steps)
    peak = max(live)
    # at exactly the peak nothing fails; one below it fails where the
    # oracle does (agents removed by pair rules near the edge are holes on
    # the GPU until a binning or a child takes their slot)
    for cap, fails in ((peak, False), (peak - 1, True)):
        m = base.with_(capacity=cap)
        _, t_fail = _oracle_history(m, steps)
        assert (t_fail is not None) == fails
        g = mabm.Sim(m, record=True)
        g.set_param(mabm.PARAM_BIN_EVERY_MAX, bin_max)
        G, _ = g.grid()
        every = g.get_param(mabm.PARAM_BIN_EVERY)
        o = oracle.OracleSim(m, grid_n=G)
        for t in range(1, steps + 1):
            g.step(1)
            if t == t_fail:
                with pytest.raises(mabm.MabmError) as e:
                    g.counts()
                assert e.value.code == mabm.E_CAPACITY
                break
            o.step(1)
            gc, _ = g.counts()
            assert gc.sum() == live[t - 1], (cap, t)
            if t % 10 == 0:
                assert_same(g.export(), o.export(), f"cap={cap} t={t}")
        say(f"[capacity] cap={cap} bin_every={every} fails_at={t_fail}")
