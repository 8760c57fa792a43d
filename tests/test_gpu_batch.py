"""GPU parity of batches: every simulation of a batch against the CPU oracle
run alone on the same model, bit for bit (positions, species, ids, cell ids
at that simulation's grid, events, partners), and the batch's
per-simulation counts against the oracle's.

The batches mix sizes (so grids differ: 16^3 to 64^3 cells), seeds and
initial counts (doses), and include an empty simulation; the C3-like batch
has births (ids per simulation, slots ranked by simulation then parent) and
membrane crossings.
"""
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
    mabm.lib()  # raises if the HIP library is not built


def run_batch(models, checkpoints, record=True):
    import paper_2606_14603_amd as mabm
    say(f"[batch] {len(models)} x {models[0].name}, sizes "
        f"{[m.n_agents for m in models]}, checkpoints {checkpoints}")
    b = mabm.Batch(models, record=record)
    orcs = []
    for k, m in enumerate(models):
        G, _ = b.grid(k)
        orcs.append(oracle.OracleSim(m, grid_n=G if record else 0))
    done = 0
    for c in checkpoints:
        b.step(c - done)
        for o in orcs:
            o.step(c - done)
        done = c
        counts, t = b.counts()
        assert t == c
        digests = b.digest()
        for k, (m, o) in enumerate(zip(models, orcs)):
            ge, oe = b.export(k), o.export()
            # the library's per-simulation state digest is that of the
            # oracle's state
            assert int(digests[k]) == state_digest(oe), (k, c)
            if not record:
                for f in ("key", "event", "partner"):
                    ge.pop(f)
                    oe.pop(f)
            assert_same(ge, oe, f"{m.name} (simulation {k}) t={c}")
            oc, ot = o.counts()
            assert ot == c
            assert np.array_equal(counts[k], oc), (k, counts[k], oc)
            n_live, next_id = b.size(k)
            assert n_live == len(oe["id"])
            assert next_id == o.size()[1]
    say(f"[batch] ok, live={b.counts()[0].sum(axis=1).tolist()}")
    return b


def test_c2_dose_replicate_batch():
    # doses and replicates of the C2 cascade, sizes on both sides of the
    # 32^3 / 64^3 grid switch
    models = []
    for k, (n, frac) in enumerate([(6000, 4e-4), (40_000, 4e-3), (3000, 4e-2), (25_000, 0.43),
                                   (9000, 0.1), (50_000, 1e-3)]):
        m = W.c2(n, seed=64 * k + 3, steps=60, inhibitor_fraction=frac)
        m.name = f"c2_dose{k}"
        models.append(m)
    run_batch(models, [1, 2, 10, 60])


def test_c3_batch_births_and_translocation():
    models = [W.c3(n, seed=s, n_genes=g) for n, s, g in
              [(8000, 12, 120), (20_000, 42, 300), (5000, 314, 90)]]
    run_batch(models, [1, 5, 40, 150])


def test_box_batch_with_an_empty_simulation_and_no_recording():
    models = [W.c1(n_a=a, n_b=b, box_um=L, unbind_p=2e-2) for a, b, L in
              [(800, 700, 0.4), (0, 0, 0.3), (3000, 3000, 0.6), (1, 0, 0.2)]]
    for k, m in enumerate(models):
        m.seed = 100 + k
    run_batch(models, [1, 3, 30], record=False)
    run_batch(models, [2, 25], record=True)


def test_batch_of_one_equals_a_single_simulation():
    import paper_2606_14603_amd as mabm
    m = W.c2(30_000, seed=5, steps=30)
    b = mabm.Batch([m], record=True)
    g = mabm.Sim(m, record=True)
    b.step(30)
    g.step(30)
    assert_same(b.export(0), g.export(), "batch of one vs single")
    assert np.array_equal(b.counts()[0][0], g.counts()[0])


def test_batch_agent_updates_and_errors():
    import paper_2606_14603_amd as mabm
    models = [W.c2(4000, seed=1), W.c2(7000, seed=2)]
    b = mabm.Batch(models)
    b.step(5)
    u = b.agent_updates()
    counts, _ = b.counts()
    assert 5 * sum(m.n_agents for m in models) >= u >= 5 * int(counts.sum()) - 100
    with pytest.raises(mabm.MabmError):
        b.size(2)
    with pytest.raises(mabm.MabmError):
        b.import_state([0], [0], [0.0], [0.0], [0.0], 1)
    bad = W.c1(n_a=10, n_b=10)
    with pytest.raises(mabm.MabmError):
        mabm.Batch([models[0], bad])


def test_many_tiny_simulations_share_waves():
    # 40 simulations of 1-120 agents: most waves hold agents of several
    # simulations, so the per-wave simulation resolution takes many passes;
    # the split rule makes births of many simulations in one step
    rng = np.random.default_rng(8)
    models = []
    for k in range(40):
        n = int(rng.integers(1, 121))
        m = W.c1(n_a=(n + 1) // 2, n_b=n // 2, box_um=0.08 + 0.002 * k, unbind_p=0.05)
        m.seed = 1000 + k
        models.append(m)
    run_batch(models, [1, 2, 5, 20, 60])


def test_batch_tuner_choice_changes_no_result():
    # the batch tuner's cell density and launch shape: the tuned batch's
    # states equal the default batch's bit for bit
    import paper_2606_14603_amd as mabm
    from paper_2606_14603_amd import tune
    models = [W.c2(n, seed=70 + k, steps=12) for k, n in enumerate((20_000, 45_000, 8_000))]
    for k, m in enumerate(models):
        m.name = f"c2_tuned{k}"
    tr = tune.tune_batch(models, steps=4, warm=2)
    say(f"[batch] tuned: {tr.agents_per_cell} agents per cell, lanes {tr.lanes}, "
        f"workgroups {tr.min_workgroups}")
    a = mabm.Batch(tr.models(models), record=True)
    tr.apply(a)
    b = mabm.Batch(models, record=True)
    a.step(12)
    b.step(12)
    for k in range(len(models)):
        ea, eb = a.export(k), b.export(k)
        for f in ("id", "species", "x", "y", "z", "event", "partner"):
            x, y = ea[f], eb[f]
            if x.dtype == np.float32:
                x, y = x.view(np.uint32), y.view(np.uint32)
            assert np.array_equal(x, y), (k, f)
