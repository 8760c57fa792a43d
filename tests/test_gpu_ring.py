"""Counts over time from the device counts ring: every entry equals the
oracle's counts at that step (graph replay and direct launches, ring
wrap-around, batches), and a model loaded from a model file runs bit for
bit like the oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import assert_same, run_pair, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_14603_amd as mabm
    mabm.lib()


def _oracle_series(m, every, total):
    o = oracle.OracleSim(m)
    out = []
    for t in range(every, total + 1, every):
        o.step(every)
        c, tt = o.counts()
        assert tt == t
        out.append(c)
    return np.array(out)


@pytest.mark.parametrize("graphs", [True, False])
def test_ring_matches_oracle_counts(graphs):
    import paper_2606_14603_amd as mabm
    m = W.c3(12_000, seed=12, n_genes=200)
    want = _oracle_series(m, 7, 140)
    g = mabm.Sim(m, graphs=graphs)
    g.record_counts(7, entries=64)
    for n in (37, 1, 62, 40):
        g.step(n)
    steps, counts = g.ring()
    assert list(steps) == list(range(7, 141, 7))
    assert np.array_equal(counts[:, 0, :], want)
    # a ring of 4 keeps the newest 4 entries
    h = mabm.Sim(m, graphs=graphs)
    h.record_counts(7, entries=4)
    h.step(140)
    steps, counts = h.ring()
    assert list(steps) == [119, 126, 133, 140]
    assert np.array_equal(counts[:, 0, :], want[-4:])
    say(f"[ring] graphs={graphs} ok")


def test_ring_of_a_batch():
    import paper_2606_14603_amd as mabm
    models = [W.c2(5000, seed=1), W.c2(9000, seed=2, inhibitor_fraction=0.1)]
    b = mabm.Batch(models)
    b.record_counts(10, entries=8)
    b.step(50)
    steps, counts = b.ring()
    assert list(steps) == [10, 20, 30, 40, 50]
    for k, m in enumerate(models):
        assert np.array_equal(counts[:, k, :], _oracle_series(m, 10, 50))


def test_model_file_runs_like_the_oracle():
    from paper_2606_14603_amd import model_io
    doc = {"name": "file", "geometry": {"kind": "nested", "radius_um": 1.0, "inner_radius_um": 0.5},
           "dt_s": 1e-6, "seed": 4, "steps": 30,
           "species": [{"name": "K", "mw_kda": 60.0, "concentration_M": 4e-6},
                       {"name": "S", "mw_kda": 40.0, "concentration_M": 2e-5,
                        "compartment": "nucleus"},
                       {"name": "pS", "mw_kda": 40.0, "count": 0, "compartment": "nucleus"}],
           "reactions": [{"reactants": ["K", "S"], "products": ["K", "pS"], "radius_nm": 12,
                          "probability": 0.5},
                         {"reactants": ["K"], "products": ["K"], "placement": "translocate",
                          "from": "cytosol", "to": "nucleus", "release_nm": 5,
                          "probability": 0.01},
                         {"reactants": ["K"], "products": ["K"], "placement": "translocate",
                          "from": "nucleus", "to": "cytosol", "release_nm": 5,
                          "probability": 0.01},
                         {"reactants": ["pS"], "products": ["S"], "kcat_per_s": 500.0}]}
    m = model_io.load_model(doc)
    run_pair(m, [1, 10, 30])


def test_tuner_picks_a_candidate_and_caches_it(tmp_path):
    from paper_2606_14603_amd import tune
    m = W.c2(60_000, seed=3)
    r = tune.tune_cell(m, steps=5, warm=2, cache_path=str(tmp_path / "cells.json"))
    assert r.cell_um in r.ms_per_step and len(r.ms_per_step) == len(tune.candidates(m))
    assert (r.lanes, r.min_workgroups) in r.ms_per_shape
    assert set(r.ms_per_shape) == set(tune.shapes(r.cell_um, m))
    assert set(r.ms_per_mode) == {1, 2} and r.mode == min(r.ms_per_mode, key=r.ms_per_mode.get)
    c = tune.tune_cell(W.c2(60_000, seed=4))
    assert c.cached and (c.cell_um, c.lanes, c.min_workgroups, c.mode) == (
        r.cell_um, r.lanes, r.min_workgroups, r.mode)
    say(f"[tune] {m.name}: {r.cell_um:.4f} um from {r.ms_per_step}, "
        f"shape {r.lanes, r.min_workgroups} from {r.ms_per_shape}")


@pytest.mark.parametrize("which", ["c2_27cell", "c2_8cell", "c3", "box"])
def test_launch_shape_leaves_results_unchanged(which):
    # lanes per claimer and the propose split change only how the search is
    # spread over lanes and workgroups: exports stay bit-identical to the
    # oracle's, also when the shape changes between graph-replayed steps
    import paper_2606_14603_amd as mabm
    if which.startswith("c2"):
        m = W.c2(50_000, seed=21, steps=40)
        rmax = max(r.radius_um for r in m.rules if r.kind == W.BIMOL)
        cell = 1.5 * rmax if which == "c2_27cell" else 2.05 * rmax
    elif which == "c3":
        m, cell = W.c3(15_000, seed=22, n_genes=200), None
    else:
        m, cell = W.c1(n_a=3000, n_b=2500, box_um=0.5, unbind_p=2e-2), None
    shapes = [(32, 0), (4, 1 << 16), (8, 1), (16, 512), (0, 0)]
    g = mabm.Sim(m, record=True, cell_um=cell, graphs=True)
    g.set_param(mabm.PARAM_PROPOSE_MODE, 1)  # the chunked search, which the shape steers
    G, _ = g.grid()
    o = oracle.OracleSim(m, grid_n=G)
    for k, (lanes, minwg) in enumerate(shapes):
        g.set_param(mabm.PARAM_PROPOSE_LANES, lanes)
        g.set_param(mabm.PARAM_PROPOSE_MIN_WORKGROUPS, minwg)
        g.step(8 + k)
        o.step(8 + k)
        assert_same(g.export(), o.export(), f"{m.name} shape {lanes, minwg}")
    with pytest.raises(mabm.MabmError):
        g.set_param(mabm.PARAM_PROPOSE_LANES, 3)
    with pytest.raises(mabm.MabmError):
        g.set_param(mabm.PARAM_PROPOSE_MIN_WORKGROUPS, (1 << 20) + 1)
    with pytest.raises(mabm.MabmError):
        g.set_param(99, 0)
    say(f"[shape] {which} G={G} ok")
