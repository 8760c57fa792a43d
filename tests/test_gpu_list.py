"""Both neighbour searches on the GPU, bit for bit against the oracle: the
claimer list (PARAM_PROPOSE_MODE = 2) and the chunked search (1) on the
kept-binning cases (both stencils, holes carried over kept steps, the
periodic box, agents placed in extra chains and the global list), crowded
stencils; the list with dense claimers (groups of 16 lanes, several passes
per workgroup), over 2,000 steps of the nuclear-signalling workload, under
graph replay; the mode switched in mid-run.  The automatic choice takes the
list for sparse claimers and small simulations and the chunked search for
large dense ones; a batch refuses the list."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import assert_same, say
from test_gpu_skin import CASES, PLACING, expected_bin_every

pytestmark = pytest.mark.gpu

LIST, CHUNKS = 2, 1


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_14603_amd as mabm
    mabm.lib()


def run_list(m, checkpoints, cell=None, graphs=False, mode=LIST, record=True):
    import paper_2606_14603_amd as mabm
    g = mabm.Sim(m, record=record, cell_um=cell, graphs=graphs)
    g.set_param(mabm.PARAM_PROPOSE_MODE, mode)
    assert g.get_param(mabm.PARAM_PROPOSE_MODE) == mode
    G, _ = g.grid()
    o = oracle.OracleSim(m, grid_n=G if record else 0)
    done = 0
    for c in checkpoints:
        g.step(c - done)
        o.step(c - done)
        done = c
        ge, oe = g.export(), o.export()
        if not record:
            for e in (ge, oe):
                for f in ("key", "event", "partner"):
                    e.pop(f, None)
        assert_same(ge, oe, f"{m.name} list t={c}")
        assert np.array_equal(g.counts()[0], o.counts()[0])
    return g


def test_automatic_mode():
    import paper_2606_14603_amd as mabm
    sparse = mabm.Sim(W.c3(20_000, seed=1))  # 4 genes claim among 20k agents
    assert sparse.get_param(mabm.PARAM_PROPOSE_MODE) == LIST
    small = mabm.Sim(W.c1(seed=1))           # 10k claimers: 16 lanes each in one pass
    assert small.get_param(mabm.PARAM_PROPOSE_MODE) == LIST
    small.close()
    dense = mabm.Sim(W.c2(600_000, seed=1))  # about 6 % claimers, 34.5k of them
    assert dense.get_param(mabm.PARAM_PROPOSE_MODE) == CHUNKS
    dense.set_param(mabm.PARAM_PROPOSE_MODE, LIST)
    assert dense.get_param(mabm.PARAM_PROPOSE_MODE) == LIST
    sparse.set_param(mabm.PARAM_PROPOSE_MODE, CHUNKS)
    assert sparse.get_param(mabm.PARAM_PROPOSE_MODE) == CHUNKS
    with pytest.raises(mabm.MabmError):
        sparse.set_param(mabm.PARAM_PROPOSE_MODE, 3)
    b = mabm.Batch([W.c3(9000, seed=2), W.c3(12_000, seed=3)])
    assert b.get_param(mabm.PARAM_PROPOSE_MODE) == CHUNKS
    with pytest.raises(mabm.MabmError):
        b.set_param(mabm.PARAM_PROPOSE_MODE, LIST)
    for s in (sparse, dense, b):
        s.close()


@pytest.mark.parametrize("mode", [LIST, CHUNKS])
@pytest.mark.parametrize("name,make,cell", CASES + PLACING, ids=[c[0] for c in CASES + PLACING])
def test_both_searches_over_kept_binnings(name, make, cell, mode):
    import paper_2606_14603_amd as mabm
    m = make()
    g = run_list(m, [1, 2, 3, 7, 16, 33], cell=cell, mode=mode)
    k = g.get_param(mabm.PARAM_BIN_EVERY)
    assert k == expected_bin_every(m, g.grid()[0]) and k > 1
    say(f"[search {mode}] {name} bin_every={k} ok")


@pytest.mark.parametrize("mode", [LIST, CHUNKS])
@pytest.mark.parametrize("bin_max", [0, 1])
def test_both_searches_in_crowded_cells(bin_max, mode):
    # cells far larger than the contact radius in a dense box: hundreds of
    # candidates per stencil (the list shares a cell among a group's lanes)
    import paper_2606_14603_amd as mabm
    m = W.c1(n_a=9000, n_b=9000, n_c=2000, box_um=0.9, seed=31, unbind_p=0.02)
    g = mabm.Sim(m, record=True, cell_um=0.15)
    g.set_param(mabm.PARAM_PROPOSE_MODE, mode)
    g.set_param(mabm.PARAM_BIN_EVERY_MAX, bin_max)
    o = oracle.OracleSim(m, grid_n=g.grid()[0])
    done = 0
    for c in (1, 2, 5, 12, 30):
        g.step(c - done)
        o.step(c - done)
        done = c
        assert_same(g.export(), o.export(), f"crowded list t={c}")


def test_dense_claimers_take_several_passes():
    # 40k claimers (half the agents): groups of 16 lanes, two passes of the
    # search's grid
    m = W.c1(n_a=40_000, n_b=40_000, box_um=0.7 * (80 / 12) ** (1 / 3), seed=44, unbind_p=0.05)
    run_list(m, [1, 2, 5, 20], cell=0.07)


def test_nuclear_signalling_long_run():
    # the crowded-membrane regime of the nuclear-signalling workload
    # (translocated carriers piling up near the membrane), 2,000 steps
    m = W.c3(20_000, seed=45, n_genes=60)
    run_list(m, [1, 10, 200, 1000, 2000], record=False)


def test_list_search_under_graph_replay():
    m = W.c3(20_000, seed=46, n_genes=100)
    run_list(m, [1, 5, 40, 120], graphs=True)


def test_mode_switched_mid_run():
    import paper_2606_14603_amd as mabm
    m = W.c2(30_000, seed=47, steps=60)
    g = mabm.Sim(m, record=True)
    o = oracle.OracleSim(m, grid_n=g.grid()[0])
    done = 0
    for c, mode in ((3, CHUNKS), (9, LIST), (14, CHUNKS), (25, LIST), (31, 0)):
        g.set_param(mabm.PARAM_PROPOSE_MODE, mode)
        g.step(c - done)
        o.step(c - done)
        done = c
        assert_same(g.export(), o.export(), f"mode {mode} t={c}")
