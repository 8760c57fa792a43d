"""Steps that keep the previous binning: between two binnings the agents
keep their slots and the neighbour search reads the last binning's cell
lists.  The library does so only within a bound under which every partner
is still found (contact radius plus the largest possible Brownian moves
since the binning within the stencil's reach), so every result stays bit
for bit the oracle's, which bins every step.  Checked here: the steps
between binnings the library picks against that bound restated, and
parity with the oracle across binning cycles for both stencils, the
periodic box, holes carried over kept steps, batches, graphs, the counts
ring, and a change of the limit in mid-run."""
import math

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


def expected_bin_every(m, G, cap=8):
    """The bound restated.  A step moves an agent at most 5.78 sigma along
    an axis, sigma of its species at the time; a claimer species' targets
    move at most dmax per step, the largest such bound over every species
    that is or can turn into a target of its rules.  Its reach after j kept
    steps, largest contact radius + j dmax, must stay within the 27-cell
    stencil's (a cell, less 1 %); where the grid allows the 8-cell stencil
    (half a cell), the binning is kept only while the claimer species that
    would need 27 cells hold at most an eighth of the initial claimers."""
    bim = [r for r in m.rules if r.kind == W.BIMOL]
    if not bim:
        return 1
    f32 = np.float32
    ns = len(m.species)
    sigma = [float(f32(math.sqrt(2.0 * float(f32(s.diffusion_um2_s)) * float(f32(m.dt_s)))))
             for s in m.species]
    becomes = np.eye(ns, dtype=bool)
    for r in m.rules:
        if r.products[0] >= 0:
            becomes[r.reactants[0], r.products[0]] = True
        if r.kind == W.BIMOL and r.products[1] >= 0:
            becomes[r.reactants[1], r.products[1]] = True
    for k in range(ns):
        becomes |= becomes[:, [k]] & becomes[[k], :]
    rmax, dmax = {}, {}
    for r in bim:
        a, t = r.reactants
        rmax[a] = max(rmax.get(a, 0.0), float(f32(r.radius_um)))
        d = max(float(f32(5.78 * sigma[k])) for k in range(ns) if becomes[k, t])
        dmax[a] = max(dmax.get(a, 0.0), d)
    ext = float(f32(m.box_um)) if m.geometry == W.PERIODIC_BOX else float(f32(f32(m.outer_radius_um) * f32(2)))
    h = float(f32(ext / G))
    stencil8 = ext / G >= 2.02 * max(rmax.values())
    k = cap
    for a in rmax:
        if dmax[a] > 0:
            k = min(k, 1 + max(0, math.floor((0.99 * h - rmax[a]) / dmax[a])))
    if stencil8:
        while k > 1:
            wide = sum(m.species[a].count for a in rmax if rmax[a] + (k - 1) * dmax[a] > 0.495 * h)
            if 8 * wide <= sum(m.species[a].count for a in rmax):
                break
            k -= 1
    return k


def slow_c2(n, seed):
    # every species at 0.5 um^2/s, so the 27-cell stencil keeps a binning too
    m = W.c2(n, seed=seed, steps=60)
    for s in m.species:
        s.diffusion_um2_s = 0.5
    m.name = "c2_slow"
    return m


def box_no_births(n, seed):
    # A + B -> C in the periodic box, C -> A by conversion (no births)
    m = W.c1(n_a=n // 2, n_b=n - n // 2, box_um=0.6, seed=seed)
    m.rules[1] = W.unimol(2, 0, 2e-2)
    m.name = "box_abc_conversion"
    return m


def holes_c2(n, seed):
    # degradation at 2 % per step: many holes kept across kept steps
    m = W.c2(n, seed=seed, steps=60)
    m.rules = W.c2_rules(deg_p=2e-2)
    m.name = "c2_holes"
    return m


# cells of 40 nm to 150 nm: 2 to 8 steps per binning; at 61 nm and 100 nm
# the kinase-1 claimers (whose inhibitor targets are fast) search 27 cells in
# the later kept steps, everyone else 8
CASES = [
    ("c2_cell40nm", lambda: W.c2(50_000, seed=30, steps=60), 0.04),
    ("c2_cell61nm", lambda: W.c2(50_000, seed=31, steps=60), 0.06),
    ("c2_cell100nm", lambda: W.c2(50_000, seed=32, steps=60), 0.10),
    ("c2_cell150nm", lambda: W.c2(50_000, seed=33, steps=60), 0.15),
    ("c2_27cell", lambda: slow_c2(40_000, 34), 0.019),
    ("box", lambda: box_no_births(6000, 35), 0.06),
    ("holes", lambda: holes_c2(40_000, 36), 0.10),
]


@pytest.mark.parametrize("graphs", [False, True])
@pytest.mark.parametrize("name,make,cell", CASES, ids=[c[0] for c in CASES])
def test_kept_binning_is_bit_exact(name, make, cell, graphs):
    import paper_2606_14603_amd as mabm
    m = make()
    g = mabm.Sim(m, record=True, cell_um=cell, graphs=graphs)
    G, _ = g.grid()
    k = g.get_param(mabm.PARAM_BIN_EVERY)
    say(f"[skin] {name} graphs={graphs} G={G} bin_every={k}")
    assert k == expected_bin_every(m, G) and k > 1
    o = oracle.OracleSim(m, grid_n=G)
    done = 0
    for c in (1, 2, 3, 5, 11, 24, 41):
        g.step(c - done)
        o.step(c - done)
        done = c
        assert_same(g.export(), o.export(), f"{name} t={c}")
        assert np.array_equal(g.counts()[0], o.counts()[0])


def test_live_agent_count_over_kept_steps():
    # agent-updates sum the live agents at every step's start; holes that
    # kept steps carry must not be counted
    import paper_2606_14603_amd as mabm
    m = holes_c2(30_000, 37)
    g = mabm.Sim(m, cell_um=0.15)
    assert g.get_param(mabm.PARAM_BIN_EVERY) >= 3
    o = oracle.OracleSim(m)
    want = 0
    for _ in range(30):
        want += int(o.counts()[0].sum())
        o.step(1)
    g.step(30)
    assert g.agent_updates() == want
    h = mabm.Sim(m, cell_um=0.15)
    h.set_param(mabm.PARAM_BIN_EVERY_MAX, 1)
    assert h.get_param(mabm.PARAM_BIN_EVERY) == 1
    h.step(30)
    assert h.agent_updates() == want
    assert_same(g.export(), h.export(), "kept binning vs every step")


def shuttle(n, seed, p_move=0.3):
    # carriers (A) cross the nuclear membrane at p_move per step each way,
    # so many cross twice within one kept binning; B binds A on contact in
    # both compartments, and the complex splits back (births)
    m = W.c3(n, seed=seed, n_genes=50)
    sp = [W.Species("A", 0.2, n // 2, W.CYTOPLASM), W.Species("B", 0.2, n - n // 2, W.CYTOPLASM),
          W.Species("AB", 0.1, 0, W.CYTOPLASM)]
    rules = [W.unimol(0, -1, p_move, placement=W.TRANSLOCATE, release=0.005,
                      from_comp=W.CYTOPLASM, to_comp=W.NUCLEUS),
             W.unimol(0, -1, p_move, placement=W.TRANSLOCATE, release=0.005,
                      from_comp=W.NUCLEUS, to_comp=W.CYTOPLASM),
             W.bimol(1, 0, 2, -1, 0.02, 0.7),
             W.unimol(2, 1, 0.05, placement=W.SPLIT, p2=0, release=0.005)]
    return m.with_(name="shuttle", species=sp, rules=rules, capacity=n + n // 2 + 4096)


PLACING = [
    ("c1_splits", lambda: W.c1(n_a=6000, n_b=6000, box_um=0.7, unbind_p=0.05), 0.07),
    ("c3_births_translocation", lambda: W.c3(20_000, seed=41, n_genes=400), 0.4),
    ("shuttle_placed_twice", lambda: shuttle(12_000, 42), 0.25),
]


@pytest.mark.parametrize("graphs", [False, True])
@pytest.mark.parametrize("name,make,cell", PLACING, ids=[c[0] for c in PLACING])
def test_kept_binning_with_placements_is_bit_exact(name, make, cell, graphs):
    # newborns, translocated agents and split parents join extra chains at
    # their new cells while a binning is kept; agents placed twice join the
    # global list; results stay the oracle's
    import paper_2606_14603_amd as mabm
    m = make()
    g = mabm.Sim(m, record=True, cell_um=cell, graphs=graphs)
    G, _ = g.grid()
    k = g.get_param(mabm.PARAM_BIN_EVERY)
    say(f"[skin] {name} graphs={graphs} G={G} bin_every={k}")
    assert k == expected_bin_every(m, G) and k > 1
    o = oracle.OracleSim(m, grid_n=G)
    done = 0
    for c in (1, 2, 3, 7, 16, 33):
        g.step(c - done)
        o.step(c - done)
        done = c
        assert_same(g.export(), o.export(), f"{name} t={c}")
    assert np.array_equal(g.counts()[0], o.counts()[0])
    assert g.size() == o.size()


def test_placing_batch_keeps_binning():
    import paper_2606_14603_amd as mabm
    from test_gpu_batch import run_batch
    models = [W.c3(n, seed=s, n_genes=gn) for n, s, gn in [(9000, 51, 150), (15_000, 52, 300)]]
    b = run_batch(models, [1, 4, 9, 30])
    assert b.get_param(mabm.PARAM_BIN_EVERY) > 1


def test_limit_changed_mid_run():
    import paper_2606_14603_amd as mabm
    m = W.c2(40_000, seed=38, steps=60)
    g = mabm.Sim(m, record=True, cell_um=0.15, graphs=True)
    G, _ = g.grid()
    o = oracle.OracleSim(m, grid_n=G)
    for n, lim in ((7, 0), (6, 1), (9, 3), (20, 0)):
        g.set_param(mabm.PARAM_BIN_EVERY_MAX, lim)
        g.step(n)
        o.step(n)
        assert_same(g.export(), o.export(), f"limit {lim}")
    with pytest.raises(mabm.MabmError):
        g.set_param(mabm.PARAM_BIN_EVERY_MAX, 9)


def test_batch_keeps_binning():
    import paper_2606_14603_amd as mabm
    from test_gpu_batch import run_batch
    models = []
    for k, (n, frac) in enumerate([(20_000, 1e-3), (45_000, 0.1), (8000, 4e-2)]):
        m = W.c2(n, seed=90 + k, steps=60, inhibitor_fraction=frac)
        m.name = f"c2_batch{k}"
        models.append(m)
    b = run_batch(models, [1, 4, 9, 33])
    assert b.get_param(mabm.PARAM_BIN_EVERY) > 1


def test_ring_over_kept_steps():
    import paper_2606_14603_amd as mabm
    m = holes_c2(20_000, 39)
    o = oracle.OracleSim(m)
    want = []
    for _ in range(12):
        o.step(3)
        want.append(o.counts()[0])
    g = mabm.Sim(m, cell_um=0.1, graphs=True)
    assert g.get_param(mabm.PARAM_BIN_EVERY) > 1
    g.record_counts(3, entries=32)
    g.step(17)
    g.step(19)
    steps, counts = g.ring()
    assert list(steps) == list(range(3, 37, 3))
    assert np.array_equal(counts[:, 0, :], np.array(want))


def test_cascade_default_grid_keeps_binning_four_steps():
    # the 2M-agent cascade on its default 128^3 grid: the kinase-1 claimers
    # need 27 cells from the second kept step on, so a binning lasts 4 steps
    import paper_2606_14603_amd as mabm
    m = W.c2(2_000_000)
    g = mabm.Sim(m)
    G, _ = g.grid()
    assert G == 128
    assert g.get_param(mabm.PARAM_BIN_EVERY) == expected_bin_every(m, G) == 4
