"""GPU parity: the HIP library against the CPU oracle, bit for bit.

Positions (float32 bits), species, ids, cell ids at the library's grid,
unimolecular events and confirmed partners are compared for every live
agent, id-keyed, at several checkpoints; species counts and the step
counter are compared too.  Sizes: the C1 workload at full size and horizon,
scaled C2/C3 models that the oracle finishes in seconds while spanning many
cells and a ragged tail (the scaled C3 to 2,000 steps, where translocated
agents crowd the nuclear membrane and births have refilled many holes), and
the full 2M-agent C2 and 5M-agent C3 for 20 steps in the launch
configuration the benchmark times, then again recording cell ids, events
and partners for the comparison at step 20.  The small cases run with the
neighbour search the library chooses (the claimer list, at their sizes)
and with the chunked one.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import assert_same, run_pair, say

from paper_2606_14603_amd import PARAM_PROPOSE_MODE as PARAM_MODE

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_14603_amd as mabm
    mabm.lib()  # raises if the HIP library is not built


# the neighbour search as the library chooses (the claimer list at these
# sizes) and forced to the chunked search
SEARCH = pytest.mark.parametrize("mode", [0, 1], ids=["auto", "chunks"])


@SEARCH
def test_c1_small_every_step(mode):
    m = W.c1(n_a=1500, n_b=1500, box_um=2.0 * (3000 / 20000) ** (1 / 3), unbind_p=2e-2)
    run_pair(m, list(range(1, 31)) + [60, 120], params={PARAM_MODE: mode})


def test_c1_full_size_full_horizon():
    run_pair(W.c1(), [1, 2, 10, 100, 250, 500, 1000])


@SEARCH
def test_c2_scaled(mode):
    run_pair(W.c2(20_000, seed=42, steps=200), [1, 5, 50, 200], params={PARAM_MODE: mode})


@SEARCH
def test_c3_scaled_births_and_translocation(mode):
    m = W.c3(20_000, seed=12, n_genes=300)
    run_pair(m, [1, 10, 100, 300, 800, 2000], params={PARAM_MODE: mode})


def test_c1_parity_grid_of_17_cells():
    # the reversible-binding workload on a 17-cell grid (2/17 um cells, a
    # Morton grid padded to 32 per axis) for its whole horizon
    run_pair(W.c1(), [1, 100, 1000], cell_um=2.0 / 17 * (1 + 1e-6))


def test_c2_scaled_full_horizon():
    # the cascade scaled to 20k agents for the workload's 5,000 steps
    run_pair(W.c2(20_000, seed=43), [1, 1000, 5000])


def test_c3_scaled_full_horizon():
    # the nuclear-signalling model scaled to 20k agents for the workload's
    # 10,000 steps (the crowded-membrane regime, births refilling holes)
    run_pair(W.c3(20_000, seed=13, n_genes=12), [1, 2000, 10_000], record=False)


def test_c2_full_size_in_bench_configuration():
    # the benchmark's configuration: 2M agents, no recording, library-chosen grid
    run_pair(W.c2(), [1, 3, 20], record=False)
    run_pair(W.c2(), [20], record=True)


def test_c3_full_size_twenty_steps():
    # 5M agents in nested compartments with births, at full size
    run_pair(W.c3(), [1, 20], record=False)
    run_pair(W.c3(), [20], record=True)


@SEARCH
def test_ragged_and_tiny_sizes(mode):
    for n in (1, 2, 3, 255, 256, 257, 1023, 4097):
        m = W.c1(n_a=(n + 1) // 2, n_b=n // 2, box_um=0.2, unbind_p=0.05)
        run_pair(m, [1, 7], params={PARAM_MODE: mode})


@SEARCH
def test_empty_simulation(mode):
    m = W.c1(n_a=0, n_b=0, box_um=1.0)
    run_pair(m, [1, 3], params={PARAM_MODE: mode})


def test_cell_size_does_not_change_results():
    import paper_2606_14603_amd as mabm
    m = W.c2(20_000, seed=7)
    outs = []
    for cell in (0.0, 0.05, 0.19):
        g = mabm.Sim(m, record=True, cell_um=cell)
        say(f"[cell] cell_um={cell} grid={g.grid()}")
        g.step(40)
        e = g.export()
        e.pop("key")
        outs.append(e)
    for e in outs[1:]:
        for k in e:
            assert np.array_equal(e[k].view(np.uint32) if e[k].dtype == np.float32 else e[k],
                                  outs[0][k].view(np.uint32) if e[k].dtype == np.float32
                                  else outs[0][k]), k


def test_two_runs_bit_identical_and_record_flag_neutral():
    import paper_2606_14603_amd as mabm
    m = W.c3(20_000, seed=101010, n_genes=200)
    res = []
    for rec in (True, True, False):
        g = mabm.Sim(m, record=rec)
        g.step(120)
        e = g.export()
        for f in ("key", "event", "partner"):
            e.pop(f)
        res.append(e)
    for e in res[1:]:
        for k in e:
            a, b = e[k], res[0][k]
            if a.dtype == np.float32:
                a, b = a.view(np.uint32), b.view(np.uint32)
            assert np.array_equal(a, b), k


def _import_pair(agents, next_id, t=0):
    def imp(sim):
        sim.import_state([a[0] for a in agents], [a[1] for a in agents],
                         [a[2] for a in agents], [a[3] for a in agents],
                         [a[4] for a in agents], next_id, t)
    imp.t0 = t
    return imp


@SEARCH
def test_engineered_contacts_match_oracle(mode):
    R = 2.0 ** -7
    A, B, C = 0, 1, 2
    m = W.Model("claims", W.PERIODIC_BOX, 1e-6, 0,
                [W.Species("A", 0.0, 0), W.Species("B", 0.0, 0), W.Species("C", 0.0, 0)],
                [W.bimol(A, B, C, -1, R, 1.0)], box_um=1.0, capacity=64)
    h = 0.5
    agents = [(10, A, h, h, h), (3, B, h, h - R, h), (5, B, h + R, h, h),
              (11, A, 0.25, 0.25, 0.25), (20, B, 0.25 + R + 2.0 ** -10, 0.25, 0.25),
              (12, A, 2.0 ** -10, 0.75, 0.75), (21, B, 1.0 - 2.0 ** -8, 0.75, 0.75),
              (30, B, h, 0.25, 0.75), (31, A, h - 2.0 ** -8, 0.25, 0.75),
              (32, A, h + 2.0 ** -8, 0.25, 0.75),
              (33, B, h + 2.0 ** -8 + 2.0 ** -8 + 2.0 ** -9, 0.25, 0.75)]
    run_pair(m, [1, 2], importer=_import_pair(agents, 64), params={PARAM_MODE: mode})
    sp = [W.Species(n, 0.0, 0) for n in ("A", "P", "D", "X", "E", "S", "Q")]
    rules = [W.bimol(0, 0, 1, 2, R, 1.0), W.bimol(0, 3, 1, 3, R, 1.0), W.unimol(3, 3, 1.0),
             W.bimol(4, 5, 4, 6, R, 1.0)]
    m2 = W.Model("homo", W.PERIODIC_BOX, 1e-6, 7, sp, rules, box_um=1.0, capacity=64)
    agents2 = [(9, 0, 0.5, 0.5, 0.5), (4, 0, 0.5 + 2.0 ** -8, 0.5, 0.5),
               (6, 0, 0.25, 0.25, 0.25), (7, 3, 0.25 + 2.0 ** -8, 0.25, 0.25),
               (1, 4, 0.75, 0.75, 0.75), (2, 5, 0.75, 0.75 + 2.0 ** -8, 0.75)]
    run_pair(m2, [1], importer=_import_pair(agents2, 16, t=9), params={PARAM_MODE: mode})


@SEARCH
def test_dense_random_contacts_match_oracle(mode):
    rng = np.random.default_rng(3)
    n, L = 3000, 0.25
    m = W.Model("dense", W.PERIODIC_BOX, 1e-6, 11,
                [W.Species("A", 0.5, 0), W.Species("B", 0.5, 0), W.Species("C", 0.2, 0),
                 W.Species("D", 0.2, 0)],
                [W.bimol(0, 1, 2, 3, 0.02, 0.7), W.bimol(0, 0, 2, 2, 0.015, 0.5),
                 W.unimol(2, 0, 0.05, placement=W.SPLIT, p2=1, release=0.01),
                 W.unimol(3, 1, 0.05)],
                box_um=L, capacity=2 * n)
    pos = rng.uniform(0, L, (n, 3)).astype(np.float32)
    agents = [(int(i), int(s), float(p[0]), float(p[1]), float(p[2]))
              for i, s, p in zip(rng.permutation(5 * n)[:n], rng.integers(0, 2, n), pos)]
    run_pair(m, [1, 2, 5, 20], importer=_import_pair(agents, 5 * n, t=3), params={PARAM_MODE: mode})


@SEARCH
def test_nested_dense_membrane_contacts(mode):
    rng = np.random.default_rng(4)
    n = 4000
    m = W.Model("memb", W.NESTED_SPHERES, 1e-6, 5,
                [W.Species("A", 1.0, 0), W.Species("B", 1.0, 0), W.Species("C", 0.5, 0)],
                [W.bimol(0, 1, 2, -1, 0.02, 0.8),
                 W.unimol(2, 0, 0.02, placement=W.SPLIT, p2=1, release=0.01),
                 W.unimol(0, -1, 0.01, placement=W.TRANSLOCATE, release=0.005, from_comp=0,
                          to_comp=1),
                 W.unimol(1, -1, 0.01, placement=W.TRANSLOCATE, release=0.005, from_comp=1,
                          to_comp=0)],
                outer_radius_um=0.5, inner_radius_um=0.3, capacity=2 * n)
    # a shell of agents hugging the membrane on both sides
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = 0.3 + rng.uniform(-0.02, 0.02, n)
    p = (d * r[:, None]).astype(np.float32)
    agents = [(i, int(s), float(q[0]), float(q[1]), float(q[2]))
              for i, (s, q) in enumerate(zip(rng.integers(0, 2, n), p))]
    run_pair(m, [1, 2, 10, 40], importer=_import_pair(agents, n), params={PARAM_MODE: mode})


def test_graph_replay_matches_direct_launches():
    # Steps replayed from captured graphs (single steps and 16-step graphs of
    # both starting parities) against direct launches, checked after every
    # run of steps, with eager queries between the replays.
    import paper_2606_14603_amd as mabm
    for m in (W.c3(20_000, seed=42, n_genes=300), W.c2(30_000, seed=9)):
        g = mabm.Sim(m, record=True, graphs=True)
        e = mabm.Sim(m, record=True, graphs=False)
        done = 0
        for n in (37, 1, 16, 50, 3, 33):
            g.step(n)
            e.step(n)
            done += n
            assert_same(g.export(), e.export(), f"{m.name} graphs t={done}")
            assert np.array_equal(g.counts()[0], e.counts()[0])
            assert g.agent_updates() == e.agent_updates()
        say(f"[graphs] {m.name} ok at t={done}")


def test_dense_box_overflows_the_workgroup_proposal_stage():
    # 8,000 agents in a 0.2 um box with binding certain on contact: in the
    # first step 2,259 of the 4,000 claimers bind.  With one workgroup per
    # chunk of 1,024 agents, most of a chunk's ~500 claimers propose, more
    # than the 256 proposals a workgroup stages in LDS, so the rest reserve
    # their list entries one by one; results stay the oracle's
    import paper_2606_14603_amd as mabm
    m = W.c1(n_a=4000, n_b=4000, box_um=0.2, bind_p=1.0, unbind_p=0.02)
    m.seed = 77
    g = mabm.Sim(m, record=True)
    g.set_param(mabm.PARAM_PROPOSE_MODE, 1)  # the chunked search, one workgroup per chunk
    g.set_param(mabm.PARAM_PROPOSE_MIN_WORKGROUPS, 1)
    G, _ = g.grid()
    o = oracle.OracleSim(m, grid_n=G)
    done = 0
    for c in (1, 2, 5, 12):
        g.step(c - done)
        o.step(c - done)
        done = c
        assert_same(g.export(), o.export(), f"dense box t={c}")
    assert o.counts()[0][2] > 2000


def largest_tables(seed=7):
    """64 species and 255 rules, the library's table limits: 180 pair rules
    over distinct unordered species pairs (a few homotypic, some consuming
    the target), and 75 unimolecular conversions and degradations, eight on
    each of the first nine species (the most one species takes), in a
    sphere at the cascade's density."""
    rng = np.random.default_rng(seed)
    ns = 64
    sp = [W.Species(f"s{k}", float(rng.uniform(0.2, 3.0)), 300) for k in range(ns)]
    pairs = set()
    rules = []
    while len(rules) < 180:
        a, b = (int(v) for v in rng.integers(0, ns, 2))
        if len(pairs) < 6:
            b = a
        key = (min(a, b), max(a, b))
        if key in pairs:
            continue
        pairs.add(key)
        p1 = int(rng.integers(0, ns))
        p2 = -1 if rng.random() < 0.3 else int(rng.integers(0, ns))
        rules.append(W.bimol(a, b, p1, p2, float(rng.uniform(0.005, 0.015)),
                             float(rng.uniform(0.3, 1.0))))
    for k in range(75):
        a = k // 8 if k < 72 else 9
        p1 = -1 if k % 5 == 0 else int(rng.integers(0, ns))
        rules.append(W.unimol(a, p1, 0.01))
    n = 300 * ns
    radius = (n / 2000.0 * 3.0 / (4.0 * np.pi)) ** (1.0 / 3.0)
    return W.Model("largest_tables", W.SPHERE, 1e-6, seed, sp, rules,
                   outer_radius_um=float(radius), capacity=n + 256, steps=40)


def test_largest_tables_match_oracle():
    m = largest_tables()
    assert len(m.species) == 64 and len(m.rules) == 255
    run_pair(m, [1, 2, 5, 20, 40])


@pytest.mark.parametrize("radius_um,grid", [(2.7, 512), (5.4, 1024)])
def test_largest_grids_match_oracle(radius_um, grid):
    # 512 cells per axis (27-bit Morton keys, scan tiles of 2^6 passes: 134M
    # cells in at most 1,024 tiles) and 1,024, the library's largest grid
    # (30-bit keys, tiles of 2^9 passes: 2^30 cells, 12.9 GB of cell tables)
    # (20k cascade agents in a sphere: 10.5 nm cells, just above the largest
    # contact radius)
    import paper_2606_14603_amd as mabm
    m = W.c2(20_000, seed=8, steps=6).with_(outer_radius_um=radius_um)
    g = mabm.Sim(m, record=True, cell_um=0.01054)
    assert g.grid()[0] == grid == min(grid, mabm.MAX_GRID)
    g.close()
    run_pair(m, [1, 3, 6], cell_um=0.01054)


def test_beyond_2_28_slots_matches_oracle():
    # 272M nuclear-signalling agents, more than 2^28, so the records in use
    # reach past 4 GiB and agent-indexed byte addresses need more than 32
    # bits, on the 1,023-cell grid; two steps with translocations and
    # births; the state digest and counts against the oracle's (comparing
    # the full export would take minutes)
    import torch
    import paper_2606_14603_amd as mabm
    from parity import state_digest
    m = W.c3(272_000_000)
    g = mabm.Sim(m, cell_um=2 * m.outer_radius_um / 1024 * (1 + 1e-6))
    g.step(2)
    gd, (gc, gt) = int(g.digest()[0]), g.counts()
    say(f"[big] {m.n_agents} agents, grid {g.grid()[0]}, gpu digest {gd:#x}")
    g.close()
    del g
    torch.cuda.empty_cache()
    oracle.threads(16)
    o = oracle.OracleSim(m)
    o.step(1)
    say("[big] oracle step 1")
    o.step(1)
    oc, ot = o.counts()
    e = o.export()
    o.close()
    od, n = 0, len(e["id"])
    for a in range(0, n, 20_000_000):
        od = (od + state_digest({k: v[a:a + 20_000_000] for k, v in e.items()})) % (1 << 64)
    assert gt == ot == 2 and np.array_equal(gc, oc)
    assert gd == od, (hex(gd), hex(od))


@pytest.mark.parametrize("bin_max", [0, 1])
def test_crowded_stencils_searched_by_whole_waves(bin_max):
    # cells far larger than the contact radius in a dense box: every
    # claimer's stencil lists hundreds of candidates, so the search deals
    # them over a whole wave; with and without kept binnings (splits place
    # agents in extra chains), against the oracle
    import paper_2606_14603_amd as mabm
    m = W.c1(n_a=9000, n_b=9000, n_c=2000, box_um=0.9, seed=31, unbind_p=0.02)
    g = mabm.Sim(m, record=True, cell_um=0.15)
    g.set_param(mabm.PARAM_BIN_EVERY_MAX, bin_max)
    G, _ = g.grid()
    say(f"[crowded] {m.n_agents} agents, grid {G}, {m.n_agents / G ** 3:.0f} per cell, "
        f"bin_every {g.get_param(mabm.PARAM_BIN_EVERY)}")
    o = oracle.OracleSim(m, grid_n=G)
    done = 0
    for c in (1, 2, 5, 12, 30):
        g.step(c - done)
        o.step(c - done)
        done = c
        assert_same(g.export(), o.export(), f"crowded t={c}")


def test_crowded_stencils_in_a_batch():
    import paper_2606_14603_amd as mabm
    models = [W.c1(n_a=n, n_b=n, n_c=n // 5, box_um=0.9 * (n / 9000) ** (1 / 3), seed=40 + k,
                   unbind_p=0.02).with_(cell_um=0.15 * (n / 9000) ** (1 / 3), name=f"crowd{k}")
              for k, n in enumerate([9000, 3000, 6000])]
    b = mabm.Batch(models, record=True)
    orcs = [oracle.OracleSim(m, grid_n=b.grid(k)[0]) for k, m in enumerate(models)]
    done = 0
    for c in (1, 6, 20):
        b.step(c - done)
        for o in orcs:
            o.step(c - done)
        done = c
        for k, o in enumerate(orcs):
            assert_same(b.export(k), o.export(), f"{models[k].name} t={c}")


def test_crowded_wide_stencils_in_kept_steps():
    # a contact radius above half the cell size forces the 27-cell stencil
    # on every claimer, and a dense box makes every stencil crowded, so
    # claimers are searched over 27 cells by a whole wave, in binning and
    # kept steps
    import paper_2606_14603_amd as mabm
    m = W.c1(n_a=9000, n_b=9000, n_c=2000, box_um=0.9, seed=33, unbind_p=0.02,
             radius_um=0.08, release_um=0.04)
    g = mabm.Sim(m, record=True, cell_um=0.13)  # 6 cells of 150 nm < 2.02 x 80 nm
    G, _ = g.grid()
    every = g.get_param(mabm.PARAM_BIN_EVERY)
    say(f"[crowded wide] grid {G}, bin_every {every}")
    assert G == 6 and every >= 3
    o = oracle.OracleSim(m, grid_n=G)
    done = 0
    for c in (1, 3, 7, 16):
        g.step(c - done)
        o.step(c - done)
        done = c
        assert_same(g.export(), o.export(), f"crowded wide t={c}")
