"""Randomised models against the oracle: geometry, species (some that never
move), pair rules (homotypic ones, products that are consumed, contact
probabilities of 0 and 1) and unimolecular rules of every placement
(conversions, degradations, splits and emissions with release radii large
enough that many placements are rejected near walls and membranes,
translocations both ways), dense enough that claims conflict.  The GPU must
match the oracle bit for bit on every one, with the cell lists kept between
binnings as the library chooses and with binning every step, and with the
neighbour search per chunk and over the claimer list."""
import numpy as np
import pytest

import workloads as W
from parity import run_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_14603_amd as mabm
    mabm.lib()


def random_model(seed: int, ns: int = 0, bimol_tries: int = 0, unimol_tries: int = 0) -> W.Model:
    rng = np.random.default_rng(seed)
    geometry = [W.PERIODIC_BOX, W.SPHERE, W.NESTED_SPHERES][seed % 3]
    ncomp = 2 if geometry == W.NESTED_SPHERES else 1
    ns = ns or int(rng.integers(3, 13))
    n = int(rng.integers(1500, 4000))
    counts = rng.multinomial(n, rng.dirichlet(np.ones(ns)))
    species = []
    for k in range(ns):
        d = 0.0 if rng.random() < 0.2 else float(rng.uniform(0.1, 5.0))
        species.append(W.Species(f"s{k}", d, int(counts[k]), int(rng.integers(0, ncomp))))
    rules = []
    pairs = set()
    for _ in range(bimol_tries or int(rng.integers(1, 2 * ns))):
        a, b = (int(v) for v in rng.integers(0, ns, 2))
        if rng.random() < 0.15:
            b = a
        if (min(a, b), max(a, b)) in pairs:
            continue
        pairs.add((min(a, b), max(a, b)))
        p = [0.0, 1.0, float(rng.uniform(0.05, 1.0))][int(rng.integers(0, 3))]
        p1 = int(rng.integers(-1, ns))
        p2 = int(rng.integers(-1, ns))
        rules.append(W.bimol(a, b, p1, p2, float(rng.uniform(0.006, 0.03)), p))
    budget = {(k, c): 1.0 for k in range(ns) for c in range(ncomp)}
    n_uni = {k: 0 for k in range(ns)}
    for _ in range(unimol_tries or int(rng.integers(1, 3 * ns))):
        if len(rules) >= 255:
            break
        a = int(rng.integers(0, ns))
        if n_uni[a] >= 4:
            continue
        kinds = [W.KEEP, W.SPLIT, W.EMIT] + ([W.TRANSLOCATE] if ncomp == 2 else [])
        placement = kinds[int(rng.integers(0, len(kinds)))]
        frm = int(rng.integers(0, ncomp)) if (placement == W.TRANSLOCATE or rng.random() < 0.3) \
            and ncomp == 2 else -1
        comps = range(ncomp) if frm < 0 else [frm]
        p = float(rng.uniform(0.002, 0.05))
        if any(budget[(a, c)] < p for c in comps):
            continue
        for c in comps:
            budget[(a, c)] -= p
        release = float(rng.uniform(0.002, 0.06))
        if placement == W.KEEP:
            rules.append(W.unimol(a, int(rng.integers(-1, ns)), p))
        elif placement == W.TRANSLOCATE:
            rules.append(W.unimol(a, int(rng.integers(-1, ns)), p, placement=W.TRANSLOCATE,
                                  release=release, from_comp=frm, to_comp=1 - frm))
        else:
            p1 = int(rng.integers(0, ns)) if placement == W.SPLIT else int(rng.integers(-1, ns))
            rules.append(W.unimol(a, p1, p, placement=placement, p2=int(rng.integers(0, ns)),
                                  release=release, from_comp=frm))
        n_uni[a] += 1
    # dense: about 4,000 agents per cubic micrometre
    vol = n / 4000.0
    kw = {}
    if geometry == W.PERIODIC_BOX:
        kw["box_um"] = float(max(vol ** (1 / 3), 0.2))
    else:
        r = float(max((vol * 3 / (4 * np.pi)) ** (1 / 3), 0.15))
        kw["outer_radius_um"] = r
        if geometry == W.NESTED_SPHERES:
            kw["inner_radius_um"] = 0.6 * r
    return W.Model(f"fuzz{seed}", geometry, 1e-6, seed, species, rules, capacity=4 * n + 4096,
                   **kw)


@pytest.mark.parametrize("seed", range(24))
def test_random_models_match_oracle(seed):
    m = random_model(seed)
    run_pair(m, [1, 2, 5, 12, 25])


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("seed", range(24))
def test_random_models_in_either_search(seed, mode):
    # the same random models with the chunked search and over the claimer
    # list (the automatic choice takes the list for most of these sizes)
    import paper_2606_14603_amd as mabm
    m = random_model(seed)
    run_pair(m, [1, 2, 5, 12, 25], params={mabm.PARAM_PROPOSE_MODE: mode})


@pytest.mark.parametrize("seed", [100, 101, 102])
def test_random_models_binning_every_step(seed):
    import paper_2606_14603_amd as mabm
    m = random_model(seed)
    g, _ = run_pair(m, [1, 7, 20])
    h = mabm.Sim(m, record=True, cell_um=0.0)
    h.set_param(mabm.PARAM_BIN_EVERY_MAX, 1)
    h.step(20)
    a, b = g.export(), h.export()
    for k in a:
        assert np.array_equal(a[k].view(np.uint32) if a[k].dtype == np.float32 else a[k],
                              b[k].view(np.uint32) if b[k].dtype == np.float32 else b[k]), k


@pytest.mark.parametrize("seed", range(200, 240))
def test_random_model_batches_match_oracle(seed):
    # one random model, five simulations of it with their own seeds, volumes
    # and initial counts (one of them empty), stepped as one batch
    from test_gpu_batch import run_batch
    base = random_model(seed)
    rng = np.random.default_rng(seed + 1)
    models = []
    for k in range(5):
        scale = 0.0 if k == 3 else float(rng.uniform(0.3, 1.5))
        species = [W.Species(s.name, s.diffusion_um2_s, int(s.count * scale), s.compartment)
                   for s in base.species]
        f = max(scale, 0.3) ** (1 / 3)
        kw = ({"box_um": base.box_um * f} if base.geometry == W.PERIODIC_BOX else
              {"outer_radius_um": base.outer_radius_um * f,
               "inner_radius_um": base.inner_radius_um * f})
        n = sum(s.count for s in species)
        models.append(base.with_(name=f"{base.name}_{k}", seed=seed * 10 + k, species=species,
                                 capacity=4 * n + 4096, **kw))
    run_batch(models, [1, 3, 10, 20])


def scaled(m: W.Model, n: int) -> W.Model:
    """m with about n agents at the same density, its splits and emissions
    five times rarer (births stay within a step's limit and the capacity)."""
    from dataclasses import replace
    rules = [r if r.kind == W.BIMOL or r.placement in (W.KEEP, W.TRANSLOCATE)
             else replace(r, prob_per_step=r.prob_per_step / 5) for r in m.rules]
    m = m.with_(rules=rules)
    f = n / max(m.n_agents, 1)
    species = [W.Species(s.name, s.diffusion_um2_s, int(round(s.count * f)), s.compartment)
               for s in m.species]
    g = f ** (1 / 3)
    kw = ({"box_um": m.box_um * g} if m.geometry == W.PERIODIC_BOX else
          {"outer_radius_um": m.outer_radius_um * g, "inner_radius_um": m.inner_radius_um * g})
    total = sum(s.count for s in species)
    return m.with_(species=species, capacity=4 * total + 4096, **kw)


@pytest.mark.parametrize("seed", range(300, 310))
def test_random_larger_models_and_launch_shapes(seed):
    # 20k-60k agents (many chunks, scan tiles and a ragged tail), a random
    # cell size, launch shape and graph replay: results stay the oracle's
    import oracle
    import paper_2606_14603_amd as mabm
    from parity import assert_same
    rng = np.random.default_rng(seed)
    m = scaled(random_model(seed), int(rng.integers(20_000, 60_000)))
    rmax = max([r.radius_um for r in m.rules if r.kind == W.BIMOL] + [0.006])
    cell = 0.0 if rng.random() < 0.3 else float(rmax * rng.uniform(1.05, 4.0))
    g = mabm.Sim(m, record=True, cell_um=cell, graphs=bool(rng.random() < 0.5))
    g.set_param(mabm.PARAM_PROPOSE_LANES, int(rng.choice([0, 8, 16])))
    g.set_param(mabm.PARAM_PROPOSE_MIN_WORKGROUPS, int(rng.choice([0, 256, 4096])))
    g.set_param(mabm.PARAM_PROPOSE_MODE, int(rng.choice([0, 1, 2])))
    G, _ = g.grid()
    o = oracle.OracleSim(m, grid_n=G)
    done = 0
    for c in (1, 4, 17, 40):
        g.step(c - done)
        o.step(c - done)
        done = c
        assert_same(g.export(), o.export(), f"{m.name} t={c} G={G}")


@pytest.mark.parametrize("seed", range(400, 406))
def test_checkpoint_resume_continues_the_trajectory(seed):
    # export a random model's state mid-run, import it into a fresh
    # simulation at the same step, and run both on: identical to the
    # uninterrupted run, and to the oracle
    import oracle
    import paper_2606_14603_amd as mabm
    from parity import assert_same
    m = random_model(seed)
    g = mabm.Sim(m, record=True)
    G, _ = g.grid()
    o = oracle.OracleSim(m, grid_n=G)
    g.step(13)
    o.step(13)
    e = g.export()
    n, next_id = g.size()
    _, t = g.counts()
    assert t == 13
    h = mabm.Sim(m, record=True)
    h.import_state(e["id"], e["species"], e["x"], e["y"], e["z"], next_id, t)
    assert h.grid()[0] == G
    done = 0
    for c in (1, 5, 12):
        for sim in (g, h, o):
            sim.step(c - done)
        done = c
        a, b = g.export(), h.export()
        for f in ("id", "species", "x", "y", "z", "key"):
            assert np.array_equal(a[f].view(np.uint32) if a[f].dtype == np.float32 else a[f],
                                  b[f].view(np.uint32) if b[f].dtype == np.float32 else b[f]), f
        assert_same(a, o.export(), f"{m.name} t={13 + c}")
        assert h.counts()[1] == 13 + c


@pytest.mark.parametrize("seed", range(500, 506))
def test_random_models_at_the_table_limits(seed):
    # 64 species and up to 255 rules (pair rules with indices above 127)
    m = random_model(seed, ns=64, bimol_tries=170, unimol_tries=400)
    assert len(m.species) == 64 and len(m.rules) > 200
    run_pair(m, [1, 3, 10, 20])


@pytest.mark.parametrize("seed", [600, 601, 602])
def test_random_batch_counts_ring(seed):
    # the device counts ring of a batch of random models, against the
    # oracle's counts of each simulation run alone
    import oracle
    import paper_2606_14603_amd as mabm
    base = random_model(seed)
    models = [base.with_(name=f"{base.name}_{k}", seed=seed * 10 + k) for k in range(3)]
    b = mabm.Batch(models, graphs=True)
    b.record_counts(4, entries=64)
    b.step(9)
    b.step(15)
    steps, counts = b.ring()
    assert list(steps) == [4, 8, 12, 16, 20, 24]
    for k, m in enumerate(models):
        o = oracle.OracleSim(m)
        for e, st in enumerate(steps):
            o.step(int(st) - (int(steps[e - 1]) if e else 0))
            want, t = o.counts()
            assert t == st
            assert np.array_equal(counts[e, k, :len(m.species)], want), (k, st)


def test_random_models_served_concurrently():
    # requests of different random models served concurrently on streams
    # of their own: each final state equals, agent by agent, the oracle's
    # for the model run alone
    from paper_2606_14603_amd import serve
    from test_gpu_serve import check_served
    models = [random_model(700 + k).with_(steps=30 + 7 * k) for k in range(6)]
    res = serve.Server(1 << 34, max_active=4, chunk=16, record=True,
                       keep_state=True).run(models, np.zeros(len(models)))
    check_served(res, models, "random models, concurrent")


def test_hundred_more_random_models_in_both_searches():
    # 100 further random models (every fourth scaled to 20k-80k agents),
    # each with the chunked search and over the claimer list; where the
    # oracle outgrows the capacity, the library reports E_CAPACITY at the
    # same checkpoint
    import oracle
    import paper_2606_14603_amd as mabm
    from parity import assert_same
    overflowed = 0
    for seed in range(1000, 1100):
        rng = np.random.default_rng(seed)
        m = random_model(seed)
        if seed % 4 == 0:
            m = scaled(m, int(rng.integers(20_000, 80_000)))
        for mode in (1, 2):
            g = mabm.Sim(m, record=True, graphs=bool(seed % 3 == 0))
            g.set_param(mabm.PARAM_PROPOSE_MODE, mode)
            o = oracle.OracleSim(m, grid_n=g.grid()[0])
            done = 0
            for c in (1, 6, 30):
                g.step(c - done)
                try:
                    o.step(c - done)
                except oracle.OracleError:
                    with pytest.raises(mabm.MabmError) as err:
                        g.counts()
                    assert err.value.code == mabm.E_CAPACITY
                    overflowed += 1
                    break
                done = c
                assert_same(g.export(), o.export(), f"{m.name} mode {mode} t={c}")
    assert overflowed <= 8
