"""Pins of the oracle's step against laws that the mathematics fixes (CPU).

Each test targets one phase of the step definition, chosen so that a
plausible slip (a dropped factor, a wrong sign, a boundary rule that is
not exactly stationary, a wrong release placement) fails it:

* Brownian move: MSD = 6 D t within 2 % (about 3.5 standard errors at 20k
  agents) and per-axis one-step variance 2 D dt.
* Placement and boundaries: uniform law in box, sphere and shell (KS), and
  exact stationarity of the uniform law under the reject-the-move sphere.
* Rules: conservation of A + C and B + C; binomial degradation and emission
  counts; the two-state Markov law of translocation; the release geometry of
  a split; the detailed-balance steady state of A + B <-> C.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads as W


def min_image(d, L):
    return d - L * np.round(d / L)


def test_msd_equals_6Dt():
    D, dt, steps, L = 1.0, 1e-6, 1000, 2.0
    m = W.Model("msd", W.PERIODIC_BOX, dt, 12, [W.Species("A", D, 20000)], [], box_um=L,
                capacity=20000)
    s = oracle.OracleSim(m)
    e0 = s.export()
    s.step(1)
    e1 = s.export()
    d1 = np.stack([min_image(e1[k].astype(np.float64) - e0[k], L) for k in "xyz"])
    var1 = d1.var(axis=1)
    assert np.all(np.abs(var1 / (2 * D * dt) - 1.0) < 4.0 * math.sqrt(2.0 / 20000))
    s.step(steps - 1)
    e = s.export()
    assert np.array_equal(e["id"], e0["id"])
    d = np.stack([min_image(e[k].astype(np.float64) - e0[k], L) for k in "xyz"])
    msd = (d ** 2).sum(axis=0).mean()
    assert abs(msd / (6 * D * dt * steps) - 1.0) < 0.02


def test_uniform_placement_box_sphere_shell():
    box = oracle.OracleSim(W.Model("b", W.PERIODIC_BOX, 1e-6, 42, [W.Species("A", 1, 20000)],
                                   box_um=2.0, capacity=20000)).export()
    for k in "xyz":
        assert box[k].min() >= 0 and box[k].max() < 2.0
        assert stats.kstest(box[k] / 2.0, "uniform").pvalue > 1e-3
    R = 5.0
    sph = oracle.OracleSim(W.Model("s", W.SPHERE, 1e-6, 42, [W.Species("A", 1, 20000)],
                                   outer_radius_um=R, capacity=20000)).export()
    p = np.stack([sph[k].astype(np.float64) for k in "xyz"])
    r = np.sqrt((p ** 2).sum(0))
    assert r.max() <= R
    assert stats.kstest((r / R) ** 3, "uniform").pvalue > 1e-3
    assert stats.kstest((p[2] / r + 1) / 2, "uniform").pvalue > 1e-3
    assert stats.kstest((np.arctan2(p[1], p[0]) + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-3
    rin, rout = 1.0, 2.0
    nest = oracle.OracleSim(W.Model("n", W.NESTED_SPHERES, 1e-6, 42,
                                    [W.Species("in", 1, 10000, W.NUCLEUS),
                                     W.Species("out", 1, 10000, W.CYTOPLASM)],
                                    outer_radius_um=rout, inner_radius_um=rin,
                                    capacity=20000)).export()
    p = np.stack([nest[k].astype(np.float64) for k in "xyz"])
    r = np.sqrt((p ** 2).sum(0))
    inner = nest["species"] == 0
    assert r[inner].max() < rin and r[~inner].min() >= rin and r[~inner].max() <= rout
    assert stats.kstest((r[inner] / rin) ** 3, "uniform").pvalue > 1e-3
    assert stats.kstest((r[~inner] ** 3 - rin ** 3) / (rout ** 3 - rin ** 3),
                        "uniform").pvalue > 1e-3


def test_sphere_reject_move_keeps_uniform_law():
    # a 0.1 um sphere with D = 5 um^2/s: most agents meet the wall in 500 steps
    R = 0.1
    s = oracle.OracleSim(W.Model("s", W.SPHERE, 1e-6, 314, [W.Species("A", 5.0, 20000)],
                                 outer_radius_um=R, capacity=20000))
    s.step(500)
    e = s.export()
    p = np.stack([e[k].astype(np.float64) for k in "xyz"])
    r = np.sqrt((p ** 2).sum(0))
    assert r.max() <= R * (1 + 1e-6)
    assert stats.kstest((r / R) ** 3, "uniform").pvalue > 1e-3


def test_conservation_and_pair_invariants_c1():
    m = W.c1(n_a=4000, n_b=4000, box_um=2.0 * (8000 / 20000) ** (1 / 3), unbind_p=5e-3)
    s = oracle.OracleSim(m, grid_n=11)
    last_c = 0
    for _ in range(150):
        s.step(1)
        (na, nb, nc), _ = s.counts()
        assert na + nc == 4000 and nb + nc == 4000
        e = s.export()
        assert np.all(np.diff(e["id"].astype(np.int64)) > 0)
        paired = e["partner"] != oracle.NONE32
        # a confirmed A+B pair leaves a C (the claimer) whose partner B died
        assert np.all(e["species"][paired] == 2)
        assert not np.isin(e["partner"][paired], e["id"]).any()
        # a C that split this step released its products within 2 delta
        split = e["event"] == 1
        assert np.all(e["species"][split] == 0)
        last_c = nc
    assert last_c > 0


def test_brute_force_equals_cell_list_search():
    for m in (W.c1(n_a=1000, n_b=1000, box_um=2.0 * (2000 / 20000) ** (1 / 3), unbind_p=2e-2),
              W.c2(2000, seed=42), W.c3(2000, seed=12, n_genes=40)):
        a = oracle.OracleSim(m, grid_n=7, search="cells")
        b = oracle.OracleSim(m, grid_n=7, search="brute")
        for _ in range(4):
            a.step(10)
            b.step(10)
            ea, eb = a.export(), b.export()
            for k in ea:
                assert np.array_equal(ea[k], eb[k]), (m.name, k)


def test_degradation_is_binomial():
    p, n0, t = 0.01, 10000, 100
    m = W.Model("deg", W.SPHERE, 1e-6, 101010, [W.Species("X", 1.0, n0)],
                [W.unimol(0, -1, p)], outer_radius_um=1.0, capacity=n0)
    s = oracle.OracleSim(m)
    s.step(t)
    (n,), _ = s.counts()
    q = (1 - p) ** t
    assert abs(n - n0 * q) <= 3 * math.sqrt(n0 * q * (1 - q))


def test_emission_is_binomial_and_ids_follow_parents():
    p, g, t = 0.02, 500, 100
    m = W.Model("emit", W.SPHERE, 1e-6, 42, [W.Species("G", 0.0, g), W.Species("M", 1.0, 0)],
                [W.unimol(0, -1, p, placement=W.EMIT, p2=1, release=0.005)],
                outer_radius_um=1.0, capacity=g + 4000)
    s = oracle.OracleSim(m)
    prev_next = g
    for _ in range(t):
        s.step(1)
        e = s.export()
        n, nid = s.size()
        born = e["id"] >= prev_next
        # children of one step: consecutive ids, given in increasing parent-id order
        assert np.array_equal(np.sort(e["id"][born]), np.arange(prev_next, nid))
        em = np.sort(e["id"][(e["event"] == 0)])
        assert len(em) == nid - prev_next
        prev_next = nid
        # a child sits within delta of its (immobile) parent
        if born.any():
            gpos = np.stack([e[k][e["species"] == 0] for k in "xyz"], 1).astype(np.float64)
            gid = e["id"][e["species"] == 0]
            emitted = np.sort(gid[np.isin(gid, em)])
            kids = np.stack([e[k][born] for k in "xyz"], 1).astype(np.float64)
            kid_ids = e["id"][born]
            order = np.argsort(kid_ids)
            par = gpos[np.searchsorted(gid, emitted)]
            dist = np.sqrt(((kids[order] - par) ** 2).sum(1))
            assert np.all(dist <= 0.005 * (1 + 1e-5))
    (ng, nm), _ = s.counts()
    assert ng == g
    mean, sd = g * t * p, math.sqrt(g * t * p * (1 - p))
    assert abs(nm - mean) <= 3 * sd


def test_translocation_two_state_law():
    n, p_in, p_out, t = 10000, 0.01, 0.02, 50
    rin, rout = 1.0, 2.0
    m = W.Model("tr", W.NESTED_SPHERES, 1e-6, 12, [W.Species("E", 1.0, n, W.CYTOPLASM)],
                [W.unimol(0, -1, p_in, placement=W.TRANSLOCATE, release=0.005,
                          from_comp=W.CYTOPLASM, to_comp=W.NUCLEUS),
                 W.unimol(0, -1, p_out, placement=W.TRANSLOCATE, release=0.005,
                          from_comp=W.NUCLEUS, to_comp=W.CYTOPLASM)],
                outer_radius_um=rout, inner_radius_um=rin, capacity=n)
    s = oracle.OracleSim(m)
    s.step(t)
    e = s.export()
    r = np.sqrt(sum(e[k].astype(np.float64) ** 2 for k in "xyz"))
    n_in = int((r < rin).sum())
    pi = p_in / (p_in + p_out)
    q = pi * (1 - (1 - p_in - p_out) ** t)
    assert abs(n_in - n * q) <= 3 * math.sqrt(n * q * (1 - q))
    # translocated agents sit just across the membrane, radially
    moved = e["event"] >= 0
    assert moved.any()
    assert np.all(np.abs(np.abs(r[moved] - rin) - 0.005) < 1e-5)


def test_split_places_products_uniformly_in_release_ball():
    n, delta = 4000, 0.005
    m = W.Model("split", W.PERIODIC_BOX, 1e-6, 42,
                [W.Species("A", 1.0, 0), W.Species("B", 1.0, 0), W.Species("C", 0.0, n)],
                [W.unimol(2, 0, 1.0, placement=W.SPLIT, p2=1, release=delta)],
                box_um=2.0, capacity=2 * n)
    s = oracle.OracleSim(m)
    e0 = s.export()
    s.step(1)
    e = s.export()
    a = e["species"] == 0
    b = e["species"] == 1
    assert a.sum() == n and b.sum() == n
    # child ids follow parent ids, so the k-th child belongs to the k-th C
    pa = np.stack([e[k][a] for k in "xyz"], 1).astype(np.float64)
    pb = np.stack([e[k][b] for k in "xyz"], 1).astype(np.float64)
    p0 = np.stack([e0[k] for k in "xyz"], 1).astype(np.float64)
    mid = p0  # D_C = 0: the complex does not move before splitting
    ua = min_image(pa - mid, 2.0)
    ub = min_image(pb - mid, 2.0)
    assert np.allclose(ua, -ub, atol=1e-6)
    rad = np.sqrt((ua ** 2).sum(1)) / delta
    assert rad.max() <= 1 + 1e-5
    assert stats.kstest(np.minimum(rad, 1.0) ** 3, "uniform").pvalue > 1e-3


def _solve_steady(n0, K_over_V):
    lo, hi = 0.0, float(n0)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid - K_over_V * (n0 - mid) ** 2 < 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def test_mass_action_steady_state_detailed_balance():
    """A + B <-> C with release uniform in the R-ball: detailed balance fixes
    q E[N_C] = p (V_R / V) E[N_A N_B].  Start at the stationary composition
    with uniform positions and compare time-averaged N_C over 12 seeds with
    the closed-form root, within 3 standard errors of the seed mean; the
    measured flux ratio q N_C / (p (V_R / V) N_A N_B) likewise within 3
    standard errors of 1.

    Scaled setup (so that the CPU run takes seconds and relaxes within the
    horizon): A + C = B + C = 2,000 agents in a periodic 1 um cube, contact
    radius 10 nm with p = 0.5, unbinding q = 1e-2 per step (release ball
    5 nm), 12 seeds x 1,500 steps sampled every 25.  The relaxation time
    falls with q, so the reversible-binding workload's own q = 1e-3 would
    need about ten times the horizon."""
    L, R, p, q, n0 = 1.0, 0.010, 0.5, 1e-2, 2000
    K_over_V = p * (4.0 / 3.0 * math.pi * R ** 3) / q / L ** 3
    nc_star = _solve_steady(n0, K_over_V)
    nc0 = int(round(nc_star))
    means, flux = [], []
    for seed in range(12):
        m = W.c1(n_a=n0 - nc0, n_b=n0 - nc0, n_c=nc0, box_um=L, seed=seed, bind_p=p,
                 unbind_p=q, radius_um=R, release_um=R / 2)
        s = oracle.OracleSim(m)
        ncs, prods = [], []
        for _ in range(60):
            s.step(25)
            (na, nb, nc), _ = s.counts()
            ncs.append(int(nc))
            prods.append(int(na) * int(nb))
        means.append(np.mean(ncs))
        flux.append(q * np.mean(ncs) / (K_over_V * q * np.mean(prods)))
    means = np.array(means)
    se = means.std(ddof=1) / math.sqrt(len(means))
    assert abs(means.mean() - nc_star) <= 3 * se, (means.mean(), nc_star, se)
    fr = np.array(flux)
    fse = fr.std(ddof=1) / math.sqrt(len(fr))
    assert abs(fr.mean() - 1.0) <= 3 * fse, (fr.mean(), fse)


def test_thread_count_changes_no_result():
    """The oracle's move phase and neighbour search run on several threads;
    children get ids in parent-id order and every other write is the
    agent's own, so one thread and four give the same id-keyed state on a
    model with births, deaths, splits, translocations and contact rules."""
    m = W.c3(30_000, steps=60)
    m = m.with_(rules=[r if r.prob_per_step >= 0.01 else dataclasses.replace(r, prob_per_step=r.prob_per_step * 50)
                       for r in m.rules])
    outs = []
    before = oracle.threads()
    try:
        for nt in (1, 4):
            assert oracle.threads(nt) == nt
            s = oracle.OracleSim(m, grid_n=64)
            s.step(60)
            outs.append((s.export(), s.counts()))
    finally:
        oracle.threads(before)
    (a, ca), (b, cb) = outs
    assert np.array_equal(ca[0], cb[0]) and ca[1] == cb[1]
    assert len(a["id"]) > m.n_agents  # births happened
    for k in a:
        x, y = a[k], b[k]
        if x.dtype == np.float32:
            x, y = x.view(np.uint32), y.view(np.uint32)
        assert np.array_equal(x, y), k
