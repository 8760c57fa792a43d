"""Engineered contact configurations that pin the propose/claim/apply phases
of the oracle (CPU).

Positions sit on a 2^-10 um lattice and the contact radius is 2^-7 um, so
every difference and squared distance is exact in float: a pair at exactly
the contact radius, ties between equidistant partners, pairs across the
periodic seam, two claimers contending for one target, homotypic pairs,
busy agents and pairs split by the nuclear membrane each have one correct
outcome that can be stated by hand.  Immobile species (D = 0) keep their
positions through the move.
"""
import math

import numpy as np
from scipy import stats

import oracle
import workloads as W

R = 2.0 ** -7
NONE = oracle.NONE32


def run_one(model, agents, next_id=None):
    """One step from an explicit state, with both neighbour searches; they
    must agree."""
    ids = [a[0] for a in agents]
    res = []
    for search in ("cells", "brute"):
        s = oracle.OracleSim(model, search=search)
        s.import_state(ids, [a[1] for a in agents], [a[2] for a in agents],
                       [a[3] for a in agents], [a[4] for a in agents],
                       next_id if next_id is not None else max(ids) + 1, 0)
        s.step(1)
        e = s.export()
        res.append({int(i): (int(sp), int(pa))
                    for i, sp, pa in zip(e["id"], e["species"], e["partner"])})
    assert res[0] == res[1]
    return res[0]


def prio(a, b, t=0, seed=0):
    lo, hi = min(a, b), max(a, b)
    return int(oracle.philox([lo, t, 4, hi], [seed & 0xFFFFFFFF, seed >> 32])[0])


def test_binding_ties_radius_seam_and_contention():
    A, B, C = 0, 1, 2
    m = W.Model("claims", W.PERIODIC_BOX, 1e-6, 0,
                [W.Species("A", 0.0, 0), W.Species("B", 0.0, 0), W.Species("C", 0.0, 0)],
                [W.bimol(A, B, C, -1, R, 1.0)], box_um=1.0, capacity=64)
    h = 0.5
    agents = [
        # tie at exactly the contact radius: the lower id (3) wins
        (10, A, h, h, h), (3, B, h, h - R, h), (5, B, h + R, h, h),
        # just beyond the radius: no contact
        (11, A, 0.25, 0.25, 0.25), (20, B, 0.25 + R + 2.0 ** -10, 0.25, 0.25),
        # across the periodic seam
        (12, A, 2.0 ** -10, 0.75, 0.75), (21, B, 1.0 - 2.0 ** -8, 0.75, 0.75),
        # two claimers for one target; the loser does not fall back to B 33
        (30, B, h, 0.25, 0.75), (31, A, h - 2.0 ** -8, 0.25, 0.75),
        (32, A, h + 2.0 ** -8, 0.25, 0.75), (33, B, h + 2.0 ** -8 + 2.0 ** -8 + 2.0 ** -9, 0.25, 0.75),
    ]
    out = run_one(m, agents)
    assert out[10] == (C, 3) and 3 not in out and out[5] == (B, NONE)
    assert out[11] == (A, NONE) and out[20] == (B, NONE)
    assert out[12] == (C, 21) and 21 not in out
    win = 31 if (prio(31, 30) << 32 | 31) < (prio(32, 30) << 32 | 32) else 32
    lose = 63 - win
    assert out[win] == (C, 30) and 30 not in out
    assert out[lose] == (A, NONE) and out[33] == (B, NONE)


def test_homotypic_catalysis_and_busy_agents():
    A, P, Dsp, X, E, S, Q = range(7)
    sp = [W.Species(n, 0.0, 0) for n in ("A", "P", "D", "X", "E", "S", "Q")]
    rules = [W.bimol(A, A, P, Dsp, R, 1.0),       # homotypic: lower id takes the claimer's role
             W.bimol(A, X, P, X, R, 1.0),         # X is always busy, so never a partner
             W.unimol(X, X, 1.0),                 # X converts to itself every step
             W.bimol(E, S, E, Q, R, 1.0)]         # catalysis: both survive
    m = W.Model("homo", W.PERIODIC_BOX, 1e-6, 7, sp, rules, box_um=1.0, capacity=64)
    agents = [(9, A, 0.5, 0.5, 0.5), (4, A, 0.5 + 2.0 ** -8, 0.5, 0.5),
              (6, A, 0.25, 0.25, 0.25), (7, X, 0.25 + 2.0 ** -8, 0.25, 0.25),
              (1, E, 0.75, 0.75, 0.75), (2, S, 0.75, 0.75 + 2.0 ** -8, 0.75)]
    out = run_one(m, agents)
    assert out[4] == (P, 9) and out[9] == (Dsp, 4)
    assert out[6] == (A, NONE) and out[7] == (X, NONE)
    assert out[1] == (E, 2) and out[2] == (Q, 1)


def test_pairs_never_cross_the_membrane():
    A, B, C = 0, 1, 2
    m = W.Model("memb", W.NESTED_SPHERES, 1e-6, 3,
                [W.Species("A", 0.0, 0), W.Species("B", 0.0, 0), W.Species("C", 0.0, 0)],
                [W.bimol(A, B, C, -1, R, 1.0)], outer_radius_um=1.0, inner_radius_um=0.5,
                capacity=64)
    agents = [(1, A, 0.5 - 2.0 ** -9, 0.0, 0.0), (2, B, 0.5 + 2.0 ** -9, 0.0, 0.0),
              (3, A, 0.0, 0.25, 0.0), (4, B, 0.0, 0.25 + 2.0 ** -8, 0.0)]
    out = run_one(m, agents)
    assert out[1] == (A, NONE) and out[2] == (B, NONE)
    assert out[3] == (C, 4) and 4 not in out


def test_competing_unimolecular_rules_have_exact_probabilities():
    n, p_deg, p_conv = 20000, 0.3, 0.2
    m = W.Model("comp", W.SPHERE, 1e-6, 42, [W.Species("X", 1.0, n), W.Species("Y", 1.0, 0)],
                [W.unimol(0, -1, p_deg), W.unimol(0, 1, p_conv)], outer_radius_um=1.0,
                capacity=n)
    s = oracle.OracleSim(m)
    s.step(1)
    (nx, ny), _ = s.counts()
    died = n - nx - ny
    for k, p in ((died, p_deg), (ny, p_conv)):
        assert abs(k - n * p) <= 3.5 * math.sqrt(n * p * (1 - p))
    e = s.export()
    assert np.all(e["event"][e["species"] == 1] == 1)


def test_random_dense_claims_are_a_matching_of_nearest_partners():
    """Dense random A/B mixture, p = 1: every confirmed pair is within R, each
    agent is in at most one pair, and every proposal whose key is the
    smallest at both ends is confirmed (checked against the brute-force
    candidate lists computed here from the moved positions, D = 0)."""
    rng = np.random.default_rng(12)
    n = 600
    L = 0.25
    m = W.Model("dense", W.PERIODIC_BOX, 1e-6, 11,
                [W.Species("A", 0.0, 0), W.Species("B", 0.0, 0), W.Species("C", 0.0, 0),
                 W.Species("D", 0.0, 0)],
                [W.bimol(0, 1, 2, 3, 0.02, 1.0)], box_um=L, capacity=n)
    pos = (np.floor(rng.uniform(0, L, (n, 3)) * 1024) / 1024).astype(np.float32)
    spc = rng.integers(0, 2, n)
    ids = rng.permutation(10 * n)[:n]
    s = oracle.OracleSim(m)
    s.import_state(ids, spc, pos[:, 0], pos[:, 1], pos[:, 2], 10 * n, 5)
    s.step(1)
    e = s.export()
    by_id = {int(i): k for k, i in enumerate(e["id"])}
    order = np.argsort(ids)
    P = pos[order].astype(np.float64)
    I = ids[order]
    Sp = spc[order]
    d = P[:, None, :] - P[None, :, :]
    d -= L * np.round(d / L)
    d2 = (d ** 2).sum(-1)
    R2 = np.float32(0.02) ** 2
    prop = {}
    for a in np.where(Sp == 0)[0]:
        cand = [b for b in np.where(Sp == 1)[0] if d2[a, b] <= R2]
        if cand:
            b = min(cand, key=lambda b: (np.float32(d2[a, b]), I[b]))
            prop[a] = b
    key = lambda x, y: (prio(int(I[x]), int(I[y]), t=5, seed=11) << 32) | int(I[y])
    slot = {}
    for a, b in prop.items():
        slot[a] = min(slot.get(a, 1 << 64), key(a, b))
        slot[b] = min(slot.get(b, 1 << 64), key(b, a))
    confirmed = {a: b for a, b in prop.items() if slot[a] == key(a, b) and slot[b] == key(b, a)}
    assert len(confirmed) > 5
    for a, b in confirmed.items():
        k = by_id[int(I[a])]
        assert e["species"][k] == 2 and e["partner"][k] == I[b]
        kb = by_id[int(I[b])]
        assert e["species"][kb] == 3 and e["partner"][kb] == I[a]
    n_pairs = int((e["species"] == 2).sum())
    assert n_pairs == len(confirmed)
