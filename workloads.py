"""Seeded synthetic workloads of the molecule-agent step (model definitions).

This module is the only thing shared by the HIP library's tests and the CPU
oracle: it builds *inputs* (species, initial counts, rules, geometry) and
holds none of the step's arithmetic.  Every random choice is drawn from a
numpy Generator with a stated seed.

The paper's models (the MAPK/ERK + dabrafenib model of Sec. 3.1 with the
initial concentrations of its species table, and the cFos network of
Sec. 3.4) need parameters from earlier work that are not available, so the
workloads below are synthetic stand-ins with the paper's concentration
ratios, compartment structure and rule types:

* ``c1`` reversible binding A + B <-> C in a periodic 2 um cube, 20k agents.
* ``c2`` an 8-species MAPK-like cascade in a 5 um sphere, 2M agents, counts
  from the species-table ratios with seeded log-normal jitter.
* ``c3`` a two-compartment nuclear-signalling network (nucleus 3 um inside a
  cell of 8 um), ~5M agents, with translocation, transcription (emission),
  an Erlang-delayed negative regulator and degradation.
* ``c4_sweep`` the dose x replicate set of scaled copies of c2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Tuple

import numpy as np

# interface enums (same values as the C headers)
PERIODIC_BOX, SPHERE, NESTED_SPHERES = 0, 1, 2
BIMOL, UNIMOL = 0, 1
KEEP, SPLIT, EMIT, TRANSLOCATE = 0, 1, 2, 3
NUCLEUS, CYTOPLASM = 0, 1  # compartments of the nested geometry


@dataclass
class Species:
    name: str
    diffusion_um2_s: float
    count: int
    compartment: int = 0


@dataclass
class Rule:
    kind: int
    reactants: Tuple[int, int]
    products: Tuple[int, int]
    prob_per_step: float
    radius_um: float = 0.0
    placement: int = KEEP
    release_radius_um: float = 0.0
    from_comp: int = -1
    to_comp: int = -1


@dataclass
class Model:
    name: str
    geometry: int
    dt_s: float
    seed: int
    species: List[Species]
    rules: List[Rule] = field(default_factory=list)
    box_um: float = 0.0
    outer_radius_um: float = 0.0
    inner_radius_um: float = 0.0
    capacity: int = 0
    cell_um: float = 0.0
    steps: int = 1

    @property
    def n_agents(self) -> int:
        return sum(s.count for s in self.species)

    def with_(self, **kw) -> "Model":
        return replace(self, **kw)


def bimol(a, b, p1, p2, radius, prob) -> Rule:
    return Rule(BIMOL, (a, b), (p1, p2), prob, radius_um=radius)


def unimol(a, p1, prob, placement=KEEP, p2=-1, release=0.0, from_comp=-1, to_comp=-1) -> Rule:
    return Rule(UNIMOL, (a, -1), (p1, p2), prob, placement=placement,
                release_radius_um=release, from_comp=from_comp, to_comp=to_comp)


# --------------------------------------------------------------------------
# C1: reversible binding A + B <-> C
# --------------------------------------------------------------------------
def c1(n_a: int = 10_000, n_b: int = 10_000, n_c: int = 0, box_um: float = 2.0,
       seed: int = 0, steps: int = 1000, bind_p: float = 0.5, unbind_p: float = 1e-3,
       radius_um: float = 0.010, release_um: float = 0.005) -> Model:
    """A + B -> C on contact (radius 10 nm, p = 0.5), C -> A + B at 1e-3/step
    releasing the pair +-u from the complex, u uniform in the 5 nm ball."""
    sp = [Species("A", 1.0, n_a), Species("B", 1.0, n_b), Species("C", 0.5, n_c)]
    rules = [bimol(0, 1, 2, -1, radius_um, bind_p),
             unimol(2, 0, unbind_p, placement=SPLIT, p2=1, release=release_um)]
    n = n_a + n_b + n_c
    return Model("c1_ab_c", PERIODIC_BOX, 1e-6, seed, sp, rules, box_um=box_um,
                 capacity=n + max(64, n // 16), steps=steps)


# --------------------------------------------------------------------------
# C2: MAPK-like cascade in one cytoplasm
# --------------------------------------------------------------------------
C2_SPECIES = ["kinase1", "inhibitor", "kinase2", "p-kinase2", "kinase3", "p-kinase3",
              "phosphatase", "kinase1-inhibitor"]
C2_D = [1.0, 5.0, 1.0, 1.0, 1.0, 1.0, 1.0, 0.5]
# molar ratios from the paper's species table: BRAF 3 nM; MEK 1.2 uM;
# pERK + ppERK = 1.1986 uM; phosphatase 1 + 2 = 0.1203 uM; the inhibitor at
# 60.9 nM, the geometric middle of the 3-decade dose range below the 1.9246 uM
# top dose; unphosphorylated kinase3, p-kinase2 and the complex start at 0.
_TABLE_TOTAL_M = 3e-9 + 0.0 + 8.0074e-8 + 1.1185e-6 + 1.2e-6 + 0.0 + 0.0 + 3e-10 + 1.2e-7
C2_BASE_M = [3e-9, 1.9246e-6 * 10 ** -1.5, 1.2e-6, 0.0, 0.0, 8.0074e-8 + 1.1185e-6,
             3e-10 + 1.2e-7, 0.0]
C2_TOP_DOSE_FRACTION = 1.9246e-6 / (1.9246e-6 + _TABLE_TOTAL_M)


def c2_counts(n_total: int, seed: int = 0, inhibitor_fraction: float | None = None,
              jitter_sd: float = 0.25) -> List[int]:
    """Integer species counts from the ratio vector times exp(N(0, sd^2))
    jitter (numpy seed ``seed``), normalised to ``n_total``; the rounding
    remainder goes to the largest species.  With ``inhibitor_fraction`` the
    inhibitor count is fixed to that fraction first."""
    rng = np.random.default_rng(seed)
    jit = np.exp(rng.normal(0.0, jitter_sd, len(C2_BASE_M)))
    w = np.array(C2_BASE_M) * jit
    counts = np.zeros(len(w), np.int64)
    rest = n_total
    if inhibitor_fraction is not None:
        counts[1] = int(round(inhibitor_fraction * n_total))
        w[1] = 0.0
        rest = n_total - counts[1]
    share = np.floor(rest * w / w.sum()).astype(np.int64)
    counts += share
    counts[int(np.argmax(w))] += n_total - int(counts.sum())
    return [int(c) for c in counts]


def c2_rules(deg_p: float = 1e-5) -> List[Rule]:
    """5 contact rules (inhibitor binding, two catalytic phosphorylations, two
    dephosphorylations) and 7 first-order degradations: 12 rules."""
    k1, I, k2, pk2, k3, pk3, ph, k1i = range(8)
    rules = [bimol(k1, I, k1i, -1, 0.010, 0.5),
             bimol(k1, k2, k1, pk2, 0.0075, 0.2),
             bimol(pk2, k3, pk2, pk3, 0.0075, 0.2),
             bimol(ph, pk2, ph, k2, 0.005, 0.1),
             bimol(ph, pk3, ph, k3, 0.005, 0.1)]
    for s in (k1, I, k2, pk2, k3, pk3, k1i):
        rules.append(unimol(s, -1, deg_p))
    return rules


def c2(n_total: int = 2_000_000, seed: int = 0, steps: int = 5000,
       inhibitor_fraction: float | None = None, radius_um: float | None = None,
       count_seed: int = 0) -> Model:
    """Reflecting 5 um sphere at the density of 2M agents (3,820 /um^3);
    smaller ``n_total`` shrinks the radius to keep that density."""
    if radius_um is None:
        radius_um = 5.0 * (n_total / 2_000_000) ** (1.0 / 3.0)
    counts = c2_counts(n_total, count_seed, inhibitor_fraction)
    sp = [Species(nm, d, c) for nm, d, c in zip(C2_SPECIES, C2_D, counts)]
    return Model("c2_mapk", SPHERE, 1e-6, seed, sp, c2_rules(), outer_radius_um=radius_um,
                 capacity=n_total, steps=steps)


# --------------------------------------------------------------------------
# C3: two-compartment nuclear signalling
# --------------------------------------------------------------------------
C3_SPECIES = ["carrier", "gene", "gene-repressed", "mRNA", "protein", "p-protein",
              "F1", "F2", "F3", "F"]


def c3(n_total: int = 5_000_000, seed: int = 0, steps: int = 10_000, n_genes: int | None = None,
       scale_radius: bool = True) -> Model:
    """Nucleus (R = 3 um) inside a cell (R = 8 um).  Carriers (ERK-like)
    cross the membrane at 1e-4/step each way; genes in the nucleus emit mRNA
    at 0.01/step; mRNA degrades at 1e-4/step, leaves the nucleus at
    1e-3/step and in the cytoplasm emits protein at 1e-3/step; protein is
    phosphorylated on contact with a carrier; the phosphorylated protein
    induces the regulator through an Erlang chain F1 -> F2 -> F3 -> F
    (1e-3/step per stage), F enters the nucleus, is bound by genes (repression) and
    is released again at 1e-3/step."""
    s = (n_total / 5_000_000) ** (1.0 / 3.0) if scale_radius else 1.0
    r_in, r_out = 3.0 * s, 8.0 * s
    if n_genes is None:
        n_genes = max(1, n_total // 5000)
    car, gene, grep, mrna, prot, pprot, f1, f2, f3, f = range(10)
    sp = [Species("carrier", 1.0, n_total - n_genes, CYTOPLASM),
          Species("gene", 0.0, n_genes, NUCLEUS),
          Species("gene-repressed", 0.0, 0, NUCLEUS),
          Species("mRNA", 0.5, 0, NUCLEUS),
          Species("protein", 1.0, 0, CYTOPLASM),
          Species("p-protein", 1.0, 0, CYTOPLASM),
          Species("F1", 1.0, 0, CYTOPLASM),
          Species("F2", 1.0, 0, CYTOPLASM),
          Species("F3", 1.0, 0, CYTOPLASM),
          Species("F", 1.0, 0, CYTOPLASM)]
    rules = [
        unimol(car, -1, 1e-4, placement=TRANSLOCATE, release=0.005, from_comp=CYTOPLASM,
               to_comp=NUCLEUS),
        unimol(car, -1, 1e-4, placement=TRANSLOCATE, release=0.005, from_comp=NUCLEUS,
               to_comp=CYTOPLASM),
        unimol(gene, -1, 0.01, placement=EMIT, p2=mrna, release=0.005, from_comp=NUCLEUS),
        unimol(mrna, -1, 1e-4),
        unimol(mrna, -1, 1e-3, placement=TRANSLOCATE, release=0.005, from_comp=NUCLEUS,
               to_comp=CYTOPLASM),
        unimol(mrna, -1, 1e-3, placement=EMIT, p2=prot, release=0.005, from_comp=CYTOPLASM),
        bimol(prot, car, pprot, car, 0.0075, 0.2),
        unimol(prot, -1, 1e-4),
        unimol(pprot, -1, 1e-4),
        unimol(pprot, -1, 1e-3, placement=EMIT, p2=f1, release=0.005),
        unimol(f1, f2, 1e-3),
        unimol(f2, f3, 1e-3),
        unimol(f3, f, 1e-3),
        unimol(f, -1, 1e-4, placement=TRANSLOCATE, release=0.005, from_comp=CYTOPLASM,
               to_comp=NUCLEUS),
        unimol(f, -1, 1e-4),
        bimol(gene, f, grep, -1, 0.010, 0.5),
        unimol(grep, gene, 1e-3, placement=SPLIT, p2=f, release=0.005),
    ]
    return Model("c3_nuclear", NESTED_SPHERES, 1e-6, seed, sp, rules, outer_radius_um=r_out,
                 inner_radius_um=r_in, capacity=int(n_total * 1.5) + 4096, steps=steps)


# --------------------------------------------------------------------------
# C4: dose x replicate sweep of scaled copies of C2
# --------------------------------------------------------------------------
def c5_request(k: int, rng: np.random.Generator, n_min: int, n_max: int, h_min: int,
               h_max: int) -> Model:
    """One serving request: a random non-empty subset of C2's contact rules,
    closed under its species (every C2 rule, contact or degradation, whose
    reactants and products all lie in the subset's species is included), its
    species renumbered 0.. in C2 order, counts from a random positive ratio
    vector scaled to a log-uniform size, a uniform horizon, seed k; C2's
    density in a sphere."""
    full = c2_rules()
    bim = [r for r in full if r.kind == BIMOL]
    while True:
        pick = [r for r in bim if rng.random() < 0.5]
        if pick:
            break
    used = sorted({s for r in pick for s in (*r.reactants, *r.products) if s >= 0})
    while True:  # closure under the species in use
        rules = [r for r in full if all(s < 0 or s in used for s in (*r.reactants, *r.products))]
        grown = sorted(set(used) | {s for r in rules for s in (*r.reactants, *r.products) if s >= 0})
        if grown == used:
            break
        used = grown
    remap = {s: i for i, s in enumerate(used)}
    n_total = int(math.exp(rng.uniform(math.log(n_min), math.log(n_max))))
    w = rng.uniform(0.05, 1.0, len(used))
    counts = np.floor(w / w.sum() * n_total).astype(np.int64)
    counts[np.argmax(counts)] += n_total - int(counts.sum())
    sp = [Species(C2_SPECIES[s], C2_D[s], int(c)) for s, c in zip(used, counts)]
    rr = [replace(r, reactants=tuple(remap.get(s, -1) if s >= 0 else -1 for s in r.reactants),
                  products=tuple(remap.get(s, -1) if s >= 0 else -1 for s in r.products))
          for r in rules]
    horizon = int(rng.integers(h_min, h_max + 1))
    radius = 5.0 * (n_total / 2_000_000) ** (1.0 / 3.0)
    return Model(f"c5_req{k}", SPHERE, 1e-6, k, sp, rr, outer_radius_um=radius,
                 capacity=n_total, steps=horizon)


def c5_requests(n: int = 256, seed: int = 0, n_min: int = 50_000, n_max: int = 1_000_000,
                h_min: int = 200, h_max: int = 2000) -> List[Model]:
    """A stream of n serving requests (numpy seed ``seed``), each a model of
    its own from ``c5_request``; ``steps`` is the request's horizon."""
    rng = np.random.default_rng(seed)
    return [c5_request(k, rng, n_min, n_max, h_min, h_max) for k in range(n)]


def poisson_arrivals(n: int, rate_per_s: float, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, n))


def c4_sweep(n_doses: int = 16, n_reps: int = 64, n_min: int = 20_000, n_max: int = 200_000,
             steps: int = 2000, size_seed: int = 0) -> List[Model]:
    """16 inhibitor doses log-spaced over 3 decades below the top-dose
    fraction, x 64 replicates (seed 64 j + k); sizes log-uniform in
    [n_min, n_max] from numpy seed ``size_seed``; each copy keeps C2's
    density."""
    rng = np.random.default_rng(size_seed)
    sizes = np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_doses * n_reps))
    models = []
    for j in range(n_doses):
        frac = C2_TOP_DOSE_FRACTION * 10.0 ** (-3.0 + 3.0 * j / max(1, n_doses - 1))
        for k in range(n_reps):
            n = int(sizes[j * n_reps + k])
            m = c2(n, seed=n_reps * j + k, steps=steps, inhibitor_fraction=frac)
            m.name = f"c4_d{j}_r{k}"
            models.append(m)
    return models
