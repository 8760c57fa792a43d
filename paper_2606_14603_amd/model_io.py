"""Model files and the host-side model checks of the paper's simulator.

The paper's simulator takes a model as a structured JSON file (Sec. 2): the
molecular species (functional class, molecular weight, initial
concentration, localisation) and the reactions they take part in (partners,
rates, products), plus the volume and, with compartments, their sizes and
translocation rates.  From these it derives what the agents need: a sphere
radius per molecule from its molecular weight, a diffusion coefficient from
the Stokes-Einstein relation, molecule counts from concentrations and
volumes.  Before a run it checks the model's consistency (Sec. 2): every
referenced molecule exists, interaction definitions are reciprocal,
molecular weights are plausible and the volume fits the concentrations.

``load_model`` turns such a file (or dict) into a model the library runs
(``Sim(load_model(...))``); ``check_model`` lists every inconsistency.

File format (keys not listed are rejected; units in the key names):

    {"name": "mapk",
     "geometry": {"kind": "sphere", "radius_um": 5.0}      # or box_um / nested
     "dt_s": 1e-6, "seed": 0, "steps": 1000,
     "temperature_k": 310.15, "viscosity_pa_s": 6.913e-4,  # optional
     "species": [{"name": "BRAF", "class": "active", "mw_kda": 84.4,
                  "concentration_M": 3e-9, "compartment": "cytosol",
                  "partners": ["MEK"]}, ...],              # or diffusion_um2_s / count
     "reactions": [
        {"reactants": ["BRAF", "MEK"], "products": ["BRAF", "pMEK"],
         "radius_nm": 7.5, "probability": 0.2},            # contact (bimolecular)
        {"reactants": ["C"], "products": ["A", "B"], "placement": "split",
         "release_nm": 5, "probability": 1e-3},            # first order
        {"reactants": ["ES"], "products": ["E", "P"], "placement": "split",
         "release_nm": 5, "kcat_per_s": 20.0},             # k_cat timing
        {"reactants": ["ERK"], "products": ["ERK"], "placement": "translocate",
         "from": "cytosol", "to": "nucleus", "release_nm": 5, "probability": 1e-4}]}
"""
from __future__ import annotations

import json
import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

N_A = 6.02214076e23          # 1/mol
K_B = 1.380649e-23           # J/K
PROTEIN_DENSITY_G_CM3 = 1.35  # mean density of a folded protein (reading)
WATER_37C_PA_S = 6.913e-4    # viscosity of water at 37 C
MW_PLAUSIBLE_KDA = (0.1, 10_000.0)
MAX_VOLUME_FRACTION = 0.4    # molecules' own volume per compartment volume

BIMOL, UNIMOL = 0, 1
PLACEMENT = {"keep": 0, "split": 1, "emit": 2, "translocate": 3}
GEOMETRY = {"box": 0, "sphere": 1, "nested": 2}
COMPARTMENT = {"nucleus": 0, "cytosol": 1}
CLASSES = ("active", "inactive", "inhibited", "expressor")


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
    placement: int = 0
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


class ModelError(ValueError):
    def __init__(self, problems: List[str]):
        super().__init__("; ".join(problems))
        self.problems = problems


def radius_nm(mw_kda: float) -> float:
    """Radius of a sphere of protein density holding one molecule of the
    given molecular weight: r = (3 M / (4 pi rho N_A))^(1/3)."""
    mass_g = mw_kda * 1e3 / N_A
    vol_cm3 = mass_g / PROTEIN_DENSITY_G_CM3
    return (3.0 * vol_cm3 / (4.0 * math.pi)) ** (1.0 / 3.0) * 1e7


def stokes_einstein_um2_s(mw_kda: float, temperature_k: float = 310.15,
                          viscosity_pa_s: float = WATER_37C_PA_S) -> float:
    """D = k_B T / (6 pi eta r) for the molecule's sphere (Sec. 2)."""
    r_m = radius_nm(mw_kda) * 1e-9
    return K_B * temperature_k / (6.0 * math.pi * viscosity_pa_s * r_m) * 1e12


def compartment_volumes_um3(geom: dict) -> Dict[int, float]:
    kind = geom["kind"]
    if kind == "box":
        return {0: geom["box_um"] ** 3}
    if kind == "sphere":
        return {0: 4.0 / 3.0 * math.pi * geom["radius_um"] ** 3}
    vin = 4.0 / 3.0 * math.pi * geom["inner_radius_um"] ** 3
    vout = 4.0 / 3.0 * math.pi * geom["radius_um"] ** 3
    return {0: vin, 1: vout - vin}


def count_from_concentration(c_molar: float, volume_um3: float) -> int:
    """N = c V N_A, V in litres (1 um^3 = 1e-15 L), rounded."""
    return int(round(c_molar * volume_um3 * 1e-15 * N_A))


def kcat_probability(kcat_per_s: float, dt_s: float) -> float:
    """Per-step probability of a first-order event of rate k_cat: the
    enzyme-substrate complex releases its product after an exponential
    waiting time of mean 1/k_cat (Sec. 2: reaction timing from turnover
    numbers)."""
    return -math.expm1(-kcat_per_s * dt_s)


def _comp_index(spec: dict, geom_kind: str, where: str, problems: List[str]) -> int:
    name = spec.get("compartment", "cytosol")
    if geom_kind != "nested":
        return 0
    if name not in COMPARTMENT:
        problems.append(f"{where}: unknown compartment {name!r}")
        return 1
    return COMPARTMENT[name]


def check_model(doc: dict) -> List[str]:
    """Every inconsistency of a model document (empty list: consistent)."""
    problems: List[str] = []
    allowed = {"name", "geometry", "dt_s", "seed", "steps", "capacity", "temperature_k",
               "viscosity_pa_s", "species", "reactions", "cell_um"}
    for k in doc:
        if k not in allowed:
            problems.append(f"unknown key {k!r}")
    geom = doc.get("geometry", {})
    kind = geom.get("kind")
    if kind not in GEOMETRY:
        problems.append(f"geometry kind must be one of {sorted(GEOMETRY)}")
        return problems
    need = {"box": ("box_um",), "sphere": ("radius_um",), "nested": ("radius_um", "inner_radius_um")}[kind]
    for k in need:
        if not (isinstance(geom.get(k), (int, float)) and geom[k] > 0):
            problems.append(f"geometry.{k} must be > 0")
    if kind == "nested" and not problems and not geom["inner_radius_um"] < geom["radius_um"]:
        problems.append("geometry: the nucleus must be smaller than the cell")
    if not (isinstance(doc.get("dt_s"), (int, float)) and doc["dt_s"] > 0):
        problems.append("dt_s must be > 0")
    if problems:
        return problems
    vols = compartment_volumes_um3(geom)
    species = doc.get("species", [])
    names = [s.get("name") for s in species]
    if not species:
        problems.append("no species")
    for n in set(names):
        if names.count(n) > 1:
            problems.append(f"species {n!r} defined twice")
    excluded = {c: 0.0 for c in vols}
    for s in species:
        w = f"species {s.get('name')!r}"
        if s.get("class", "inactive") not in CLASSES:
            problems.append(f"{w}: class must be one of {CLASSES}")
        mw = s.get("mw_kda")
        if mw is not None and not (MW_PLAUSIBLE_KDA[0] <= mw <= MW_PLAUSIBLE_KDA[1]):
            problems.append(f"{w}: molecular weight {mw} kDa outside "
                            f"{MW_PLAUSIBLE_KDA[0]}-{MW_PLAUSIBLE_KDA[1]} kDa")
        if mw is None and "diffusion_um2_s" not in s:
            problems.append(f"{w}: needs mw_kda or diffusion_um2_s")
        if ("concentration_M" in s) == ("count" in s):
            problems.append(f"{w}: give exactly one of concentration_M and count")
        comp = _comp_index(s, kind, w, problems)
        if "concentration_M" in s:
            c = s["concentration_M"]
            n = count_from_concentration(c, vols[comp])
            if c < 0:
                problems.append(f"{w}: negative concentration")
            elif c > 0 and n < 1:
                problems.append(f"{w}: {c} M is less than one molecule in "
                                f"{vols[comp]:.4g} um^3; enlarge the volume")
        else:
            n = int(s.get("count", 0))
        if mw is not None and n > 0:
            excluded[comp] += n * 4.0 / 3.0 * math.pi * (radius_nm(mw) * 1e-3) ** 3
        for p in s.get("partners", []):
            if p not in names:
                problems.append(f"{w}: partner {p!r} is not defined")
            else:
                other = species[names.index(p)]
                if s.get("name") not in other.get("partners", [s.get("name")]):
                    problems.append(f"{w}: lists {p!r} as a partner but {p!r} does not list it")
    for c, v in excluded.items():
        if v > MAX_VOLUME_FRACTION * vols[c]:
            problems.append(f"compartment {c}: molecules fill {v / vols[c]:.0%} of its volume; "
                            f"the concentrations do not fit the volume")
    contact_pairs = set()
    uni_sum: Dict[Tuple[str, int], float] = {}
    for k, r in enumerate(doc.get("reactions", [])):
        w = f"reaction {k}"
        reac, prod = r.get("reactants", []), r.get("products", [])
        for n in list(reac) + [p for p in prod if p is not None]:
            if n not in names:
                problems.append(f"{w}: molecule {n!r} is not defined")
        has_p, has_k = "probability" in r, "kcat_per_s" in r
        if has_p == has_k:
            problems.append(f"{w}: give exactly one of probability and kcat_per_s")
        p = r.get("probability", 0.0)
        if has_k:
            p = kcat_probability(r["kcat_per_s"], doc["dt_s"])
        if not 0.0 <= p <= 1.0:
            problems.append(f"{w}: probability {p} outside [0, 1]")
        if len(reac) == 2:
            if not (r.get("radius_nm", 0) > 0):
                problems.append(f"{w}: a contact reaction needs radius_nm > 0")
            if len(prod) != 2:
                problems.append(f"{w}: a contact reaction has two products (null: consumed)")
            pair = tuple(sorted(reac))
            if pair in contact_pairs:
                problems.append(f"{w}: second contact reaction for {pair}")
            contact_pairs.add(pair)
        elif len(reac) == 1:
            pl = r.get("placement", "keep")
            if pl not in PLACEMENT:
                problems.append(f"{w}: placement must be one of {sorted(PLACEMENT)}")
            frm = r.get("from")
            key = (reac[0], COMPARTMENT.get(frm, -1) if frm else -1)
            uni_sum[key] = uni_sum.get(key, 0.0) + p
        else:
            problems.append(f"{w}: one or two reactants")
    for (n, c), p in uni_sum.items():
        if p > 1.0 + 1e-12:
            problems.append(f"first-order probabilities of {n!r} sum to {p} > 1")
    # a declared partnership needs a contact reaction
    for s in species:
        for p in s.get("partners", []):
            if p in names and tuple(sorted((s.get("name"), p))) not in contact_pairs:
                problems.append(f"species {s.get('name')!r}: partner {p!r} has no contact reaction")
    return problems


def load_model(src) -> Model:
    """A model from a JSON file path, JSON text or dict; raises ModelError
    listing every inconsistency."""
    if isinstance(src, dict):
        doc = src
    elif isinstance(src, str) and src.lstrip().startswith("{"):
        doc = json.loads(src)
    else:
        with open(src) as f:
            doc = json.load(f)
    problems = check_model(doc)
    if problems:
        raise ModelError(problems)
    geom = doc["geometry"]
    kind = geom["kind"]
    vols = compartment_volumes_um3(geom)
    T = doc.get("temperature_k", 310.15)
    eta = doc.get("viscosity_pa_s", WATER_37C_PA_S)
    idx = {s["name"]: i for i, s in enumerate(doc["species"])}
    species = []
    for s in doc["species"]:
        comp = COMPARTMENT.get(s.get("compartment", "cytosol"), 1) if kind == "nested" else 0
        D = s["diffusion_um2_s"] if "diffusion_um2_s" in s else stokes_einstein_um2_s(
            s["mw_kda"], T, eta)
        n = (count_from_concentration(s["concentration_M"], vols[comp])
             if "concentration_M" in s else int(s["count"]))
        species.append(Species(s["name"], float(D), n, comp))
    rules = []
    for r in doc.get("reactions", []):
        p = r["probability"] if "probability" in r else kcat_probability(r["kcat_per_s"], doc["dt_s"])
        prod = [idx[x] if x is not None else -1 for x in r.get("products", [])]
        prod = (prod + [-1, -1])[:2]
        if len(r["reactants"]) == 2:
            rules.append(Rule(BIMOL, (idx[r["reactants"][0]], idx[r["reactants"][1]]),
                              tuple(prod), float(p), radius_um=r["radius_nm"] * 1e-3))
        else:
            frm, to = r.get("from"), r.get("to")
            rules.append(Rule(UNIMOL, (idx[r["reactants"][0]], -1), tuple(prod), float(p),
                              placement=PLACEMENT[r.get("placement", "keep")],
                              release_radius_um=r.get("release_nm", 0.0) * 1e-3,
                              from_comp=COMPARTMENT[frm] if frm else -1,
                              to_comp=COMPARTMENT[to] if to else -1))
    n = sum(s.count for s in species)
    return Model(doc.get("name", "model"), GEOMETRY[kind], float(doc["dt_s"]),
                 int(doc.get("seed", 0)), species, rules,
                 box_um=float(geom.get("box_um", 0.0)),
                 outer_radius_um=float(geom.get("radius_um", 0.0)),
                 inner_radius_um=float(geom.get("inner_radius_um", 0.0)),
                 capacity=int(doc.get("capacity", max(n + n // 8, 64))),
                 cell_um=float(doc.get("cell_um", 0.0)), steps=int(doc.get("steps", 1)))


def concentration_molar(counts, volume_um3: float):
    """Counts to molar concentrations in a volume (c = N / (V N_A))."""
    return [c / (volume_um3 * 1e-15 * N_A) for c in counts]
