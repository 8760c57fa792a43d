"""Threshold monitoring of species concentrations over time.

The paper's simulator lets the user pick species to watch and give each a
concentration threshold within a time window, e.g. a phosphorylated kinase
that must not exceed its healthy plateau before a given time (Sec. 2); a
crossing flags aberrant signalling or a therapy that failed to restore it.

Here the counts over time come from the library's device counts ring
(``Sim.record_counts``), so watching costs no per-step host
synchronisation; ``check`` evaluates the thresholds on the recorded entries.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

N_A = 6.02214076e23


@dataclass
class Threshold:
    species: int                 # species index in the model
    above_M: Optional[float] = None   # flag a concentration above this (molar)
    below_M: Optional[float] = None   # flag a concentration below this (molar)
    from_s: float = 0.0          # window start (simulated seconds)
    to_s: float = float("inf")   # window end
    volume_um3: float = 1.0      # volume the species' count is measured in
    simulation: int = 0          # simulation index (batches)


@dataclass
class Crossing:
    threshold: Threshold
    step: int
    time_s: float
    concentration_M: float


def concentration(count, volume_um3: float):
    """Molar concentration of a count in a volume: N / (V N_A), V in litres."""
    return np.asarray(count, dtype=np.float64) / (volume_um3 * 1e-15 * N_A)


def check(steps: np.ndarray, counts: np.ndarray, dt_s: float,
          thresholds: Sequence[Threshold]) -> List[Crossing]:
    """First crossing of every threshold within its window, if any.
    ``steps`` and ``counts`` are ``Sim.ring()``'s output (counts shaped
    (entries, simulations, species))."""
    out = []
    t = np.asarray(steps, dtype=np.float64) * dt_s
    for th in thresholds:
        c = concentration(counts[:, th.simulation, th.species], th.volume_um3)
        inside = (t >= th.from_s) & (t <= th.to_s)
        bad = np.zeros_like(inside)
        if th.above_M is not None:
            bad |= c > th.above_M
        if th.below_M is not None:
            bad |= c < th.below_M
        hit = np.nonzero(inside & bad)[0]
        if len(hit):
            k = hit[0]
            out.append(Crossing(th, int(steps[k]), float(t[k]), float(c[k])))
    return out
