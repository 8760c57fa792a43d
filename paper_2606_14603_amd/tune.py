"""Cell-size autotuner.

The spatial hash's cell size h is a pure performance choice: the step's
results do not depend on it (only the exported cell ids do).  Coarse cells
make the counting sort cheap and the neighbour search long (more candidates
per stencil cell); fine cells the reverse; the 8-cell stencil needs
h >= 2.02 x the largest contact radius, finer cells the 27-cell one.  The
tuner times a few steps of the model at each candidate grid, from the same
initial state, and keeps the fastest; results are cached per (geometry,
agents, density, largest contact radius), so models of one shape are tuned
once.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass
from typing import Dict, List, Optional

from . import Sim

_CACHE: Dict[str, float] = {}


def _extent(m) -> float:
    return m.box_um if m.geometry == 0 else 2.0 * m.outer_radius_um


def _volume(m) -> float:
    if m.geometry == 0:
        return m.box_um ** 3
    return 4.0 / 3.0 * math.pi * m.outer_radius_um ** 3


def _rmax(m) -> float:
    r = [x.radius_um for x in m.rules if x.kind == 0]
    return max(r) if r else 0.0


def shape_key(m) -> str:
    """Models of one shape share a tuned cell size: geometry, agents and
    density to the nearest power of 2^(1/2), largest contact radius in nm."""
    n = max(1, m.n_agents)
    dens = n / _volume(m)
    return (f"g{m.geometry}:n{round(2 * math.log2(n))}:d{round(2 * math.log2(dens))}:"
            f"r{round(_rmax(m) * 1e3, 2)}")


def candidates(m) -> List[float]:
    """Cell sizes to try: power-of-two grids around one cell per agent, and
    the finest cell the 8-cell stencil allows."""
    ext, rmax = _extent(m), _rmax(m)
    g0 = 2 ** round(math.log2(max(3.0, (max(1, m.capacity)) ** (1.0 / 3.0))))
    grids = {max(3, g0 // 4), max(3, g0 // 2), g0, min(512, 2 * g0)}
    if rmax > 0:
        grids.add(max(3, min(512, int(ext / (2.02 * rmax)))))
    out = []
    for g in sorted(grids):
        h = ext / g
        if rmax > 0 and h < 1.01 * rmax:
            continue
        out.append(h * (1.0 - 1e-6))  # the library takes floor(ext / h) cells
    return out


@dataclass
class TuneResult:
    cell_um: float
    ms_per_step: Dict[float, float]
    cached: bool = False


def tune_cell(model, steps: int = 20, warm: int = 5, cache_path: Optional[str] = None) -> TuneResult:
    """Fastest cell size for ``model`` among ``candidates`` (ms per step
    measured with HIP events on each candidate's stream)."""
    import torch
    key = shape_key(model)
    if cache_path and not _CACHE and os.path.exists(cache_path):
        with open(cache_path) as f:
            _CACHE.update(json.load(f))
    if key in _CACHE:
        return TuneResult(_CACHE[key], {}, cached=True)
    timings = {}
    for h in candidates(model):
        sim = Sim(model, cell_um=h)
        sim.step(warm)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        sim.step(steps)
        e1.record(sim.stream)
        torch.cuda.synchronize()
        timings[h] = e0.elapsed_time(e1) / steps
        sim.close()
    best = min(timings, key=timings.get)
    _CACHE[key] = best
    if cache_path:
        with open(cache_path, "w") as f:
            json.dump(_CACHE, f, indent=1, sort_keys=True)
    return TuneResult(best, timings)
