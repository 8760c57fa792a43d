"""Cell-size and launch-shape autotuner, for one simulation (tune_cell) and
for a batch (tune_batch).

The spatial hash's cell size h is a pure performance choice: the step's
results do not depend on it (only the exported cell ids do).  Coarse cells
make the counting sort cheap and the neighbour search long (more candidates
per stencil cell); fine cells the reverse; the 8-cell stencil needs
h >= 2.02 x the largest contact radius, finer cells the 27-cell one.  The
tuner times a few steps of the model at each candidate grid, from the same
initial state, and keeps the fastest; results are cached per (geometry,
agents, density, largest contact radius), so models of one shape are tuned
once.

At the chosen cell size the tuner then times the neighbour search's launch
shape, also a pure performance choice: lanes per claimer (each lane scans at
most two stencil cells, so more lanes mean shorter, more parallel searches
and fewer claimers per wave) and the fewest workgroups the search launches
(chunks of sorted agents shared by more workgroups fill the chip at small
agent counts, at the price of re-reading the chunk's claim flags).
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

from . import Sim

_CACHE: Dict[str, dict] = {}


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
    from . import MAX_GRID
    grids = {max(3, g0 // 4), max(3, g0 // 2), g0, min(MAX_GRID, 2 * g0)}
    if rmax > 0:
        grids.add(max(3, min(MAX_GRID, int(ext / (2.02 * rmax)))))
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
    lanes: int = 0              # 0: the library's choice
    min_workgroups: int = 0     # 0: the library's choice
    ms_per_shape: Dict[Tuple[int, int], float] = field(default_factory=dict)
    mode: int = 0               # search mode (0: the library's choice)
    ms_per_mode: Dict[int, float] = field(default_factory=dict)

    def apply(self, sim) -> None:
        """Set the tuned launch shape and search mode on a simulation built
        at ``cell_um``."""
        from . import PARAM_PROPOSE_LANES, PARAM_PROPOSE_MIN_WORKGROUPS, PARAM_PROPOSE_MODE
        sim.set_param(PARAM_PROPOSE_LANES, self.lanes)
        sim.set_param(PARAM_PROPOSE_MIN_WORKGROUPS, self.min_workgroups)
        sim.set_param(PARAM_PROPOSE_MODE, self.mode)


def shapes(cell_um: float, model) -> List[Tuple[int, int]]:
    """Launch shapes to try: the default, twice the default lanes, and
    fewer or more workgroups."""
    ext, rmax = _extent(model), _rmax(model)
    g = int(ext / cell_um)
    stencil8 = rmax > 0 and ext / g >= 2.02 * rmax
    lanes = 4 if stencil8 else 16
    return [(0, 0), (2 * lanes, 0), (0, 512), (0, 8192)]


def _time(model, cell_um: float, shape: Tuple[int, int], steps: int, warm: int,
          mode: int = 0) -> float:
    import torch
    from . import PARAM_PROPOSE_LANES, PARAM_PROPOSE_MIN_WORKGROUPS, PARAM_PROPOSE_MODE
    sim = Sim(model, cell_um=cell_um)
    sim.set_param(PARAM_PROPOSE_LANES, shape[0])
    sim.set_param(PARAM_PROPOSE_MIN_WORKGROUPS, shape[1])
    sim.set_param(PARAM_PROPOSE_MODE, mode)
    sim.step(warm)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    sim.close()
    return e0.elapsed_time(e1) / steps


def tune_cell(model, steps: int = 20, warm: int = 5, cache_path: Optional[str] = None,
              launch_shape: bool = True) -> TuneResult:
    """Fastest cell size for ``model`` among ``candidates``, then (with
    ``launch_shape``) the fastest neighbour-search launch shape among
    ``shapes`` at that cell size, then the faster search mode (per chunk
    or over the claimer list) at that shape; ms per step measured with HIP
    events on each trial's stream."""
    key = shape_key(model)
    if cache_path and not _CACHE and os.path.exists(cache_path):
        with open(cache_path) as f:
            _CACHE.update(json.load(f))
    if key in _CACHE:
        c = _CACHE[key]
        if isinstance(c, dict):
            return TuneResult(c["cell_um"], {}, True, c.get("lanes", 0), c.get("min_workgroups", 0),
                              mode=c.get("mode", 0))
        return TuneResult(float(c), {}, cached=True)
    timings = {h: _time(model, h, (0, 0), steps, warm) for h in candidates(model)}
    best = min(timings, key=timings.get)
    per_shape = {(0, 0): timings[best]}
    per_mode: Dict[int, float] = {}
    mode = 0
    if launch_shape:
        for sh in shapes(best, model)[1:]:
            per_shape[sh] = _time(model, best, sh, steps, warm)
    lanes, minwg = min(per_shape, key=per_shape.get)
    if launch_shape and any(r.kind == 0 for r in model.rules):
        # both searches at the chosen shape (the list ignores the shape)
        per_mode = {m: _time(model, best, (lanes, minwg), steps, warm, m) for m in (1, 2)}
        mode = min(per_mode, key=per_mode.get)
    _CACHE[key] = {"cell_um": best, "lanes": lanes, "min_workgroups": minwg, "mode": mode}
    if cache_path:
        with open(cache_path, "w") as f:
            json.dump(_CACHE, f, indent=1, sort_keys=True)
    return TuneResult(best, timings, False, lanes, minwg, per_shape, mode, per_mode)


@dataclass
class BatchTuneResult:
    agents_per_cell: float      # 0: the library's default grid for every simulation
    lanes: int = 0
    min_workgroups: int = 0
    ms_per_step: Dict[str, float] = field(default_factory=dict)

    def models(self, models):
        """``models`` with the tuned cell size set on each."""
        return [m.with_(cell_um=batch_cell(m, self.agents_per_cell)) for m in models]

    def apply(self, batch) -> None:
        from . import PARAM_PROPOSE_LANES, PARAM_PROPOSE_MIN_WORKGROUPS
        batch.set_param(PARAM_PROPOSE_LANES, self.lanes)
        batch.set_param(PARAM_PROPOSE_MIN_WORKGROUPS, self.min_workgroups)


def batch_cell(m, agents_per_cell: float) -> float:
    """Cell size giving about ``agents_per_cell`` agents per cell over the
    simulation's volume (0: the library's default), kept at or above the
    largest contact radius and within the largest grid."""
    if agents_per_cell <= 0 or m.n_agents == 0:
        return 0.0
    h = (_volume(m) * agents_per_cell / m.n_agents) ** (1.0 / 3.0)
    from . import MAX_GRID
    h = max(h, 1.01 * _rmax(m), _extent(m) / MAX_GRID)
    return h * (1.0 + 1e-6)


def _time_batch(models, agents_per_cell: float, shape: Tuple[int, int], steps: int,
                warm: int) -> float:
    import torch
    from . import Batch, PARAM_PROPOSE_LANES, PARAM_PROPOSE_MIN_WORKGROUPS
    b = Batch([m.with_(cell_um=batch_cell(m, agents_per_cell)) for m in models], graphs=True)
    b.set_param(PARAM_PROPOSE_LANES, shape[0])
    b.set_param(PARAM_PROPOSE_MIN_WORKGROUPS, shape[1])
    b.step(warm)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    b.close()
    return e0.elapsed_time(e1) / steps


def tune_batch(models, steps: int = 32, warm: int = 16) -> BatchTuneResult:
    """Cell density and neighbour-search launch shape for a batch, timed on
    the batch itself: every simulation at about 0.5, 1, 2, 4 or 8 agents
    per cell, or at the library's default grids, then the launch shapes of
    ``shapes`` at the fastest.  Results do not depend on either."""
    timings = {a: _time_batch(models, a, (0, 0), steps, warm)
               for a in (0.0, 0.5, 1.0, 2.0, 4.0, 8.0)}
    best = min(timings, key=timings.get)
    per = {f"cells:{a}": t for a, t in timings.items()}
    shape_t = {(0, 0): timings[best]}
    for sh in [(8, 0), (0, 512), (0, 8192)]:
        shape_t[sh] = _time_batch(models, best, sh, steps, warm)
        per[f"shape:{sh[0]},{sh[1]}"] = shape_t[sh]
    lanes, minwg = min(shape_t, key=shape_t.get)
    return BatchTuneResult(best, lanes, minwg, per)
