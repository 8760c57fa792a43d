"""Benchmark: agent-updates/s of the molecule-agent step on one MI355X.

Workload: the 2M-agent MAPK-like cascade (8 species, 12 rules, reflecting
5 um sphere, dt = 1 us; workloads.c2), the configuration the headline metric
is quoted at.  A step is one pass of the whole step (event draw, Brownian
move, boundaries, binning, counting sort, neighbour scan + claim, rule
firing, compaction).  Agent state is resident in HBM before timing starts.

Prints one JSON line with the metric, the dominant kernel's roofline (HIP
events on the simulation's stream over the timed region) and the CPU
oracle's rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "agent-updates/s at 2M agents; batched sweep sims/s vs serial; p50/p99 latency"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

# Algorithmic bytes per launch of each step kernel, as bytes per live agent
# (a) and per cell of the spatial hash (c): what the kernel must read or
# write at least once for its function.
#   move:    reads x, y, z, id, species (17 B); writes x, y, z, species (13),
#            cell key (4), in-cell rank (4), busy flag (1)           = 39 B
#   scatter: reads key, rank, 17 B state, flag, cell start (30); writes
#            17 B state, flag, claim slot (26)                       = 56 B
#   propose: reads species + flag (2), writes proposal (4); claimers' own
#            positions and cell starts are a small extra             = 6 B
#   apply:   reads the proposal                                      = 4 B
#   scan_reduce: 4 B per cell; scan_down: 12 B per cell (read, start, clear)
KERNEL_BYTES = {
    "move": (39, 0), "scatter": (56, 0), "propose": (6, 0), "apply": (4, 0),
    "scan_reduce": (0, 4), "scan_down": (0, 12), "scan_top": (0, 0), "births": (0, 0),
}


def cpu_baseline(model, budget_s: float = 12.0, max_steps: int = 40) -> dict:
    import oracle
    o = oracle.OracleSim(model)
    n0, _ = o.size()
    updates, steps, t0 = 0, 0, time.perf_counter()
    while steps < max_steps and (time.perf_counter() - t0) < budget_s:
        n, _ = o.size()
        o.step(1)
        updates += n
        steps += 1
    dt = time.perf_counter() - t0
    return {"value": updates / dt, "unit": "agent-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{model.name}, {n0} agents, first {steps} steps, single-threaded C oracle"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--agents", type=int, default=2_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="time without per-kernel events (no roofline)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        return 2

    import torch
    import paper_2606_14603_amd as mabm
    import workloads as W

    model = W.c2(args.agents)
    torch.cuda.set_device(0)
    sim = mabm.Sim(model)
    G, h = sim.grid()
    sim.step(args.warmup)
    sim.counts()  # sync; surfaces any device error
    u0 = sim.agent_updates()
    if not args.no_profile:
        sim.profile(True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = sim.stream
    ev0.record(stream)
    sim.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    prof = sim.profile_read() if not args.no_profile else {}
    u1 = sim.agent_updates()
    counts, t = sim.counts()
    updates = u1 - u0
    value = updates / (ms / 1e3)
    live = updates / args.steps
    ncells = G ** 3

    roof = None
    kernels = {}
    if prof:
        for name, (launches, tot) in prof.items():
            if launches:
                kernels[name] = {"launches": launches, "avg_us": 1e3 * tot / launches}
        dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
        a, c = KERNEL_BYTES[dom]
        alg = a * live + c * ncells
        achieved = alg / (kernels[dom]["avg_us"] * 1e-6) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "alg_bytes_per_launch": int(alg)}
    out = {
        "metric": METRIC, "value": value, "unit": "agent-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"c2_mapk: {model.n_agents} agents, 8 species, 12 rules, "
                               f"reflecting sphere R={model.outer_radius_um:.3f} um, dt=1 us",
                   "agents": model.n_agents, "grid": G, "cell_um": round(h, 5),
                   "final_step": t, "live_agents_end": int(counts.sum())},
        "roofline": roof, "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(model)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
