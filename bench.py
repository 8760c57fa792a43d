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

# Algorithmic bytes per launch of each step kernel: bytes per live agent (a),
# per claimer (q) and per cell of the spatial hash (c) that the kernel must
# read or write at least once for its function.  An agent is a 16-byte
# record {x, y, z, species|flags} plus a 4-byte id.
#   move:    reads record + id (20); writes record (16) and the (cell key,
#            rank) pair (8)                                          = 44 B/agent
#   scan:    reads the count, writes the start, clears the count     = 12 B/cell
#   scatter: reads (key, rank), record, id, cell start (32); writes
#            record, id, claimer byte (21)                           = 53 B/agent
#   propose: claimer byte of the chunk (1 B/agent); per claimer its
#            record and id (20) and its proposal (4)                 = 1 B/agent + 24 B/claimer
#   finish:  per proposer only (a few hundred per step): counted as 0
KERNEL_BYTES = {"move": (44, 0, 0), "scan": (0, 0, 12), "scatter": (53, 0, 0),
                "propose": (1, 24, 0), "finish": (0, 0, 0)}


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
                    help="skip the per-kernel timing region (no roofline)")
    ap.add_argument("--graph", action="store_true",
                    help="replay each step as a captured HIP graph (default: direct launches)")
    ap.add_argument("--cell-um", type=float, default=0.0,
                    help="spatial-hash cell size (0: the library's choice)")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="first run 4 plain device copies of this many MiB (untimed), so a "
                         "counter profile of this command holds a copy kernel of known bytes")
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
    if args.copy_calib_mb:
        src = torch.ones(args.copy_calib_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    sim = mabm.Sim(model, graphs=args.graph, cell_um=args.cell_um)
    G, h = sim.grid()
    stream = sim.stream
    sim.step(args.warmup)
    sim.counts()  # synchronises; surfaces any device error

    def timed(steps: int):
        u0 = sim.agent_updates()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        sim.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1), sim.agent_updates() - u0

    # timed region: the step as users run it
    ms, updates = timed(args.steps)
    value = updates / (ms / 1e3)
    live = updates / args.steps
    counts, t = sim.counts()
    claimers = int(counts[[0, 3, 6]].sum())  # kinase1, p-kinase2, phosphatase claim

    # same number of steps with HIP events around every kernel (direct
    # launches: events cannot sit between graph nodes) for the roofline
    roof, kernels, ms_direct = None, {}, None
    if not args.no_profile:
        sim.profile(True)
        ms_direct, _ = timed(args.steps)
        prof = sim.profile_read()
        sim.profile(False)
        for name, (launches, tot) in prof.items():
            if launches:
                kernels[name] = {"launches": launches, "avg_us": round(1e3 * tot / launches, 3)}
        dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
        a, q, c = KERNEL_BYTES[dom]
        alg = a * live + q * claimers + c * G ** 3
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
                   "graphs": args.graph, "final_step": t,
                   "live_agents_end": int(counts.sum())},
        "roofline": roof, "kernels": kernels,
        "ms_per_step_kernel_timed": None if ms_direct is None else ms_direct / args.steps,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(model)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
