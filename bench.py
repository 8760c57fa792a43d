"""Benchmark: agent-updates/s of the molecule-agent step on one MI355X.

Workload: the 2M-agent MAPK-like cascade (8 species, 12 rules, reflecting
5 um sphere, dt = 1 us; workloads.c2), the configuration the headline metric
is quoted at.  A step is one pass of the whole step (event draw, Brownian
move, boundaries, binning, counting sort, neighbour scan + claim, rule
firing, compaction).  Agent state is resident in HBM before timing starts.

Prints one JSON line with the metric, the dominant kernel's roofline (kernel
durations from HIP events that each kernel's dispatch stamps at its start and
end, on the simulation's stream) and the CPU oracle's rate on a bounded
sample of the same workload.

Other workloads (--workload): c1 and c3 (agent-updates/s of the reversible
binding box and of the nested-compartment model), c4 (the dose x replicate
sweep as one tuned batch: simulations/s against one at a time, states
compared bit for bit), c5 (the serving loop: p50/p99 latency and requests/s,
concurrent against FIFO).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "agent-updates/s at 2M agents; batched sweep sims/s vs serial; p50/p99 latency"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# The paper publishes whole-run wall-clock times only (Sec. 3.2): about 10 h
# and 1.5 h for 8 h of simulated time at 3 pL and 0.3 pL, on an NVIDIA L4
# and one NVIDIA A100; no per-step rate and no time step.  Context only.
PAPER_CONTEXT = ("paper: no agent-updates/s published; 8 h of simulated time took ~10 h (3 pL, "
                 "~4.6M agents) and ~1.5 h (0.3 pL, ~0.46M agents) on NVIDIA L4 / A100, "
                 "i.e. ~2.4e6-3.6e6 agent x simulated-s per wall-s; its time step is not stated")

# Algorithmic bytes per launch of each step kernel: bytes per live agent (a),
# per claimer (q) and per cell of the spatial hash (c) that the kernel must
# read or write at least once for its function.  An agent is a 16-byte
# record {x, y, z, species|flags} plus a 4-byte id.
#   move:    reads record + id (20); writes record (16) and the agent's
#            rank in its cell (4)                                    = 40 B/agent
#            in a step that keeps the binning: the claimer byte (1)
#            instead of the rank                                     = 37 B/agent
#   scan:    reads the count, writes the start, clears the count     = 12 B/cell
#   scatter: reads rank, record, id, cell start (28); writes record, id,
#            claimer byte (21)                                       = 49 B/agent
#   propose: claimer byte of the chunk (1 B/agent); per claimer its
#            record and id (20), its proposal (4), and the search: the
#            start and end of its 8 stencil cells (64) and the record of
#            every agent in them (16 each; 8 h^3 x the density expected,
#            added at run time)                                      = 1 B/agent + 88 B/claimer
#                                                                      + 16 B/candidate
#   finish:  per proposer only (a few hundred per step): counted as 0
KERNEL_BYTES = {"move": (40, 0, 0), "scan": (0, 0, 12), "scatter": (49, 0, 0),
                "propose": (1, 88, 0), "finish": (0, 0, 0)}
MOVE_KEPT_BYTES = 37

# move is bound by vector-ALU issue, not by HBM: the arithmetic the step
# definition prescribes per agent (Philox4x32-10 block, event word and
# threshold, four uniforms, two logarithms, two square roots, two sin/cos
# evaluations, the displacement, the sphere test, the cell coordinates and
# their Morton interleave), counted as 32-bit operations (a 32x32->64 product
# = 2, a fused multiply-add = 2, a correctly rounded divide or square root =
# 1), is 323 per agent.
MOVE_OPS_PER_AGENT = 323
# a step that keeps the binning computes no cell coordinates (18) and no
# Morton key (43)
MOVE_OPS_KEPT = 323 - 18 - 43
# One 32-bit lane operation per clock per lane: 256 CUs x 64 lanes x 2.4 GHz
# (the 157.3 TFLOP/s fp32 figure counts an FMA as 2 and packed pairs as 2).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12

# HBM traffic of the step kernels per launch from rocprofv3 --pmc FETCH_SIZE
# and WRITE_SIZE (KiB per dispatch, averaged over 55 dispatches of
# "bench.py --steps 50 --warmup 5 --no-cpu-baseline --no-profile
# --copy-calib-mb 512"), scaled by what the same counters read for the
# 512 MiB device copy in that run (FETCH x2.0, WRITE x1.0).  Valid only for
# the kernel sources it was taken on (SHA-256 of the three files below).
TRAFFIC = {"fetch_scale": 2.0, "write_scale": 1.0,
           "sources_sha256": "42097d79359f869332d6888b7d7987146581af4f1135c3104f43067129259ec6",
           # kernel: (FETCH_SIZE KiB, WRITE_SIZE KiB) per dispatch
           "kib": {"move": (19629.7, 40071.2), "scan": (4631.8, 16416.1), "scatter": (34501.1, 56197.2), "propose": (17828.8, 2951.4), "finish": (152.5, 0.5)}}
KERNEL_SOURCES = ("paper_2606_14603_amd/csrc/kernels.hip",
                  "paper_2606_14603_amd/csrc/device_math.hpp",
                  "paper_2606_14603_amd/csrc/engine.hpp")


def kernel_sources_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """Calibrated HBM bytes per launch of the c2 step kernel, or None if
    there are no counters for it or they were taken on other sources."""
    t = TRAFFIC
    if kernel not in t["kib"] or t["sources_sha256"] != kernel_sources_sha():
        return None
    f, w = t["kib"][kernel]
    return int(1024 * (f * t["fetch_scale"] + w * t["write_scale"]))


def copy_ceiling_gbs(torch, mib: int = 1024, reps: int = 10) -> float:
    """Achieved read+write GB/s of a plain device-to-device copy."""
    src = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * (mib << 20) / (ms * 1e-3) / 1e9


def volume_um3(model) -> float:
    if model.geometry == 0:
        return model.box_um ** 3
    return 4.0 / 3.0 * 3.141592653589793 * model.outer_radius_um ** 3


def describe(model) -> str:
    geo = {0: f"periodic box {model.box_um:g} um", 1: f"reflecting sphere R={model.outer_radius_um:.3f} um",
           2: f"nested spheres R_in={model.inner_radius_um:.3f} um, R_out={model.outer_radius_um:.3f} um"}
    return (f"{model.name}: {model.n_agents} agents, {len(model.species)} species, "
            f"{len(model.rules)} rules, {geo[model.geometry]}, dt={model.dt_s * 1e6:g} us")


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


def _bits(e: dict) -> dict:
    return {k: (v.view("uint32") if v.dtype.kind == "f" else v) for k, v in e.items()}


def run_sweep(args, torch, mabm, W) -> dict:
    """The dose x replicate sweep: every simulation for its whole horizon,
    once as one batch (its cell density and launch shape chosen by the
    batch tuner beforehand, unless --no-tune) and once one at a time
    through the single-simulation path (a sample of simulations at their
    default grids, extrapolated), with the sampled simulations' final states
    compared bit for bit."""
    models = W.c4_sweep(n_reps=args.sweep_reps, steps=args.sweep_steps)
    n, steps = len(models), args.sweep_steps
    tuned, serial_models = None, models
    if not args.no_tune:
        # the batch's cell density and launch shape, timed on the batch
        # itself (results do not depend on them); the serial sample keeps
        # each simulation's default grid, the faster one for a lone run
        from paper_2606_14603_amd import tune
        tuned = tune.tune_batch(models)
        models = tuned.models(models)
    agents = sum(m.n_agents for m in models)
    # warm the code objects on a small batch first
    warm = mabm.Batch(models[:2])
    warm.step(3)
    warm.counts()
    del warm
    # each step of the batch is replayed from a captured graph
    batch = mabm.Batch(models, graphs=True)
    if tuned is not None:
        tuned.apply(batch)
    batch.grid()  # finalize: tables, placement
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    u0 = batch.agent_updates()
    e0.record(batch.stream)
    batch.step(steps)
    e1.record(batch.stream)
    torch.cuda.synchronize()
    ms_batch = e0.elapsed_time(e1)
    updates = batch.agent_updates() - u0
    sample = list(range(0, n, max(1, n // args.sweep_sample)))[:args.sweep_sample]
    ms_serial, same = 0.0, True
    for k in sample:
        sim = mabm.Sim(serial_models[k], graphs=True)
        sim.grid()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(sim.stream)
        sim.step(steps)
        b.record(sim.stream)
        torch.cuda.synchronize()
        ms_serial += a.elapsed_time(b)
        ge, be = _bits(sim.export()), _bits(batch.export(k))
        for f in ("id", "species", "x", "y", "z"):
            same = same and bool((ge[f] == be[f]).all()) and len(ge[f]) == len(be[f])
        sim.close()
    ms_serial_all = ms_serial * n / len(sample)
    value = n / (ms_batch * 1e-3)
    serial = n / (ms_serial_all * 1e-3)
    return {
        "metric": METRIC, "value": value, "unit": "sims/s", "n_gpus": 1, "steps": steps,
        "warmup": 0, "ms_per_step": ms_batch / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"c4_sweep: {len(models) // args.sweep_reps} doses x "
                               f"{args.sweep_reps} replicates of c2_mapk, 20k-200k agents each, "
                               f"{steps} steps", "sims": n, "agents": agents,
                   "tuned": None if tuned is None else {
                       "agents_per_cell": tuned.agents_per_cell, "lanes": tuned.lanes,
                       "min_workgroups": tuned.min_workgroups,
                       "ms_per_step": {k: round(v, 4) for k, v in tuned.ms_per_step.items()}}},
        "batched": {"ms": ms_batch, "agent_updates_per_s": updates / (ms_batch * 1e-3)},
        "serial": {"value": serial, "unit": "sims/s", "ms_extrapolated": ms_serial_all,
                   "sample": f"{len(sample)} of {n} simulations run one at a time, "
                             f"{ms_serial:.1f} ms, scaled by {n}/{len(sample)}"},
        "speedup_vs_serial": value / serial,
        "bit_identical_sample": same,
    }


def run_serving(args, torch, mabm, W) -> dict:
    """The request stream: each request a model of its own (a random closed
    subset of the cascade's rules, 50k-1M agents, 200-2000 steps).  The
    FIFO server (one request at a time) is first run on all requests
    arriving at once to measure its capacity; Poisson arrivals at 0.7 x that
    rate are then served FIFO and by the concurrent server, which keeps
    every admitted simulation resident and advances them on streams of their
    own.  Admission: arrival order, while the summed arenas fit the budget."""
    from paper_2606_14603_amd import serve

    def progress(r):  # one line per completed request, on stderr
        print(f"[serve] {r.name} done at {r.completed_s:.2f} s ({r.agents} agents, {r.steps} steps)",
              file=sys.stderr, flush=True)

    models = W.c5_requests(args.serve_requests, seed=0, n_max=args.serve_max_agents,
                           h_min=args.serve_min_steps, h_max=args.serve_max_steps)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.85 * free) if args.serve_budget_gb <= 0 else int(args.serve_budget_gb * 2**30)
    # load the code objects and the graph path once
    serve.Server(budget, max_active=2).run(W.c5_requests(2, seed=99, n_max=60_000, h_max=300),
                                           [0.0, 0.0])
    fifo = serve.Server(budget, max_active=1, chunk=args.serve_chunk, progress=progress)
    cap = serve.summarize(fifo.run(models, np.zeros(len(models))))
    rate = 0.7 * cap["sims_per_s"]
    arrivals = W.poisson_arrivals(len(models), rate, seed=0)
    res_fifo = fifo.run(models, arrivals)
    conc = serve.Server(budget, max_active=args.serve_active, chunk=args.serve_chunk,
                        progress=progress, fill_agents=args.serve_fill_agents)
    cap_conc = serve.summarize(conc.run(models, np.zeros(len(models))))
    res_conc = conc.run(models, arrivals)
    s_fifo, s_conc = serve.summarize(res_fifo), serve.summarize(res_conc)
    by_name = {r.name: r.counts for r in res_fifo}
    same = all(np.array_equal(by_name[r.name], r.counts) for r in res_conc)
    return {
        "metric": METRIC, "value": s_conc["sims_per_s"], "unit": "sims/s", "n_gpus": 1,
        "steps": int(sum(m.steps for m in models)), "warmup": 2,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"c5_requests: {len(models)} requests, random closed subsets of "
                               f"the cascade's rules, 50k-{args.serve_max_agents // 1000}k agents, "
                               f"{args.serve_min_steps}-{args.serve_max_steps} steps, Poisson "
                               f"arrivals at 0.7 x the FIFO capacity",
                   "arrival_rate_per_s": rate, "budget_bytes": budget,
                   "chunk_steps": args.serve_chunk, "max_active": args.serve_active,
                   "fill_agents": args.serve_fill_agents},
        "p50_s": s_conc["p50_s"], "p99_s": s_conc["p99_s"],
        "concurrent": s_conc, "fifo": s_fifo, "fifo_capacity": cap,
        "concurrent_capacity": cap_conc,
        "capacity_ratio": cap_conc["sims_per_s"] / cap["sims_per_s"],
        "identical_results": same,
    }


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
    ap.add_argument("--tune", action="store_true",
                    help="c2/c1/c3: time candidate cell sizes first and run with the fastest")
    ap.add_argument("--no-tune", action="store_true",
                    help="c4: skip the batch tuner (cell density, launch shape) and use the "
                         "default grids")
    ap.add_argument("--workload", choices=("c1", "c2", "c3", "c4", "c5"), default="c2",
                    help="c2: the 2M-agent cascade step (agent-updates/s, the headline); "
                         "c1: A+B<->C, 20k agents in a periodic box; c3: nested "
                         "compartments, 5M agents, births; c4: the batched dose x replicate "
                         "sweep (sims/s vs serial); c5: the serving loop (p50/p99 latency, "
                         "sims/s vs FIFO)")
    ap.add_argument("--serve-requests", type=int, default=256, help="c5: requests")
    ap.add_argument("--serve-chunk", type=int, default=256, help="c5: steps per turn")
    ap.add_argument("--serve-fill-agents", type=int, default=4_000_000,
                    help="c5: the concurrent server admits no more while its simulations "
                         "hold this many agents")
    ap.add_argument("--serve-max-agents", type=int, default=1_000_000,
                    help="c5: largest request (log-uniform from 50k)")
    ap.add_argument("--serve-min-steps", type=int, default=200, help="c5: shortest horizon")
    ap.add_argument("--serve-max-steps", type=int, default=2000, help="c5: longest horizon")
    ap.add_argument("--serve-active", type=int, default=64, help="c5: simulations admitted at once")
    ap.add_argument("--serve-budget-gb", type=float, default=0.0,
                    help="c5: HBM budget for admitted arenas (0: 85%% of free memory)")
    ap.add_argument("--sweep-reps", type=int, default=64, help="c4: replicates per dose")
    ap.add_argument("--sweep-steps", type=int, default=2000, help="c4: steps per simulation")
    ap.add_argument("--sweep-sample", type=int, default=16,
                    help="c4: simulations run one at a time for the serial baseline")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="first run 4 plain device copies of this many MiB (untimed), so a "
                         "counter profile of this command holds a copy kernel of known bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        return 2

    import torch
    import paper_2606_14603_amd as mabm
    import workloads as W

    torch.cuda.set_device(0)
    if args.workload == "c4":
        print(json.dumps(run_sweep(args, torch, mabm, W)), flush=True)
        return 0
    if args.workload == "c5":
        print(json.dumps(run_serving(args, torch, mabm, W)), flush=True)
        return 0
    if args.workload == "c1":
        model = W.c1()
    elif args.workload == "c3":
        model = W.c3(args.agents if args.agents != 2_000_000 else 5_000_000)
    else:
        model = W.c2(args.agents)
    if args.copy_calib_mb:
        src = torch.ones(args.copy_calib_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tuned = None
    if args.tune:
        from paper_2606_14603_amd import tune
        tr = tune.tune_cell(model)
        args.cell_um = tr.cell_um
        tuned = {f"{h:.5f}": round(ms, 4) for h, ms in tr.ms_per_step.items()}
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
    claim_sp = sorted({r.reactants[0] for r in model.rules if r.kind == W.BIMOL})
    claimers = int(counts[claim_sp].sum())

    # the same number of steps again, each kernel's dispatch stamping HIP
    # events at its start and end (direct launches), for per-kernel durations
    roof, kernels, ms_direct = None, {}, None
    if not args.no_profile:
        sim.profile(True)
        ms_direct, _ = timed(args.steps)
        prof = sim.profile_read()
        sim.profile(False)
        bin_launches = prof["scan"][0]
        for name, (launches, tot) in prof.items():
            if launches:
                a, q, c = KERNEL_BYTES[name]
                if name == "move":  # mean over binning and kept steps
                    a = (a * bin_launches + MOVE_KEPT_BYTES * (launches - bin_launches)) / launches
                alg = a * live + q * claimers + c * G ** 3
                if name == "propose":  # candidates: 8 cells at the mean density
                    alg += 16 * claimers * 8 * h ** 3 * live / volume_um3(model)
                us = 1e3 * tot / launches
                kernels[name] = {"launches": launches, "avg_us": round(us, 3),
                                 "alg_bytes": int(alg), "alg_gbs": round(alg / us / 1e3, 1)}
                tb = measured_traffic(name) if args.workload == "c2" and args.agents == 2_000_000 else None
                if tb is not None:
                    kernels[name]["traffic_bytes"] = tb
                    kernels[name]["traffic_gbs"] = round(tb / us / 1e3, 1)
                    kernels[name]["traffic_hbm_frac"] = round(tb / us / 1e3 / HBM_PEAK_GBS, 4)
        dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
        us = kernels[dom]["avg_us"]
        if dom == "move":
            mv = kernels["move"]["launches"]
            ops = live * (MOVE_OPS_PER_AGENT * bin_launches + MOVE_OPS_KEPT * (mv - bin_launches)) / mv
            achieved = ops / (us * 1e-6) / 1e12
            roof = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 2),
                    "peak": round(VALU_PEAK_TOPS, 2), "unit": "Tops/s",
                    "frac": round(achieved / VALU_PEAK_TOPS, 4),
                    "alg_ops_per_launch": int(ops)}
        else:
            achieved = kernels[dom]["alg_gbs"]
            roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4)}
        roof["traffic"] = kernels[dom].get("traffic_bytes")
        roof["alg_bytes_per_launch"] = kernels[dom]["alg_bytes"]
        roof["hbm_frac_alg_bytes"] = round(kernels[dom]["alg_gbs"] / HBM_PEAK_GBS, 4)
        # per step: each kernel's bytes per launch times its launches per step
        step_bytes = sum(k["alg_bytes"] * k["launches"] for k in kernels.values()) / args.steps
        roof["step_alg_bytes_per_update"] = round(step_bytes / live, 1)
        roof["step_alg_gbs"] = round(step_bytes * args.steps / (ms * 1e-3) / 1e9, 1)
        # the whole step against the HBM roofline of its algorithmic bytes
        roof["step_hbm_roofline_updates_per_s"] = round(HBM_PEAK_GBS * 1e9 / (step_bytes / live), -6)
        roof["step_hbm_frac"] = round(value / roof["step_hbm_roofline_updates_per_s"], 4)
        roof["copy_ceiling_gbs"] = round(copy_ceiling_gbs(torch), 1)
    out = {
        "metric": METRIC, "value": value, "unit": "agent-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": describe(model),
                   "agents": model.n_agents, "grid": G, "cell_um": round(h, 5),
                   "graphs": args.graph, "bin_every": sim.get_param(mabm.PARAM_BIN_EVERY),
                   "final_step": t, "tuned_ms_per_step": tuned,
                   "live_agents_end": int(counts.sum())},
        "roofline": roof, "kernels": kernels,
        "ms_per_step_kernel_timed": None if ms_direct is None else ms_direct / args.steps,
    }
    out["paper_context"] = PAPER_CONTEXT
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(model)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
