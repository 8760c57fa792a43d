"""Benchmark of the molecule-agent step on one MI355X.

Headline: agent-updates/s of the 2M-agent MAPK-like cascade (8 species, 12
rules, reflecting 5 um sphere, dt = 1 us; workloads.c2), the configuration
the metric is quoted at.  A step is one pass of the whole step (event draw,
Brownian move, boundaries, binning, counting sort, neighbour scan + claim,
rule firing, compaction).  Agent state is resident in HBM before timing
starts.  The line carries the dominant kernel's roofline (kernel durations
from HIP events that each kernel's dispatch stamps at its start and end, on
the simulation's stream) and the CPU oracle's rate on a bounded sample of
the same workload.

The default line also carries the other two parts of the metric and more
samples of the step:
  late_run  the same simulation's rate from step 2,000 (its steps 5..25 are
            the headline's);
  c3        the 5M-agent nested-compartment model with births, early
            (steps 50..250) and late (from step 2,000);
  c4        the dose x replicate sweep (1,024 simulations, 20k-200k agents,
            2,000 steps) as one batch (cell density and launch shape chosen
            by the batch tuner first, unless --no-tune) against every
            simulation run alone: simulations/s, and each simulation's final
            state compared by the library's state digest;
  c5        the serving stream at its stated ranges (sizes 50k-4M agents,
            horizons 1,000-20,000 steps, Poisson arrivals): p50/p99 latency
            and simulations/s, concurrent against FIFO, final states
            compared by digest.
--only-c2 drops c3, c4 and c5; --workload c1|c3|c4|c5 runs one of them
alone.
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

# Algorithmic bytes per launch of each step kernel, on this library's agent
# layout: bytes per live agent (a), per claimer (q) and per cell of the
# spatial hash (c) that the kernel must read or write at least once for its
# function.  An agent is a 16-byte record {x, y, z, species|flags} plus a
# 4-byte id.
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
# Algorithmic bytes independent of this library's layout:
# 17 B of agent state per agent (three float positions, a 4-byte id, a
# species byte); move reads it and writes it once (34 B per agent), and a
# whole step moves 70 B per agent-update (state read and written, cell key
# written and read, permutation, claim slot reset and confirm, cell tables
# at about one cell per agent).
STATE_MOVE_BYTES = 34
STATE_STEP_BYTES = 70

# move is bound by vector-ALU issue, not by HBM.  Its algorithmic work is
# the arithmetic the step definition prescribes per agent, each 32-bit
# lane operation counted once (a fused multiply-add once, a 32x32->64
# product once, a correctly rounded divide or square root once):
#   Philox4x32-10 block: 10 rounds x (2 products, 4 xor, 2 key adds)    80
#   event word (4 and, 3 shift, 3 or) and one threshold compare          11
#   four uniforms (shift, [add,] convert, multiply)                      14
#   two logarithms (exponent and mantissa split, fold, m -/+ 1, divide,
#     s^2, 4-term Horner, scaling, e ln 2 in two fused terms)            42
#   two radii (-2 log, square root)                                       4
#   two sin/cos of 2 pi u (quadrant, fold, two series, quadrant selects
#     and sign flips)                                                     60
#   three normals and the displacement (3 multiplies, 3 FMA)             6
#   sphere test (|p'|^2, compare, three selects)                         9
#   binning steps only: cell coordinates (3 x subtract, multiply, floor,
#     two clamps, convert) and the Morton interleave (3 x 13, combine 4)  61
MOVE_OPS_BIN = 287
MOVE_OPS_KEPT = 226
# One lane operation per lane per clock: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz = 39.3 T lane-operations/s.  (The published 157.3 TFLOP/s fp32
# vector peak counts an FMA as two flops and packed-fp32 pairs twice; this
# library is built without packed fp32.)
LANE_OP_PEAK = 256 * 64 * 2.4e9

# HBM traffic of the step kernels per launch, measured beforehand with
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch, averaged over
# 55 dispatches of "bench.py --steps 50 --warmup 5 --only-c2
# --no-cpu-baseline --no-profile --copy-calib-mb 512"), scaled by what the
# same counters read for the 512 MiB device copy in that run (FETCH x2.0,
# WRITE x1.0).  Valid only for the kernel sources it was taken on (SHA-256
# of the three files below); reported as null otherwise.
TRAFFIC = {"fetch_scale": 2.000, "write_scale": 1.000,
           "sources_sha256": "74b5b17800b2dd90018f7eb50688fd069392befb39b2901cdf72e202d772b4aa",
           # kernel: (FETCH_SIZE KiB, WRITE_SIZE KiB) per dispatch
           "kib": {"move": (19628.3, 40071.5), "scan": (4633.8, 16416.1), "scatter": (34512.7, 56205.0), "propose": (17700.9, 2952.1), "finish": (164.3, 0.5)}}
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


def cpu_baseline(model, budget_s: float = 12.0, max_steps: int = 400) -> dict:
    """The oracle as it stands, timed on this host's cores over the steps
    after its first (which also places the agents), up to ``max_steps`` or
    ``budget_s`` seconds of wall time."""
    import oracle
    threads = oracle.threads()
    o = oracle.OracleSim(model)
    o.step(1)
    n0, _ = o.size()
    updates, steps, t0 = 0, 0, time.perf_counter()
    while steps < max_steps and (time.perf_counter() - t0) < budget_s:
        n, _ = o.size()
        o.step(1)
        updates += n
        steps += 1
    dt = time.perf_counter() - t0
    return {"value": updates / dt, "unit": "agent-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{model.name}, {n0} agents, steps 2-{steps + 1} ({dt:.1f} s), C oracle on "
                      f"{threads} OpenMP threads (move phase and neighbour search in parallel)"}


def log(msg: str) -> None:
    """Progress line on stderr (the JSON result goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed_steps(torch, sim, steps: int):
    """(ms, agent-updates) of ``steps`` steps between HIP events on the
    simulation's stream, the state resident in HBM."""
    u0 = sim.agent_updates()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(sim.stream)
    sim.step(steps)
    ev1.record(sim.stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1), sim.agent_updates() - u0


def run_single(args, torch, mabm, W, model, steps: int, warmup: int, profile: bool,
               tuned=None) -> dict:
    """agent-updates/s of one simulation over ``steps`` steps after
    ``warmup`` (with the tuner's launch shape and search mode when
    ``tuned``); with ``profile``, a second region of the same length with
    per-kernel durations, and the roofline of the dominant kernel."""
    sim = mabm.Sim(model, graphs=args.graph, cell_um=args.cell_um)
    if tuned is not None:
        tuned.apply(sim)
    G, h = sim.grid()
    sim.step(warmup)
    sim.counts()  # synchronises; surfaces any device error
    ms, updates = timed_steps(torch, sim, steps)
    value = updates / (ms / 1e3)
    live = updates / steps
    counts, t = sim.counts()
    claim_sp = sorted({r.reactants[0] for r in model.rules if r.kind == W.BIMOL})
    claimers = int(counts[claim_sp].sum())
    out = {"value": value, "ms_per_step": ms / steps, "steps": steps, "warmup": warmup,
           "grid": G, "cell_um": round(h, 5), "bin_every": sim.get_param(mabm.PARAM_BIN_EVERY),
           "final_step": t, "live_agents_end": int(counts.sum())}
    if not profile:
        return out, sim
    # the same number of steps again, each kernel's dispatch stamping HIP
    # events at its start and end (direct launches), for per-kernel durations
    sim.profile(True)
    ms_direct, _ = timed_steps(torch, sim, steps)
    prof = sim.profile_read()
    sim.profile(False)
    bin_launches = prof["scan"][0]
    kernels = {}
    c2_size = args.workload == "c2" and model.n_agents == 2_000_000
    for name, (launches, tot) in prof.items():
        if not launches:
            continue
        a, q, c = KERNEL_BYTES[name]
        if name == "move":  # mean over binning and kept steps
            a = (a * bin_launches + MOVE_KEPT_BYTES * (launches - bin_launches)) / launches
        alg = a * live + q * claimers + c * G ** 3
        if name == "propose":  # candidates: 8 cells at the mean density
            alg += 16 * claimers * 8 * h ** 3 * live / volume_um3(model)
        us = 1e3 * tot / launches
        kernels[name] = {"launches": launches, "avg_us": round(us, 3),
                         "alg_bytes": int(alg), "alg_gbs": round(alg / us / 1e3, 1)}
        tb = measured_traffic(name) if c2_size else None
        if tb is not None:
            kernels[name]["traffic_bytes"] = tb
            kernels[name]["traffic_gbs"] = round(tb / us / 1e3, 1)
    mv = kernels["move"]
    us = mv["avg_us"]
    # move's prescribed lane operations, weighted by the launches of each
    # kind of step
    ops = live * (MOVE_OPS_BIN * bin_launches + MOVE_OPS_KEPT * (mv["launches"] - bin_launches)) \
        / mv["launches"]
    achieved = ops / (us * 1e-6)
    state_move = STATE_MOVE_BYTES * live
    roof = {"bound": "alu", "kernel": "move", "achieved": round(achieved / 1e12, 2),
            "peak": round(LANE_OP_PEAK / 1e12, 2), "unit": "T lane-op/s",
            "frac": round(achieved / LANE_OP_PEAK, 4),
            "traffic": mv.get("traffic_bytes"),
            "traffic_note": "FETCH_SIZE+WRITE_SIZE per launch from a stored rocprofv3 counter "
                            "run, null unless the kernel sources match its SHA-256",
            "alg_ops_per_launch": int(ops),
            "hbm": {"alg_bytes_per_launch": int(state_move),
                    "achieved_gbs": round(state_move / us / 1e3, 1), "peak_gbs": HBM_PEAK_GBS,
                    "frac": round(state_move / us / 1e3 / HBM_PEAK_GBS, 4)}}
    # the whole step against the HBM roofline of 70 B per update
    step_gbs = STATE_STEP_BYTES * value / 1e9
    roof["step"] = {"alg_bytes_per_update": STATE_STEP_BYTES, "alg_gbs": round(step_gbs, 1),
                    "hbm_roofline_updates_per_s": HBM_PEAK_GBS * 1e9 / STATE_STEP_BYTES,
                    "frac": round(step_gbs / HBM_PEAK_GBS, 4)}
    roof["copy_ceiling_gbs"] = round(copy_ceiling_gbs(torch), 1)
    out.update(roofline=roof, kernels=kernels, ms_per_step_kernel_timed=ms_direct / steps)
    return out, sim


def late_sample(torch, sim, at_step: int, steps: int, kernels: bool = True) -> dict:
    """The rate of the same simulation later in its run: advanced to step
    ``at_step`` (untimed), then ``steps`` timed steps, then (with
    ``kernels``) the same number again with per-kernel durations."""
    _, t = sim.counts()
    if t < at_step:
        sim.step(at_step - t)
        sim.counts()
    ms, updates = timed_steps(torch, sim, steps)
    _, t1 = sim.counts()
    out = {"from_step": t1 - steps, "steps": steps, "value": updates / (ms / 1e3),
           "ms_per_step": ms / steps}
    if kernels:
        sim.profile(True)
        timed_steps(torch, sim, steps)
        prof = sim.profile_read()
        sim.profile(False)
        out["kernels_avg_us"] = {k: round(1e3 * tot / n, 3) for k, (n, tot) in prof.items() if n}
        out["kernels_launches"] = {k: n for k, (n, tot) in prof.items() if n}
    return out


def _bits(e: dict) -> dict:
    return {k: (v.view("uint32") if v.dtype.kind == "f" else v) for k, v in e.items()}


def run_sweep(args, torch, mabm, W, tune_batch: bool, serial_all: bool) -> dict:
    """The dose x replicate sweep: every simulation for its whole horizon,
    once as one batch (its cell density and launch shape chosen by the batch
    tuner beforehand when ``tune_batch``) and once one at a time through the
    single-simulation path (all of them, or a sample extrapolated), with the
    final state of every simulation run alone compared with the batch's by
    the library's order-independent state digest."""
    models = W.c4_sweep(n_reps=args.sweep_reps, steps=args.sweep_steps)
    n, steps = len(models), args.sweep_steps
    tuned, serial_models = None, models
    if tune_batch:
        from paper_2606_14603_amd import tune
        tuned = tune.tune_batch(models)
        models = tuned.models(models)
    agents = sum(m.n_agents for m in models)
    warm = mabm.Batch(models[:2])  # code objects loaded before timing
    warm.step(3)
    warm.counts()
    del warm
    log(f"c4: batch of {n} simulations, {agents} agents, {steps} steps")
    batch = mabm.Batch(models, graphs=True)
    if tuned is not None:
        tuned.apply(batch)
    batch.grid()  # finalize: tables, placement
    ms_batch, updates = timed_steps(torch, batch, steps)
    batch_digest = batch.digest()
    # what launching costs at this size: the same batch's kernels timed one by
    # one (dispatch-stamped events, direct launches) over 200 more steps,
    # against the graph-replayed step
    batch.profile(True)
    batch.step(200)
    busy_ms = sum(ms for _, ms in batch.profile_read().values()) / 200
    batch.profile(False)
    batch.close()
    del batch
    sample = list(range(n)) if serial_all else \
        list(range(0, n, max(1, n // args.sweep_sample)))[:args.sweep_sample]
    log(f"c4: {len(sample)} simulations one at a time")
    ms_serial, same = 0.0, 0
    for k in sample:
        sim = mabm.Sim(serial_models[k], graphs=True)
        sim.grid()
        ms_k, _ = timed_steps(torch, sim, steps)
        ms_serial += ms_k
        same += int(sim.digest()[0] == batch_digest[k])
        sim.close()
    ms_serial_all = ms_serial * n / len(sample)
    value = n / (ms_batch * 1e-3)
    serial = n / (ms_serial_all * 1e-3)
    return {
        "value": value, "unit": "sims/s", "steps": steps, "ms_per_step": ms_batch / steps,
        "config": {"workload": f"c4_sweep: {n // args.sweep_reps} doses x {args.sweep_reps} "
                               f"replicates of c2_mapk, 20k-200k agents each, {steps} steps",
                   "sims": n, "agents": agents,
                   "tuned": None if tuned is None else {
                       "agents_per_cell": tuned.agents_per_cell, "lanes": tuned.lanes,
                       "min_workgroups": tuned.min_workgroups,
                       "ms_per_step": {k: round(v, 4) for k, v in tuned.ms_per_step.items()}}},
        "batched": {"ms": ms_batch, "agent_updates_per_s": updates / (ms_batch * 1e-3),
                    "launch": "graph-replayed steps (16 or more per graph launch)",
                    "kernel_us_per_step": busy_ms * 1e3,
                    "launch_gap_fraction": max(0.0, 1.0 - busy_ms / (ms_batch / steps))},
        "serial": {"value": serial, "unit": "sims/s", "ms": ms_serial_all,
                   "sims_run": len(sample),
                   "how": "every simulation run alone" if len(sample) == n else
                          f"{len(sample)} of {n} simulations run alone, {ms_serial:.1f} ms, "
                          f"scaled by {n}/{len(sample)}"},
        "speedup_vs_serial": value / serial,
        "identical_states": f"{same}/{len(sample)}",
        "bit_identical": same == len(sample),
    }


def run_serving(args, torch, mabm, W, n_requests: int, n_max: int, h_min: int,
                h_max: int) -> dict:
    """The request stream: each request a model of its own (a random closed
    subset of the cascade's rules), sizes log-uniform from 50k to ``n_max``
    agents, horizons uniform in [h_min, h_max].  The FIFO server (one
    request at a time) is first run on all requests arriving at once to
    measure its capacity; Poisson arrivals at 0.7 x that rate are then
    served FIFO and by the concurrent server, which keeps every admitted
    simulation resident and advances them on streams of their own.
    Admission: arrival order, while the summed arenas fit the budget.  The
    final state of every request is compared between the two servers by the
    library's state digest."""
    from paper_2606_14603_amd import serve

    def progress(r):  # one line per completed request, on stderr
        print(f"[serve] {r.name} done at {r.completed_s:.2f} s ({r.agents} agents, {r.steps} steps)",
              file=sys.stderr, flush=True)

    models = W.c5_requests(n_requests, seed=0, n_max=n_max, h_min=h_min, h_max=h_max)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.85 * free) if args.serve_budget_gb <= 0 else int(args.serve_budget_gb * 2**30)
    # load the code objects and the graph path once
    serve.Server(budget, max_active=2).run(W.c5_requests(2, seed=99, n_max=60_000, h_max=300),
                                           [0.0, 0.0])
    fifo = serve.Server(budget, max_active=1, chunk=args.serve_chunk, progress=progress)
    conc = serve.Server(budget, max_active=args.serve_active, chunk=args.serve_chunk,
                        progress=progress, fill_agents=args.serve_fill_agents)
    out = {"unit": "sims/s"}
    pairs = []  # (FIFO results, concurrent results) of the same requests
    cap = None
    if args.serve_legs in ("all", "capacity"):
        log(f"c5: {n_requests} requests, FIFO capacity")
        res_cap_fifo = fifo.run(models, np.zeros(len(models)))
        cap = serve.summarize(res_cap_fifo)
        log("c5: concurrent capacity")
        res_cap_conc = conc.run(models, np.zeros(len(models)))
        cap_conc = serve.summarize(res_cap_conc)
        pairs.append((res_cap_fifo, res_cap_conc))
        out.update(fifo_capacity=cap, concurrent_capacity=cap_conc,
                   capacity_ratio=cap_conc["sims_per_s"] / cap["sims_per_s"],
                   value=cap_conc["sims_per_s"])
    rate = args.serve_rate if args.serve_rate > 0 else (0.7 * cap["sims_per_s"] if cap else 0.0)
    if args.serve_legs in ("all", "poisson"):
        if rate <= 0:
            raise SystemExit("--serve-legs poisson needs --serve-rate")
        arrivals = W.poisson_arrivals(len(models), rate, seed=0)
        log(f"c5: Poisson arrivals at {rate:.3f}/s, FIFO")
        res_fifo = fifo.run(models, arrivals)
        log("c5: Poisson arrivals, concurrent")
        res_conc = conc.run(models, arrivals)
        s_fifo, s_conc = serve.summarize(res_fifo), serve.summarize(res_conc)
        pairs.append((res_fifo, res_conc))
        out.update(value=s_conc["sims_per_s"], p50_s=s_conc["p50_s"], p99_s=s_conc["p99_s"],
                   concurrent=s_conc, fifo=s_fifo)
    same = total = 0
    for a, b in pairs:
        by_name = {r.name: r.digest for r in a}
        same += sum(int(by_name[r.name] == r.digest) for r in b)
        total += len(b)
    out["config"] = {"workload": f"c5_requests: {len(models)} requests, random closed subsets of "
                                 f"the cascade's rules, 50k-{n_max // 1000}k agents (log-uniform), "
                                 f"{h_min}-{h_max} steps (uniform), Poisson arrivals at "
                                 + ("0.7 x the FIFO capacity" if args.serve_rate <= 0 else
                                    f"{rate:.3f}/s"),
                     "legs": args.serve_legs, "arrival_rate_per_s": rate, "budget_bytes": budget,
                     "chunk_steps": args.serve_chunk, "max_active": args.serve_active,
                     "fill_agents": args.serve_fill_agents}
    out.update(identical_states=f"{same}/{total}", bit_identical=same == total)
    return out


def base_line(value, unit, steps, warmup, ms_per_step, config, hib=True) -> dict:
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": ms_per_step, "higher_is_better": hib,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": config}


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
                    help="skip the batch tuner (cell density, launch shape) before the sweep")
    ap.add_argument("--workload", choices=("c1", "c2", "c3", "c4", "c5"), default="c2",
                    help="c2 (default): the 2M-agent cascade step (agent-updates/s, the "
                         "headline), with a late-run sample, the 5M-agent nested-compartment "
                         "model early and late, the full dose x replicate sweep and the serving "
                         "stream in the same line; c1: A+B<->C, 20k agents in a periodic box; "
                         "c3: nested compartments, 5M agents, births; c4: the batched sweep "
                         "alone (tuned); c5: the serving loop alone")
    ap.add_argument("--only-c2", action="store_true",
                    help="c2: the headline only (no c3, c4, c5 objects)")
    ap.add_argument("--late-at", type=int, default=2000, help="late-run sample from this step")
    ap.add_argument("--late-steps", type=int, default=500, help="steps of the late-run sample")
    ap.add_argument("--serve-requests", type=int, default=40, help="c5: requests")
    ap.add_argument("--serve-chunk", type=int, default=256, help="c5: steps per turn")
    ap.add_argument("--serve-fill-agents", type=int, default=4_000_000,
                    help="c5: the concurrent server admits no more while its simulations "
                         "hold this many agents")
    ap.add_argument("--serve-max-agents", type=int, default=4_000_000,
                    help="c5: largest request (log-uniform from 50k)")
    ap.add_argument("--serve-min-steps", type=int, default=1000, help="c5: shortest horizon")
    ap.add_argument("--serve-max-steps", type=int, default=20000, help="c5: longest horizon")
    ap.add_argument("--serve-active", type=int, default=64, help="c5: simulations admitted at once")
    ap.add_argument("--serve-legs", choices=("all", "capacity", "poisson"), default="all",
                    help="c5: the capacity runs (all requests at once, FIFO and concurrent), "
                         "the Poisson runs, or both")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="c5: Poisson arrival rate (0: 0.7 x the FIFO capacity measured first)")
    ap.add_argument("--serve-budget-gb", type=float, default=0.0,
                    help="c5: HBM budget for admitted arenas (0: 85%% of free memory)")
    ap.add_argument("--sweep-reps", type=int, default=64, help="c4: replicates per dose")
    ap.add_argument("--sweep-steps", type=int, default=2000, help="c4: steps per simulation")
    ap.add_argument("--sweep-sample", type=int, default=0,
                    help="c4: run only this many simulations one at a time and extrapolate "
                         "(0: all of them)")
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
        r = run_sweep(args, torch, mabm, W, tune_batch=not args.no_tune,
                      serial_all=args.sweep_sample == 0)
        line = base_line(r.pop("value"), r.pop("unit"), r.pop("steps"), 0, r.pop("ms_per_step"),
                         r.pop("config"))
        line.update(r)
        print(json.dumps(line), flush=True)
        return 0
    if args.workload == "c5":
        r = run_serving(args, torch, mabm, W, args.serve_requests, args.serve_max_agents,
                        args.serve_min_steps, args.serve_max_steps)
        line = base_line(r.pop("value"), r.pop("unit"), 0, 2, None, r.pop("config"))
        line.update(r)
        print(json.dumps(line), flush=True)
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
    tuned, tr = None, None
    if args.tune:
        from paper_2606_14603_amd import tune
        tr = tune.tune_cell(model)
        args.cell_um = tr.cell_um
        tuned = {"ms_per_step_by_cell_um": {f"{h:.5f}": round(ms, 4) for h, ms in tr.ms_per_step.items()},
                 "lanes": tr.lanes, "min_workgroups": tr.min_workgroups, "mode": tr.mode,
                 "ms_per_step_by_mode": {str(k): round(v, 4) for k, v in tr.ms_per_mode.items()}}
    log(f"{model.name}: {model.n_agents} agents, {args.warmup} warm-up + {args.steps} timed steps")
    r, sim = run_single(args, torch, mabm, W, model, args.steps, args.warmup,
                        profile=not args.no_profile, tuned=tr)
    config = {"workload": describe(model), "agents": model.n_agents, "grid": r.pop("grid"),
              "cell_um": r.pop("cell_um"), "graphs": args.graph, "bin_every": r.pop("bin_every"),
              "final_step": r.pop("final_step"), "tuned": tuned,
              "live_agents_end": r.pop("live_agents_end")}
    line = base_line(r.pop("value"), "agent-updates/s", r.pop("steps"), r.pop("warmup"),
                     r.pop("ms_per_step"), config)
    line.update(r)
    full = args.workload == "c2" and not args.only_c2
    if full or args.workload == "c3":
        log(f"late-run sample from step {args.late_at}")
        line["late_run"] = late_sample(torch, sim, args.late_at, args.late_steps)
    sim.close()
    del sim
    line["paper_context"] = PAPER_CONTEXT
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(model)
    if full:
        m3 = W.c3()
        log(f"c3: {m3.n_agents} agents, early and late samples")
        r3, s3 = run_single(args, torch, mabm, W, m3, 200, 50, profile=False)
        r3["late_run"] = late_sample(torch, s3, args.late_at, 200)
        r3["workload"] = describe(m3)
        s3.close()
        del s3
        line["c3"] = r3
        line["c4"] = run_sweep(args, torch, mabm, W, tune_batch=not args.no_tune,
                               serial_all=args.sweep_sample == 0)
        line["c5"] = run_serving(args, torch, mabm, W, args.serve_requests,
                                 args.serve_max_agents, args.serve_min_steps,
                                 args.serve_max_steps)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
