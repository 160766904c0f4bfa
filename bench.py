"""Benchmark: Z-map cells/s of the full simulation (edge discretisation, kinematics, binning,
per-cell minimum, roughness) on the 5000 x 5000 ball-end raster workload, one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one fsm_simulate call: plan tables to the device, the binned Z-map (count, scan,
write, per-tile reduction), the roughness passes and the result back on the host; the Z-map
stays resident in HBM.  Prints one JSON line.  The value comes from unprofiled steps; a second
set of steps with the library's HIP events on (recorded on the stream it launches on) gives
the per-stage kernel times and the roofline of the longest stage.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Z-map cells/s and simulations/s (p50/p99 latency), FP32 batched vs FP64 plain"
HBM_PEAK_GBS = 8000.0                          # MI355X HBM3E, GB/s
VALU_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}  # MI355X vector FP64 / FP32
KEY_BYTES = {"f64": 8, "f32": 4}
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_2603_28160_amd", "csrc", "fsm_kernels.hip")
STAGE_KERNEL = {"count": "hist_count", "write": "hist_write", "reduce": "tile_reduce"}
# the Z-map path a call took (fsm_timings.zmap_path)
PATH_NAMES = {0: "scatter", 1: "run", 2: "histogram", 3: "super"}


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def flop_per_eval(tool):
    """Algorithmic floating-point operations of one edge-point evaluation: the spindle rotation
    (4 mul + 2 add), the tilt rotations (lead or side alone: 4 mul + 2 add; both: a 3x3 product,
    9 mul + 6 add), the tool-centre offset (2 add) and the cell index (2 sub + 2 mul + 2 floor).
    Compares and integer index arithmetic are not counted."""
    lead, side = tool.tilt_lead != 0.0, tool.tilt_side != 0.0
    tilt = 15 if (lead and side) else (6 if (lead or side) else 0)
    return 6 + tilt + 2 + 6


def stored_traffic(kernel, prec):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None when the
    summary is missing or was taken on a different kernel source."""
    import hashlib
    import re
    path = os.path.join(PROFILES, f"{kernel}_{prec}_ball_r3_5000x5000_pmc.md")
    try:
        text = open(path).read()
        src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("kernel_source_sha256") != src:
        return None
    return d.get("hbm_bytes_per_launch")


def run_precision(ctx, sim, prec, steps, warmup, profile, graphs=False):
    import torch
    zmap = ctx.new_zmap(sim.grid, prec)
    # per-stage events need eager launches; the value steps may replay a captured graph
    ctx.set_graphs(graphs and not profile)
    ctx.fsm_ctx_set_profiling(profile)
    for _ in range(warmup):
        ctx.fsm_simulate(sim, prec, zmap)
    torch.cuda.synchronize()
    lat, tim = [], []
    t0 = time.perf_counter()
    r = None
    for _ in range(steps):
        a = time.perf_counter()
        _, r = ctx.fsm_simulate(sim, prec, zmap)
        lat.append((time.perf_counter() - a) * 1e3)
        if profile:
            tim.append(ctx.fsm_last_timings())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.fsm_ctx_set_profiling(False)
    out = {"elapsed_s": el, "ms_per_step": el / steps * 1e3, "lat": lat, "rough": r}
    if profile:
        for k in ("fill_ms", "scatter_ms", "rough_ms", "count_ms", "index_ms", "write_ms",
                  "reduce_ms"):
            out[k] = statistics.mean(t[k] for t in tim)
        out["n_slices"] = tim[-1]["n_slices"]
        out["zmap_path"] = tim[-1]["zmap_path"]
    return out


def batch_leg(ctx, n_sims):
    """Configuration 3 (n_sims seeded simulations, sides up to 2048): every simulation once,
    batched (one fsm_simulate_batch, eager and replayed from a captured graph), plain (one
    fsm_simulate per simulation, each waited for) and asynchronous (batches of 32 on two
    slots), in both precisions.  Z-maps resident in HBM."""
    import torch
    from paper_2603_28160_amd import workloads
    sims = workloads.config3(n_sims)
    cells = sum(s.grid.nx * s.grid.ny for s in sims)
    out = {"workload": f"config3_mix_{n_sims}", "sims": n_sims, "cells": cells}
    for prec in ("f32", "f64"):
        zmaps = [ctx.new_zmap(s.grid, prec) for s in sims]
        # one untimed pass of each form sizes and touches the workspaces, as in steady use
        ctx.fsm_simulate_batch(sims, prec, zmaps=zmaps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.fsm_simulate_batch(sims, prec, zmaps=zmaps)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        # the same batch replayed from a captured graph (the first call captures it)
        ctx.set_graphs(True)
        ctx.fsm_simulate_batch(sims, prec, zmaps=zmaps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.fsm_simulate_batch(sims, prec, zmaps=zmaps)
        torch.cuda.synchronize()
        tg = time.perf_counter() - t0
        ctx.set_graphs(False)
        for s, z in zip(sims, zmaps):
            ctx.fsm_simulate(s, prec, z)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s, z in zip(sims, zmaps):
            ctx.fsm_simulate(s, prec, z)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        # the same simulations as asynchronous batches of 32 on two slots: the host plans and
        # packs batch k + 1 while batch k runs
        def run_async(group=32):
            pending = []
            for k0 in range(0, n_sims, group):
                while len(pending) >= 2:
                    ctx.fsm_batch_wait(pending.pop(0))
                bid, _ = ctx.fsm_batch_submit(sims[k0:k0 + group], prec, zmaps=zmaps[k0:k0 + group])
                pending.append(bid)
            for bid in pending:
                ctx.fsm_batch_wait(bid)
        run_async()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_async()
        torch.cuda.synchronize()
        ta = time.perf_counter() - t0
        del zmaps
        torch.cuda.empty_cache()
        out[prec] = {"batched": {"s": tb, "sims_per_s": n_sims / tb, "cells_per_s": cells / tb},
                     "batched_graph": {"s": tg, "sims_per_s": n_sims / tg, "cells_per_s": cells / tg},
                     "plain": {"s": tp, "sims_per_s": n_sims / tp, "cells_per_s": cells / tp},
                     "async_32x2": {"s": ta, "sims_per_s": n_sims / ta, "cells_per_s": cells / ta}}
        print(f"[bench] config3 x{n_sims} {prec}: batched {tb:.3f} s, graph {tg:.3f} s, plain {tp:.3f} s, async {ta:.3f} s",
              file=sys.stderr, flush=True)
    return out


def large_leg(ctx, steps=3):
    """Configuration 5: one 40000 x 40000 field at 0.5 um (1.6e9 cells; the map is 6.4 GB in
    single and 12.8 GB in double precision), the D = 12 mm four-flute mill with variable pitch;
    both precisions: time per simulation, cells/s, and the per-stage times of one profiled step
    with the roofline of each Z-map stage (the binning passes against the vector peak, the tile
    reduction against HBM)."""
    import torch
    from paper_2603_28160_amd import fsm_plan, workloads
    sim = workloads.config5()
    plan = fsm_plan(sim, "f32")
    cells = sim.grid.nx * sim.grid.ny
    out = {"workload": sim.name, "evals": plan["n_evals"], "steps": steps}
    for prec in ("f32", "f64"):
        z = ctx.new_zmap(sim.grid, prec)
        ctx.fsm_simulate(sim, prec, z)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, r = ctx.fsm_simulate(sim, prec, z)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        ctx.fsm_ctx_set_profiling(True)
        ctx.fsm_simulate(sim, prec, z)
        t = ctx.fsm_last_timings()
        ctx.fsm_ctx_set_profiling(False)
        del z
        torch.cuda.empty_cache()
        prof = {k: t[k] for k in ("fill_ms", "scatter_ms", "rough_ms", "count_ms", "index_ms",
                                  "write_ms", "reduce_ms", "n_slices", "zmap_path")}
        prof["rough"] = r
        out[prec] = {"ms_per_sim": el * 1e3, "cells_per_s": cells / el,
                     "evals_per_s": plan["n_evals"] / el, "coverage": r["n_hit"] / cells,
                     "kernel_ms": {k[:-3]: prof[k] for k in prof if k.endswith("_ms")},
                     "n_slices": prof["n_slices"], "zmap_path": PATH_NAMES[prof["zmap_path"]],
                     "rooflines": stage_rooflines(sim, plan, prec, prof)}
        print(f"[bench] config5 {prec}: {el * 1e3:.2f} ms per simulation (count {t['count_ms']:.2f}, "
              f"write {t['write_ms']:.2f}, reduce {t['reduce_ms']:.2f} ms)", file=sys.stderr, flush=True)
    return out


def coverage_leg(ctx, steps=3):
    """Coverage-complete mode: the 200 x 200 single pass at 5 um refined by fsm_refine to a
    sample spacing of half a cell, both precisions; coverage before and after, time per
    simulation and evaluations/s."""
    import torch
    from paper_2603_28160_amd import fsm_plan, fsm_refine, workloads
    coarse = workloads.config1()
    sim = fsm_refine(coarse, coarse.grid.dd / 2)
    plan = fsm_plan(sim)
    cells = sim.grid.nx * sim.grid.ny
    out = {"workload": "config1_refined_to_half_cell", "n_edge": sim.tool.n_edge,
           "steps_per_rev": sim.cut.steps_per_rev, "evals": plan["n_evals"]}
    for prec in ("f64", "f32"):
        z = ctx.new_zmap(sim.grid, prec)
        _, r0 = ctx.fsm_simulate(coarse, prec, z)
        ctx.fsm_simulate(sim, prec, z)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, r = ctx.fsm_simulate(sim, prec, z)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        out[prec] = {"ms_per_sim": el * 1e3, "evals_per_s": plan["n_evals"] / el,
                     "coverage_coarse": r0["n_hit"] / cells, "coverage": r["n_hit"] / cells}
    print(f"[bench] refined config1: f64 {out['f64']['ms_per_sim']:.2f} ms, coverage "
          f"{out['f64']['coverage_coarse']:.3f} -> {out['f64']['coverage']:.3f}",
          file=sys.stderr, flush=True)
    return out


def dataset_leg(ctx, n=64, side=1024, dd=0.002):
    """Dataset generation (Sec. 4.3): n ball-end simulations drawn by Latin hypercube sampling
    on one side x side grid at dd, simulated in one batch, then all maps through the
    measurement chain of Sec. 4.1.1 (S-filter 10 um, least-squares plane, L-filter 0.8 mm) and
    their roughness in one texture batch, in single precision: samples/s end to end.  Then the 0.8 mm L-filter alone
    on a full 5000 x 5000 map at 1 um (synthetic, with and without empty cells), both
    precisions: time and FP64 fused multiply-add rate (2 passes x (2R + 1) taps per cell; with
    empty cells numerator and denominator)."""
    import torch
    from paper_2603_28160_amd import workloads
    sims = workloads.dataset_sims(n, side=side, dd=dd)
    prec = "f32"
    zmaps = [ctx.new_zmap(s.grid, prec) for s in sims]
    texs = [ctx.new_zmap(sims[0].grid, prec) for _ in sims]
    out = {"workload": f"lhs_ball_{n}x{side}x{side}", "precision": prec}

    def run():
        t0 = time.perf_counter()
        ctx.fsm_simulate_batch(sims, prec, zmaps=zmaps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rough = ctx.fsm_texture_batch(sims[0].grid, zmaps, prec, outs=texs)[1]
        torch.cuda.synchronize()
        return t1 - t0, time.perf_counter() - t1, rough

    run()
    ts, tt, rough = run()
    out.update({"simulate_s": ts, "texture_s": tt, "samples_per_s": n / (ts + tt),
                "mean_coverage": float(np.mean([r["n_hit"] for r in rough])) / (side * side),
                "Sa_range_um": [1e3 * min(r["Sa"] for r in rough), 1e3 * max(r["Sa"] for r in rough)]})
    del zmaps, texs
    big = workloads.centred_grid(5000, 5000, 0.001)
    R = int(math.floor(0.8 / big.dd + 1e-9))
    out["l_filter_5000x5000"] = {}
    for holes in (0.0, 0.02):
        Z = workloads.synthetic_surface(5000, 5000, 0.001, seed=5, hole_frac=holes)
        for p in ("f64", "f32"):
            z = torch.from_numpy(Z).to(dtype=torch.float64 if p == "f64" else torch.float32,
                                       device="cuda:0")
            o = ctx.new_zmap(big, p)
            ctx.fsm_filter(big, z, 0.8, p, highpass=True, out=o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                ctx.fsm_filter(big, z, 0.8, p, highpass=True, out=o)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / 3
            fma = 2 * (2 * R + 1) * 25e6 * (2 if holes else 1)
            out["l_filter_5000x5000"][f"{p}_{'holes' if holes else 'full'}"] = {
                "ms": el * 1e3, "fp64_tflops": 2 * fma / el / 1e12,
                "frac_of_fp64_peak": 2 * fma / el / 78.6e12}
            del z, o
        torch.cuda.empty_cache()
    print(f"[bench] dataset: {out['samples_per_s']:.1f} samples/s; L-filter 5000^2 f64 "
          f"{out['l_filter_5000x5000']['f64_full']['ms']:.2f} ms", file=sys.stderr, flush=True)
    return out


# EFSM wall times (s) of the paper's nine performance conditions on its laptop CPU, from the
# computation-time table of Sec. 4.3: context for the paper-mode leg, not a target
PAPER_EFSM_S = {1: 0.81, 2: 0.68, 3: 0.55, 4: 0.65, 5: 0.52, 6: 0.45, 7: 0.59, 8: 0.46, 9: 0.43}


def paper_leg(ctx, steps=3):
    """The paper's nine performance conditions in its fixed-time-step mode (Case-2 tool, 10 x 5
    mm at 5 um, dt = 0.4 us), one plain simulation each, both precisions: time per simulation,
    trajectory points/s and edge-point evaluations/s."""
    import torch
    from paper_2603_28160_amd import fsm_plan, workloads
    out = {"workload": "paper_conditions_10x5mm_dt0.4us", "conditions": {}}
    for no in range(1, 10):
        sim = workloads.paper_mode(no)
        plan = fsm_plan(sim)
        traj = sim.tool.n_teeth * plan["n_steps"]
        row = {"trajectory_points": traj, "evals": plan["n_evals"],
               "paper_efsm_s": PAPER_EFSM_S[no]}
        for prec in ("f64", "f32"):
            z = ctx.new_zmap(sim.grid, prec)
            ctx.fsm_simulate(sim, prec, z)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                ctx.fsm_simulate(sim, prec, z)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / steps
            row[prec] = {"ms": el * 1e3, "trajectory_points_per_s": traj / el,
                         "evals_per_s": plan["n_evals"] / el}
        out["conditions"][no] = row
    ms = [out["conditions"][k]["f64"]["ms"] for k in out["conditions"]]
    print(f"[bench] paper conditions f64: {min(ms):.2f}..{max(ms):.2f} ms per simulation",
          file=sys.stderr, flush=True)
    return out


SERVE_RATES = (50.0, 200.0, 500.0, 1000.0, 2000.0)


def serve_leg(ctx, rates, n_req=None, max_batch=16, n_slots=2):
    """Configuration 4 over a sweep of Poisson arrival rates: requests drawn like configuration
    3 with sides up to 4096, served with continuous batching (server-held Z-maps in a device
    arena, n_slots slots, batches of up to max_batch), in both precisions: simulations/s, p50
    and p99 latency (arrival to result on the host) per rate.  Each rate serves n_req requests
    (default 2000, 1000 at the lowest rate so it stays near 20 s).  Beside them, the same
    request mix as plain double-precision single-simulation launches one after another (no
    arrivals, no batching): simulations/s and per-launch latency."""
    import torch
    from paper_2603_28160_amd import workloads
    out = {"workload": "config4_poisson_sweep", "n_slots": n_slots, "max_batch": max_batch,
           "rates": {}}
    for rate in rates:
        n = n_req or (1000 if rate < 100 else 2000)
        reqs = workloads.config4_requests(n, rate)
        row = {"requests": n}
        for prec in ("f32", "f64"):
            res = ctx.fsm_serve_run([(s, a, None) for a, s in reqs], prec, n_slots=n_slots,
                                    max_batch=max_batch, arena_bytes=8 << 30, slot_bytes=2 << 30)
            ok = [(r, a) for r, (a, _) in zip(res, reqs) if r["status"] == 0]
            lat = [(r["done_s"] - a) * 1e3 for r, a in ok]
            span = max(r["done_s"] for r, _ in ok) - min(a for _, a in ok)
            sizes = {}
            for r, _ in ok:
                sizes[r["batch"]] = sizes.get(r["batch"], 0) + 1
            row[prec] = {"sims_per_s": len(ok) / span, "latency_ms": {"p50": pct(lat, 50),
                         "p99": pct(lat, 99)}, "completed": len(ok),
                         "mean_batch": len(ok) / max(1, len(sizes))}
            print(f"[bench] serving {rate:g}/s {prec}: {len(ok)}/{n} done, {len(ok) / span:.1f} sims/s, "
                  f"p50 {pct(lat, 50):.2f} ms, p99 {pct(lat, 99):.2f} ms, mean batch "
                  f"{row[prec]['mean_batch']:.2f}", file=sys.stderr, flush=True)
        out["rates"][f"{rate:g}"] = row
    # plain double-precision launches over the same request mix
    reqs = workloads.config4_requests(2000, rates[0])
    sims = [s for _, s in reqs]
    for s in sims[:8]:
        ctx.fsm_simulate(s, "f64")
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for s in sims:
        a = time.perf_counter()
        ctx.fsm_simulate(s, "f64")
        lat.append((time.perf_counter() - a) * 1e3)
    el = time.perf_counter() - t0
    torch.cuda.empty_cache()
    out["plain_f64"] = {"requests": len(sims), "sims_per_s": len(sims) / el,
                        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)}}
    print(f"[bench] plain f64 launches over the mix: {len(sims) / el:.1f} sims/s, p50 "
          f"{pct(lat, 50):.2f} ms, p99 {pct(lat, 99):.2f} ms", file=sys.stderr, flush=True)
    return out


def trajectory_leg(ctx, steps=5):
    """The trajectory module (Sec. 3.2) on the configuration 2 path: for every pass, step and
    tooth the lowest of the tooth's edge points in the workpiece frame, in both precisions;
    time per call and evaluations/s.  It evaluates every edge point of every step (the lowest
    point is wanted off the grid too), which the Z-map's culling skips."""
    import torch
    from paper_2603_28160_amd import fsm_plan, workloads
    sim = workloads.config2()
    plan = fsm_plan(sim)
    out = {"workload": sim.name, "evals": plan["n_evals"],
           "entries": plan["n_passes"] * plan["n_steps"] * sim.tool.n_teeth}
    for prec in ("f64", "f32"):
        ctx.fsm_trajectory(sim, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.fsm_trajectory(sim, prec)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        out[prec] = {"ms": el * 1e3, "evals_per_s": plan["n_evals"] / el}
        torch.cuda.empty_cache()
    print(f"[bench] trajectory f64 {out['f64']['ms']:.3f} ms, f32 {out['f32']['ms']:.3f} ms",
          file=sys.stderr, flush=True)
    return out


def latency_leg(ctx, steps=200):
    """Configuration 1 (200 x 200 at 5 um, one pass, double precision): launch latency of one
    plain fsm_simulate call, eager and replayed from a captured graph: p50/p99 over `steps`
    calls, each from the call to the roughness on the host."""
    import torch
    from paper_2603_28160_amd import workloads
    sim = workloads.config1()
    out = {"workload": sim.name, "precision": "f64", "steps": steps}
    z = ctx.new_zmap(sim.grid, "f64")
    for graphs in (False, True):
        ctx.set_graphs(graphs)
        for _ in range(10):
            ctx.fsm_simulate(sim, "f64", z)
        torch.cuda.synchronize()
        lat = []
        for _ in range(steps):
            a = time.perf_counter()
            ctx.fsm_simulate(sim, "f64", z)
            lat.append((time.perf_counter() - a) * 1e3)
        out["graphs" if graphs else "eager"] = {"p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                                                "mean_ms": statistics.mean(lat)}
    ctx.set_graphs(False)
    print(f"[bench] config1 f64 latency: eager p50 {out['eager']['p50_ms']:.3f} ms, graphs p50 "
          f"{out['graphs']['p50_ms']:.3f} ms", file=sys.stderr, flush=True)
    return out


def stage_rooflines(sim, plan, prec, prof):
    """Roofline of every stage of one step, per launch, from the library's HIP events (recorded
    on the stream it launches on).  The binning passes are bound by the vector rate: the
    algorithmic work is flop_per_eval(tool) times the evaluations (in super mode the write
    stage also holds the split of the super-tile buckets).  The scans move the row matrix and
    are reported by time.  The tile reduction reads every bucket entry (key + 16-bit cell) and
    writes every cell; the roughness reads every cell once more (its first pass is fused into
    the reduction)."""
    r = prof["rough"]
    n_launch = max(1, prof["n_slices"])
    cells = sim.grid.nx * sim.grid.ny
    kb = KEY_BYTES[prec]
    path = PATH_NAMES.get(prof.get("zmap_path"), "histogram")
    run_mode = path == "run"
    names = ("bin_points<%s,false>" if run_mode else "hist_count<%s>",
             "bin_points<%s,true>" if run_mode else
             ("hist_write<%s> + split_super" if path == "super" else "hist_write<%s>"))
    fpe = flop_per_eval(sim.tool)
    out = {}
    for stage, name in (("count", names[0]), ("write", names[1])):
        ms = prof[f"{stage}_ms"] / n_launch
        if ms <= 0.0:
            continue
        a = fpe * plan["n_evals"] / n_launch / (ms * 1e-3) / 1e12
        out[stage] = {"kernel": name % prec, "bound": "alu", "unit": "TFLOP/s", "launch_ms": ms,
                      "flop_per_eval": fpe, "achieved": a, "peak": VALU_PEAK_TFLOPS[prec],
                      "frac": a / VALU_PEAK_TFLOPS[prec]}
    if prof["index_ms"] > 0.0:
        out["index"] = {"kernel": "row-matrix scans" if not run_mode else "tile-count scan",
                        "bound": "hbm", "launch_ms": prof["index_ms"] / n_launch}
    ms = prof["reduce_ms"] / n_launch
    if ms > 0.0:
        work = (r["n_binned"] * (kb + 2) + cells * kb) / n_launch
        a = work / (ms * 1e-3) / 1e9
        out["reduce"] = {"kernel": f"tile_reduce<{prec}>", "bound": "hbm", "unit": "GB/s",
                         "launch_ms": ms, "bytes_per_launch": work, "achieved": a,
                         "peak": HBM_PEAK_GBS, "frac": a / HBM_PEAK_GBS}
    ms = prof["rough_ms"]
    if ms > 0.0:
        a = cells * kb / (ms * 1e-3) / 1e9
        out["roughness"] = {"kernel": f"tile_stats2<{prec}> + combines", "bound": "hbm",
                            "unit": "GB/s", "launch_ms": ms, "bytes_per_launch": cells * kb,
                            "achieved": a, "peak": HBM_PEAK_GBS, "frac": a / HBM_PEAK_GBS}
    return out


def roofline(sim, plan, prec, prof):
    """Roofline of the longest stage of the Z-map (the dominant kernel), timed with HIP events
    on the stream the library launches on (mean over the profiled steps, per launch), with the
    HBM traffic of the committed counter summary when it was taken on this kernel source."""
    stages = {k: prof[f"{k}_ms"] for k in ("count", "write", "reduce")}
    stage = max(stages, key=stages.get)
    n_launch = max(1, prof["n_slices"])
    ms = stages[stage] / n_launch
    kernel = STAGE_KERNEL[stage]
    if ms <= 0.0:
        # scatter strategy: one kernel does kinematics, binning and the minimum
        stage, kernel, n_launch, ms = "count", "scatter", 1, prof["scatter_ms"]
    r = prof["rough"]
    if stage in ("count", "write"):
        fpe = flop_per_eval(sim.tool)
        work = fpe * plan["n_evals"] / n_launch
        achieved = work / (ms * 1e-3) / 1e12
        peak = VALU_PEAK_TFLOPS[prec]
        out = {"bound": "alu", "unit": "TFLOP/s", "flop_per_eval": fpe,
               "evals_per_launch": plan["n_evals"] // n_launch}
    else:
        # bucket entries read (key + 16-bit cell), Z-map read-free first slice, Z-map written
        work = (r["n_binned"] * (KEY_BYTES[prec] + 2) + sim.grid.nx * sim.grid.ny * KEY_BYTES[prec]) / n_launch
        achieved = work / (ms * 1e-3) / 1e9
        peak = HBM_PEAK_GBS
        out = {"bound": "hbm", "unit": "GB/s", "bytes_per_launch": work}
    traffic = stored_traffic(kernel, prec)
    out.update({"kernel": f"{kernel}<{prec}>", "achieved": achieved, "peak": peak,
                "frac": achieved / peak, "traffic": traffic, "launch_ms": ms,
                "launches_per_step": n_launch, "stage_ms": stages,
                "index_ms": prof["index_ms"]})
    return out


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(sim, max_threads=16):
    """The FP64 oracle, unchanged, on the host cores: the whole workload on one thread, then
    on all the process's cores as one task per pass (a pass run alone sits at the same y as in
    the raster, so the passes' maps merge by cell-wise minimum into the same map bit for bit,
    which is checked).  Returns (record, the one-thread map)."""
    import dataclasses
    from concurrent.futures import ThreadPoolExecutor, as_completed

    import oracle
    model, nproc = cpu_info()
    print(f"[bench] cpu baseline: FP64 oracle on the full workload, 1 thread then "
          f"{min(nproc, max_threads)} ({model})", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    zo, cnt = oracle.simulate(sim)
    el1 = time.perf_counter() - t0
    pl = oracle.plan(sim)
    base = dataclasses.replace(sim.cut, x_start=pl["x_start"], n_steps=pl["n_steps"], n_passes=1)
    passes = [sim.replace(cut=dataclasses.replace(base, y_first=pl["y_first"] + float(q) * sim.cut.a_e))
              for q in range(pl["n_passes"])]
    threads = min(nproc, max_threads)
    t0 = time.perf_counter()
    acc = None
    with ThreadPoolExecutor(threads) as pool:
        for f in as_completed([pool.submit(oracle.simulate, p) for p in passes]):
            z, _ = f.result()
            acc = z if acc is None else np.minimum(acc, z, out=acc)
    eln = time.perf_counter() - t0
    same = bool(np.array_equal(acc, zo))
    n_cells = sim.grid.nx * sim.grid.ny
    rec = {"value": n_cells / el1, "unit": "cells/s", "cores": 1, "kind": "oracle",
           "sample": f"full {sim.name} FP64, one simulation, {el1:.1f} s",
           "cpu_model": model, "nproc": nproc,
           "all_cores": {"value": n_cells / eln, "unit": "cells/s", "threads": threads,
                         "s": eln, "identical_to_one_thread": same,
                         "split": f"{len(passes)} single-pass tasks merged by cell-wise minimum"}}
    return rec, zo


def f32_error(zg, rg, zo):
    """Error statement of the single-precision map against the FP64 oracle's map of the same
    workload: the library's own bound and near-boundary count, the cells whose hit state or
    height moved beyond that bound, the cells outside +-2e-6 mm, and the relative error of
    every roughness parameter."""
    import oracle
    ro = oracle.roughness(zo)
    hg, ho = np.isfinite(zg), np.isfinite(zo)
    both = hg & ho
    d = np.where(both, np.abs(zg - zo), 0.0)
    rel = {}
    for k in ("Sa", "Sq", "Sp", "Sv", "Sz", "Ssk", "Sku", "Ra_feed", "Ra_pick", "mean"):
        rel[k] = abs(rg[k] - ro[k]) / abs(ro[k]) if ro[k] else abs(rg[k] - ro[k])
    return {"against": "FP64 oracle, full map", "pos_err_mm": rg["pos_err"],
            "n_near": rg["n_near"], "n_binned": rg["n_binned"],
            "hit_state_changed": int((hg != ho).sum()),
            "cells_moved_beyond_pos_err": int((hg != ho).sum() + (d > rg["pos_err"]).sum()),
            "cells_outside_2e-6_mm": int((d > 2e-6).sum()),
            "max_abs_dz_same_hit_mm": float(d.max()),
            "rel_err": rel, "rel_err_max_areal": max(rel[k] for k in ("Sa", "Sq", "Ssk", "Sku"))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1, help="GPUs to use; only 1 is supported")
    ap.add_argument("--steps", type=int, default=10, help="timed steps (one simulation each)")
    ap.add_argument("--warmup", type=int, default=3, help="untimed steps before the timed ones")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip timing the CPU oracle on a sample of the workload")
    ap.add_argument("--precision", choices=["f64", "f32", "both"], default="both",
                    help="precision of the value (f64) and of the reported FP32 line")
    ap.add_argument("--strategy", choices=["binned", "scatter"], default="binned",
                    help="Z-map strategy of the timed steps")
    ap.add_argument("--compare-strategies", action="store_true",
                    help="also time the other Z-map strategy (reported, not the value)")
    ap.add_argument("--graphs", action="store_true",
                    help="replay the launch sequence from a HIP graph in the timed steps")
    ap.add_argument("--autotune", action="store_true",
                    help="let fsm_autotune pick the launch parameters before timing (untimed)")
    ap.add_argument("--tuning", default=os.path.join(ROOT, "paper_2603_28160_amd", "tuning_mi355x.json"),
                    help="saved tuning table to load (the library's autotuner output); "
                         "'none' to run on the default launch parameters")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batch (configuration 3) and serving (configuration 4) legs")
    ap.add_argument("--extras", default="all",
                    help="comma-separated extra legs to run (default all): latency, trajectory, "
                         "batch, serving, large_field, paper_mode, coverage_complete, dataset")
    ap.add_argument("--batch-sims", type=int, default=256, help="simulations in the batch leg")
    ap.add_argument("--serve-requests", type=int, default=0,
                    help="requests per arrival rate in the serving leg (0: 2000, 1000 below "
                         "100 requests/s)")
    ap.add_argument("--serve-rates", default=",".join(f"{r:g}" for r in SERVE_RATES),
                    help="comma-separated Poisson arrival rates of the serving leg, requests/s")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (reads 1 GiB, writes "
                         "1 GiB) five times, to scale HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (independent "
              "simulations would shard across GPUs, one process each, without communication)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        x = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": x.numel() * 8, "launches": 5}), flush=True)
        return
    from paper_2603_28160_amd import Context, fsm_plan, workloads

    sim = workloads.config2()
    plan = fsm_plan(sim)
    n_cells = sim.grid.nx * sim.grid.ny
    res = {}
    with Context(0) as ctx:
        n_tuned = 0
        if args.tuning != "none" and os.path.exists(args.tuning):
            n_tuned = ctx.load_tuning(args.tuning)
            print(f"[bench] tuning table: {n_tuned} entries from {os.path.basename(args.tuning)}",
                  file=sys.stderr, flush=True)
        precs = ["f64", "f32"] if args.precision == "both" else [args.precision]
        other = {}
        if args.compare_strategies:
            alt = "scatter" if args.strategy == "binned" else "binned"
            ctx.set_strategy(alt)
            for prec in precs:
                o = run_precision(ctx, sim, prec, args.steps, args.warmup, profile=True)
                other[prec] = {"ms_per_step": o["ms_per_step"], "zmap_ms": o["scatter_ms"]}
                print(f"[bench] {alt} {prec}: {o['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
        ctx.set_strategy(args.strategy)
        tuned = {}
        for prec in precs:
            if args.autotune:
                tuned[prec] = ctx.fsm_autotune([sim], prec)
                print(f"[bench] autotune {prec}: {tuned[prec]}", file=sys.stderr, flush=True)
            print(f"[bench] {sim.name} {prec}: warmup {args.warmup}, steps {args.steps}",
                  file=sys.stderr, flush=True)
            res[prec] = run_precision(ctx, sim, prec, args.steps, args.warmup, profile=False,
                                      graphs=args.graphs)
            res[prec]["prof"] = run_precision(ctx, sim, prec, args.steps, 1, profile=True)
            p = res[prec]["prof"]
            print(f"[bench] {prec}: {res[prec]['ms_per_step']:.3f} ms/step; z-map {p['scatter_ms']:.3f} ms "
                  f"(count {p['count_ms']:.3f}, index {p['index_ms']:.3f}, write {p['write_ms']:.3f}, "
                  f"reduce {p['reduce_ms']:.3f}), roughness {p['rough_ms']:.3f} ms",
                  file=sys.stderr, flush=True)
        # the single-precision map of the workload, for its error against the oracle
        f32_map = f32_rough = None
        if "f32" in precs and not args.no_cpu_baseline:
            z32, f32_rough = ctx.fsm_simulate(sim, "f32")
            f32_map = z32.cpu().numpy().astype(np.float64)
            del z32
        extras = {}
        rates = tuple(float(x) for x in args.serve_rates.split(",") if x)
        legs = {"latency": lambda: latency_leg(ctx),
                "trajectory": lambda: trajectory_leg(ctx),
                "batch": lambda: batch_leg(ctx, args.batch_sims),
                "serving": lambda: serve_leg(ctx, rates, args.serve_requests),
                "large_field": lambda: large_leg(ctx),
                "paper_mode": lambda: paper_leg(ctx),
                "coverage_complete": lambda: coverage_leg(ctx),
                "dataset": lambda: dataset_leg(ctx)}
        wanted = list(legs) if args.extras == "all" else [x for x in args.extras.split(",") if x]
        for name in ([] if args.no_extras else wanted):
            if name not in legs:
                raise SystemExit(f"unknown leg {name!r}; legs: {', '.join(legs)}")
            extras[name] = legs[name]()

    main_prec = "f64" if "f64" in res else precs[0]
    m = res[main_prec]
    r = m["rough"]

    def kernel_ms(p):
        return {"fill": p["fill_ms"], "zmap": p["scatter_ms"], "zmap_count": p["count_ms"],
                "zmap_index": p["index_ms"], "zmap_write": p["write_ms"],
                "zmap_reduce": p["reduce_ms"], "roughness": p["rough_ms"]}

    out = {
        "metric": METRIC,
        "value": n_cells * args.steps / m["elapsed_s"],
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_prec,
        "data": "synthetic",
        "config": {"workload": sim.name, "nx": sim.grid.nx, "ny": sim.grid.ny,
                   "dd_mm": sim.grid.dd, "tool": "ball R3 z4 helix30 tilt15",
                   "passes": plan["n_passes"], "steps_per_pass": plan["n_steps"],
                   "edge_points": sim.tool.n_edge, "evals": plan["n_evals"],
                   "precision": main_prec, "mode": "plain single-simulation launches",
                   "zmap_strategy": args.strategy,
                   "zmap_path": PATH_NAMES.get(m["prof"].get("zmap_path"), "scatter"),
                   "graphs": args.graphs,
                   "tuning_entries": n_tuned, "autotuned": tuned.get(main_prec)},
        "sims_per_s": args.steps / m["elapsed_s"],
        "latency_ms": {"p50": pct(m["lat"], 50), "p99": pct(m["lat"], 99)},
        "evals_per_s": plan["n_evals"] * args.steps / m["elapsed_s"],
        "binned_per_s": r["n_binned"] * args.steps / m["elapsed_s"],
        "coverage": r["n_hit"] / n_cells,
        "kernel_ms": kernel_ms(m["prof"]),
        "roofline": roofline(sim, plan, main_prec, m["prof"]),
        "rooflines": stage_rooflines(sim, plan, main_prec, m["prof"]),
    }
    for prec in res:
        if prec == main_prec:
            continue
        o = res[prec]
        out[prec] = {"value": n_cells * args.steps / o["elapsed_s"], "unit": "cells/s",
                     "ms_per_step": o["ms_per_step"],
                     "latency_ms": {"p50": pct(o["lat"], 50), "p99": pct(o["lat"], 99)},
                     "kernel_ms": kernel_ms(o["prof"]),
                     "roofline": roofline(sim, plan, prec, o["prof"]),
                     "rooflines": stage_rooflines(sim, plan, prec, o["prof"])}
    if other:
        out["other_strategy"] = other
    out.update(extras)
    if not args.no_cpu_baseline:
        out["cpu_baseline"], zo = cpu_baseline(sim)
        if f32_map is not None:
            out["f32_error"] = f32_error(f32_map, f32_rough, zo)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
