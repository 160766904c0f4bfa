"""Benchmark: Z-map cells/s of the full simulation (edge discretisation, kinematics, binning,
per-cell minimum, roughness) on the 5000 x 5000 ball-end raster workload, one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one fsm_simulate call: plan tables to the device, Z-map fill, scatter kernel,
two roughness passes and the result back on the host; the Z-map stays resident in HBM.
Prints one JSON line.  The dominant kernel's duration comes from HIP events the library
records on the stream it launches on.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Z-map cells/s and simulations/s (p50/p99 latency), FP32 batched vs FP64 plain"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6        # MI355X vector FP64
BYTES_PER_UPDATE = {"f64": 8, "f32": 4}   # one encoded-height compare/min-update per binned point


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def run_precision(ctx, sim, prec, steps, warmup):
    import torch
    zmap = ctx.new_zmap(sim.grid, prec)
    ctx.fsm_ctx_set_profiling(True)
    for _ in range(warmup):
        ctx.fsm_simulate(sim, prec, zmap)
    torch.cuda.synchronize()
    lat, scat, rough_ms, fill_ms = [], [], [], []
    t0 = time.perf_counter()
    r = None
    for _ in range(steps):
        a = time.perf_counter()
        _, r = ctx.fsm_simulate(sim, prec, zmap)
        lat.append((time.perf_counter() - a) * 1e3)
        t = ctx.fsm_last_timings()
        scat.append(t["scatter_ms"])
        rough_ms.append(t["rough_ms"])
        fill_ms.append(t["fill_ms"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"elapsed_s": el, "ms_per_step": el / steps * 1e3, "lat": lat,
            "scatter_ms": statistics.mean(scat), "rough_ms": statistics.mean(rough_ms),
            "fill_ms": statistics.mean(fill_ms), "rough": r}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["f64", "f32", "both"], default="both")
    ap.add_argument("--strategy", choices=["binned", "scatter"], default="binned")
    ap.add_argument("--compare-strategies", action="store_true",
                    help="also time the other Z-map strategy (reported, not the value)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (reads 1 GiB, writes "
                         "1 GiB) five times, to scale HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(simulations shard across GPUs without communication; see the design notes)",
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
        precs = ["f64", "f32"] if args.precision == "both" else [args.precision]
        other = {}
        if args.compare_strategies:
            alt = "scatter" if args.strategy == "binned" else "binned"
            ctx.set_strategy(alt)
            for prec in precs:
                o = run_precision(ctx, sim, prec, args.steps, args.warmup)
                other[prec] = {"ms_per_step": o["ms_per_step"], "zmap_ms": o["scatter_ms"]}
                print(f"[bench] {alt} {prec}: {o['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
        ctx.set_strategy(args.strategy)
        for prec in precs:
            print(f"[bench] {sim.name} {prec}: warmup {args.warmup}, steps {args.steps}",
                  file=sys.stderr, flush=True)
            res[prec] = run_precision(ctx, sim, prec, args.steps, args.warmup)
            print(f"[bench] {prec}: {res[prec]['ms_per_step']:.3f} ms/step, scatter "
                  f"{res[prec]['scatter_ms']:.3f} ms", file=sys.stderr, flush=True)

    main_prec = "f64" if "f64" in res else precs[0]
    m = res[main_prec]
    r = m["rough"]
    n_binned = r["n_binned"]
    upd_bytes = n_binned * BYTES_PER_UPDATE[main_prec]
    achieved = upd_bytes / (m["scatter_ms"] * 1e-3) / 1e9
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
                   "zmap_strategy": args.strategy},
        "sims_per_s": args.steps / m["elapsed_s"],
        "latency_ms": {"p50": pct(m["lat"], 50), "p99": pct(m["lat"], 99)},
        "evals_per_s": plan["n_evals"] * args.steps / m["elapsed_s"],
        "coverage": r["n_hit"] / n_cells,
        "kernel_ms": {"fill": m["fill_ms"], "zmap": m["scatter_ms"], "roughness": m["rough_ms"]},
        "roofline": {"bound": "hbm", "kernel": "scatter", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None,
                     "algorithmic_bytes": upd_bytes, "n_binned": n_binned},
    }
    for prec in res:
        if prec == main_prec:
            continue
        o = res[prec]
        out[prec] = {"value": n_cells * args.steps / o["elapsed_s"], "unit": "cells/s",
                     "ms_per_step": o["ms_per_step"],
                     "latency_ms": {"p50": pct(o["lat"], 50), "p99": pct(o["lat"], 99)},
                     "kernel_ms": {"fill": o["fill_ms"], "zmap": o["scatter_ms"],
                                   "roughness": o["rough_ms"]},
                     "Sa": o["rough"]["Sa"], "Sa_f64": r["Sa"]}
    if other:
        out["other_strategy"] = other
    if not args.no_cpu_baseline:
        import oracle
        print("[bench] cpu baseline: FP64 oracle on the full workload, 1 thread",
              file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        oracle.simulate(sim)
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n_cells / el, "unit": "cells/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"full {sim.name} FP64, one simulation, {el:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
