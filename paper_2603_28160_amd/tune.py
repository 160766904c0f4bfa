"""Measure launch parameters for the standard workloads and save the tuning table.

    python -m paper_2603_28160_amd.tune [--out FILE] [--quick]

Runs fsm_autotune (the library's autotuner) on the benchmark workloads in both precisions, on
device 0, and writes the context's tuning table as JSON.  A context loads it with
Context.load_tuning(FILE); calls whose workload class (precision, number of simulations,
orders of magnitude of cells and evaluations) matches an entry then use its parameters.  The
table is specific to the device type it was measured on.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuning_mi355x.json")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true", help="only the 5000 x 5000 workload")
    args = ap.parse_args(argv)

    import torch
    from paper_2603_28160_amd import Context, workloads as W

    jobs = [("config2", [W.config2()]), ("config1", [W.config1()])]
    if not args.quick:
        jobs += [("config3_mix_256", W.config3(256)),
                 ("config5", [W.config5()])]
        jobs += [(f"paper_condition{no}", [W.paper_mode(no)]) for no in range(1, 10)]
    done = []
    with Context(0) as ctx:
        for name, sims in jobs:
            for prec in ("f64", "f32"):
                zmaps = [ctx.new_zmap(s.grid, prec) for s in sims]
                t0 = time.perf_counter()
                r = ctx.fsm_autotune(sims, prec, zmaps=zmaps)
                print(f"[tune] {name} {prec}: {r} ({time.perf_counter() - t0:.1f} s)",
                      file=sys.stderr, flush=True)
                done.append({"workload": name, "precision": prec, **r})
                del zmaps
                torch.cuda.empty_cache()
        table = ctx.fsm_tune_get()
    out = {"device": torch.cuda.get_device_name(0),
           "command": "python -m paper_2603_28160_amd.tune" + (" --quick" if args.quick else ""),
           "entries": table, "measured": done}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(f"[tune] {len(table)} entries -> {args.out}", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
