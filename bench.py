"""Benchmark of the spin-ice relaxation path on one MI355X.

A step is one field step of the workload's protocol: a full-field pass over
every magnet (dipolar gather of all neighbour pairs, applied and thermal
field, switching keys) followed by the relax to stability.  The default
workload is the ~1.0M-magnet kagome lattice (577 x 577 cells, neighbour
distance 3, thermal std 0.005, rotating field of 0.08, 1000 steps per
revolution): its neighbour tables (~690 MB per pass) exceed the 256 MB
Infinity Cache, so the full-field pass is measured against HBM.

Prints one JSON line.  value = neighbour interactions/s of the whole job:
E (directed neighbour pairs) x steps / wall time, with the relax included.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "neighbour interactions/s & flips/s; batched/served runs/s + p99 vs plain"


def cpu_baseline(w, target_s: float = 15.0):
    """The C++ oracle (single thread) on the first steps of the same
    workload, until about target_s seconds of CPU work."""
    from oracle import native
    o = native.Oracle.from_workload(w)
    E = o.num_edges
    o.set_spins(w.spin0)
    steps = 0
    t0 = time.perf_counter()
    flips = 0
    while time.perf_counter() - t0 < target_s and steps < w.n_steps:
        r = o.run(w.H, steps, steps + 1)
        flips += r["n_flips"]
        steps += 1
    dt = time.perf_counter() - t0
    o.close()
    return dict(value=E * steps / dt, unit="neighbour interactions/s", cores=1, kind="oracle",
                sample=f"first {steps} of {w.n_steps} field steps of {w.name} "
                       f"({flips} flips, {dt:.1f} s, single-threaded C++ oracle)",
                flips_per_s=flips / dt)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="kagome577_rotating")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); independent instances "
              "would shard across GPUs with no communication, which this build does not run.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2002_11401_amd import asi, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = workloads.NAMED[args.workload]()
    K = w.n_steps if args.steps is None else min(args.steps, w.n_steps)
    sim = asi.Sim.from_workload(w)
    info = sim.info()
    E, N = info["n_edges"], info["n"]

    # warmup: the first steps, then back to the start state
    W = min(args.warmup, w.n_steps)
    if W > 0:
        sim.run(0, W)
    sim.set_state(w.spin0, -1)
    sim.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flips = sim.run(0, K)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tm = sim.timing()
    field_avg_s = tm["field_ms"] / max(1, tm["field_launches"]) / 1e3
    achieved = info["field_pass_bytes"] / field_avg_s / 1e9
    out = {
        "metric": METRIC,
        "value": E * K / dt,
        "unit": "neighbour interactions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": dt / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "magnets": N, "neighbour_pairs": E,
                   "max_degree": info["max_degree"], "neighbor_distance": w.neighbor_distance,
                   "thermal_std": w.thermal_std, "protocol_steps": w.n_steps,
                   "parallelism": "single instance, one GPU"},
        "flips_per_s": flips / dt,
        "flips": flips,
        "field_calcs_per_s": N * K / dt,
        "field_pass": {"avg_us": field_avg_s * 1e6, "launches": tm["field_launches"],
                       "algorithmic_bytes": info["field_pass_bytes"]},
        "relax": {"ms_total": tm["relax_ms"], "launches": tm["relax_launches"],
                  "ns_per_flip": tm["relax_ms"] * 1e6 / max(1, flips),
                  "flips_per_s_in_kernel": flips / max(1e-9, tm["relax_ms"] / 1e3)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_field (full-field pass)"},
        "paper_context": {"field_calcs_per_s": 1e8, "hardware": "NVIDIA Tesla V100 32GB",
                          "workload": "square ASI, 8-spin neighbourhood, saturated size"},
    }
    sim.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
