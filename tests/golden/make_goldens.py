"""Write the expected results of the paper-scale parity cases from the oracle.

    python tests/golden/make_goldens.py {kagome577,sweep,served,all} [--workers N]

Every value stored here comes from the tier-1 CPU oracle (oracle/relax.cpp)
running the seeded inputs of paper_2002_11401_amd/workloads.py; nothing
comes from the HIP library.  The relax is the one of Sec. II.H: at every
field step, flip the flippable magnet with the largest left-hand side of
Eq. 5 (ties: lowest index) until none is left.

Outputs (JSON, one per case, beside this script):
  kagome577_rotating.json   the whole 2000-step protocol of the ~1M-magnet
                            kagome with thermal noise: flip count, flip-log
                            checksum, per-step flip counts, SHA-256 of the
                            final spins, decision gaps per step
  batched_sweep_sample.json 16 instances of the 256-instance sweep (seed 4,
                            500 steps): the 8 largest plus 8 drawn with
                            numpy default_rng(44) from the rest
  served_stream_sample.json 64 jobs of the 2000-job stream (seed 5): the jobs
                            sorted by size and split into 64 strata of
                            consecutive sizes, one job per stratum drawn with
                            default_rng(2024), the largest job standing in
                            for the draw of the top stratum

A rerun keeps the entries already present in an output file (so an
interrupted run resumes); --fresh starts over.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import native as N  # noqa: E402
from paper_2002_11401_amd import workloads as W  # noqa: E402

OUT = {"kagome577": os.path.join(HERE, "kagome577_rotating.json"),
       "sweep": os.path.join(HERE, "batched_sweep_sample.json"),
       "served": os.path.join(HERE, "served_stream_sample.json")}

SWEEP = dict(count=256, seed=4, n_steps=500)
SWEEP_RANDOM_SEED = 44
SERVED = dict(count=2000, seed=5)
SERVED_STRATA = 64
SERVED_DRAW_SEED = 2024


def spins_sha256(s) -> str:
    return hashlib.sha256(np.ascontiguousarray(s, dtype=np.int8).tobytes()).hexdigest()


_sweep = None


def sweep():
    global _sweep
    if _sweep is None:
        _sweep = W.batched_sweep(**SWEEP)
    return _sweep


def sweep_selection():
    """Indices of the sampled instances of the sweep, largest first."""
    ws = sweep()
    ns = np.array([w.n for w in ws])
    order = sorted(range(len(ws)), key=lambda k: (-ns[k], k))
    largest = order[:8]
    rest = sorted(order[8:])
    drawn = np.random.default_rng(SWEEP_RANDOM_SEED).choice(rest, size=8, replace=False)
    return largest + sorted(int(k) for k in drawn)


def served_selection():
    """Job numbers of the stratified sample of the stream."""
    jobs = W.served_stream(**SERVED)
    order = sorted(range(len(jobs)), key=lambda k: (jobs[k].n_target, k))
    rng = np.random.default_rng(SERVED_DRAW_SEED)
    strata = np.array_split(np.array(order), SERVED_STRATA)
    pick = [int(rng.choice(s)) for s in strata]
    pick[-1] = order[-1]
    return pick


def run_oracle(w):
    """Whole protocol of workload w on the oracle."""
    t0 = time.perf_counter()
    o = N.Oracle.from_workload(w)
    o.set_spins(w.spin0)
    r = o.run(w.H, 0, w.n_steps, log_cap=1024)
    out = dict(name=w.name, n=w.n, n_edges=o.num_edges, steps=w.n_steps,
               status=r["status"], flips=int(r["n_flips"]), hash=str(r["hash"]),
               spins_sha256=spins_sha256(o.spins()),
               per_step=[int(v) for v in r["per_step"]],
               min_top2_rel=float(r["gaps"]["top2_rel"]),
               min_thresh_rel=float(r["gaps"]["thresh_rel"]),
               step_top2=[None if not np.isfinite(v) else float(v) for v in r["step_top2"]])
    o.close()
    out["oracle_seconds"] = round(time.perf_counter() - t0, 1)
    return out


def task(spec):
    kind, key = spec
    if kind == "kagome577":
        w = W.kagome_1m_rotating()
    elif kind == "sweep":
        w = sweep()[key]
    else:
        w = W.served_stream(**SERVED)[key].workload()
    r = run_oracle(w)
    if kind == "served":
        # per-step detail is not kept for the served jobs: counts and checksum
        r.pop("per_step")
        r.pop("step_top2")
    elif kind == "sweep":
        r.pop("step_top2")
    return kind, key, r


def cost(spec):
    kind, key = spec
    if kind == "kagome577":
        return 1e12
    if kind == "sweep":
        w = sweep()[key]
        return w.n * w.n_steps * (1 + w.neighbor_distance ** 2)
    j = W.served_stream(**SERVED)[key]
    return j.n_target * j.n_steps * (1 + j.d ** 2)


def load(kind):
    try:
        with open(OUT[kind]) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None


def header(kind):
    cmd = "python tests/golden/make_goldens.py " + kind
    if kind == "kagome577":
        return dict(case="kagome577_rotating: 577 x 577 kagome cells, 2000 steps",
                    source="tier-1 oracle (oracle/relax.cpp), whole protocol", command=cmd)
    if kind == "sweep":
        return dict(case="batched_sweep(count=256, seed=4, n_steps=500)",
                    selection=f"8 largest, then 8 of the rest by default_rng({SWEEP_RANDOM_SEED})",
                    source="tier-1 oracle (oracle/relax.cpp), whole protocol of each",
                    command=cmd, instances={})
    return dict(case="served_stream(count=2000, seed=5)",
                selection=(f"{SERVED_STRATA} size strata, one job each by "
                           f"default_rng({SERVED_DRAW_SEED}), the largest job in the top one"),
                source="tier-1 oracle (oracle/relax.cpp), whole protocol of each",
                command=cmd, jobs={})


def save(kind, doc):
    tmp = OUT[kind] + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, OUT[kind])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["kagome577", "sweep", "served", "all"])
    ap.add_argument("--workers", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    ap.add_argument("--fresh", action="store_true")
    args = ap.parse_args()
    kinds = ["kagome577", "sweep", "served"] if args.which == "all" else [args.which]
    docs, specs = {}, []
    for kind in kinds:
        doc = None if args.fresh else load(kind)
        docs[kind] = doc if doc else header(kind)
        if kind == "kagome577":
            if "flips" not in docs[kind]:
                specs.append((kind, 0))
        elif kind == "sweep":
            have = docs[kind]["instances"]
            specs += [(kind, k) for k in sweep_selection() if str(k) not in have]
        else:
            have = docs[kind]["jobs"]
            specs += [(kind, k) for k in served_selection() if str(k) not in have]
    specs.sort(key=cost, reverse=True)
    print(f"{len(specs)} oracle runs, {args.workers} workers", flush=True)
    N.build(force=False)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(args.workers, maxtasksperchild=1) as pool:
        for kind, key, r in pool.imap_unordered(task, specs):
            if kind == "kagome577":
                docs[kind].update(r)
            elif kind == "sweep":
                docs[kind]["instances"][str(key)] = r
            else:
                docs[kind]["jobs"][str(key)] = r
            save(kind, docs[kind])
            print(f"[{time.perf_counter() - t0:7.1f}s] {kind} {key} {r['name']} n={r['n']} "
                  f"E={r['n_edges']} flips={r['flips']} oracle {r['oracle_seconds']}s",
                  flush=True)


if __name__ == "__main__":
    main()
