"""Benchmark of the spin-ice relaxation path on one MI355X.

A step is one field step of the workload's protocol: a full-field pass over
every magnet (dipolar gather of all neighbour pairs, applied and thermal
field, switching keys) followed by the relax to stability.

Default (--mode all), three phases, one JSON line:
  1. the ~1.0M-magnet kagome lattice (577 x 577 cells, neighbour distance 3,
     thermal std 0.005, rotating field of 0.08, 1000 steps per revolution):
     W warm-up steps, the whole 2000-step protocol timed once
     (`full_protocol`), then the timed window of K steps whose flips per step
     are nearest the protocol's mean, reached by an untimed prefix.  value =
     neighbour interactions/s of the window, E x K / wall time, relax
     included; `roofline` is the full-field pass of the window (its tables,
     ~690 MB per pass, exceed the 256 MB Infinity Cache); `cpu_baseline` the
     single-threaded oracle on the same workload;
  2. `batched`: the 256-instance sweep, 500 steps, one fused batched launch
     against 256 sequential plain runs, bitwise compared;
  3. `served`: the 2000-job Poisson stream through the continuous-batching
     server in real time (runs/s, p50/p99 latency), against a sample of the
     jobs re-run alone, bitwise compared.
--mode plain / batched / served / analysis runs one phase alone.
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

HBM_PEAK_GBS = 8000.0


T_START = time.perf_counter()


def progress(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)
METRIC = "neighbour interactions/s & flips/s; batched/served runs/s + p99 vs plain"
# degree from which a full-field pass runs one workgroup per 64-row slice
HD_MIN_DEGREE = 128


PROFILE = os.path.join(ROOT, "profiles", "k_field_kagome577_rotating.md")


def field_pass_digest():
    """SHA-256 of the kernel source the full-field pass is built from: the
    device data layout header, then the kernel file's common part and its
    field-phase section."""
    csrc = os.path.join(ROOT, "paper_2002_11401_amd", "csrc")
    hdr = open(os.path.join(csrc, "asi_internal.h")).read()
    txt = open(os.path.join(csrc, "asi_kernels.hip")).read()
    a = txt.index("// ------------------------------------------------------------ neighbours")
    b = txt.index("// ------------------------------------------------------------ field phase")
    c = txt.index("// ------------------------------------------------------------ relax")
    return hashlib.sha256((hdr + txt[:a] + txt[b:c]).encode()).hexdigest()


def recorded_traffic():
    """HBM bytes per full-field pass from the committed counter summary, if it
    was taken with the current kernel source; else None."""
    try:
        rec = {}
        for line in open(PROFILE):
            if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch",
                                                      "field_pass_source_sha256"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
        if rec.get("field_pass_source_sha256") == field_pass_digest():
            return float(rec["traffic_bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        pass
    return None


def host_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(w, a, K, spins_a, gpu_window, reps: int = 3):
    """The C++ oracle, single-threaded, on the same workload: (1) one full
    field evaluation (every row's Eq. 3 sum, then Eq. 2 projected for every
    magnet at step a), the oracle's counterpart of one full-field pass, in
    neighbour interactions/s; (2) flips/s over the GPU's timed window
    [a, a + K), started from the GPU's state at its start, with its flips
    checked against the GPU's."""
    from oracle import native
    t_build = time.perf_counter()
    o = native.Oracle.from_workload(w)
    t_build = time.perf_counter() - t_build
    E = o.num_edges
    evals = []
    for _ in range(reps):
        t0 = time.perf_counter()
        o.set_spins(spins_a)
        o.fields(w.H, a)
        evals.append(time.perf_counter() - t0)
    t_eval = float(np.median(evals))
    o.set_spins(spins_a)
    t0 = time.perf_counter()
    r = o.run(w.H, a, a + K, log_cap=1024)
    dt = time.perf_counter() - t0
    o.close()
    same = (r["n_flips"] == gpu_window["flips"] and r["hash"] == gpu_window["hash"])
    return dict(value=E / t_eval, unit="neighbour interactions/s", cores=1, kind="oracle",
                sample=(f"{w.name}: one full field evaluation at step {a} (median of {reps}, "
                        f"{t_eval:.3f} s), then the GPU's window of steps {a}..{a + K - 1} "
                        f"from the GPU's state ({r['n_flips']} flips, {dt:.1f} s); "
                        f"single-threaded C++ oracle"),
                field_calcs_per_s=w.n / t_eval, full_evaluation_s=t_eval,
                flips_per_s=r["n_flips"] / dt, window_flips=int(r["n_flips"]),
                window_seconds=dt, window_flips_equal_gpu=bool(same),
                oracle_build_s=t_build, host=host_info())


def representative_window(per_step, K):
    """First step of the K consecutive steps whose mean flips per step is
    nearest the whole run's mean (the earliest such window)."""
    ps = np.asarray(per_step, dtype=np.float64)
    if K >= len(ps):
        return 0
    c = np.convolve(ps, np.ones(K) / K, mode="valid")
    return int(np.argmin(np.abs(c - ps.mean())))


def latency_reference(asi):
    """Dependent-load latencies of the device (see asi_measure_load_latency):
    one lane and a 64-lane gather, in the L2 (4 MiB) and in HBM (1 GiB)."""
    out = {}
    for label, nbytes in (("l2_4MiB", 4 << 20), ("hbm_1GiB", 1 << 30)):
        for lanes in (1, 64):
            out[f"{label}_lanes{lanes}_ns"] = asi.load_latency_ns(nbytes, hops=20000, lanes=lanes)
    return out


def bench_plain(args, asi, workloads, torch):
    """One instance, full-field pass every step: W warm-up steps, then the
    whole protocol timed once (full_protocol), then the timed window of K
    steps (value): the K consecutive steps whose flips per step are nearest
    the whole run's mean, reached by an untimed prefix of the protocol."""
    w = workloads.NAMED[args.workload]()
    if args.local_field == "gradient":
        # static spatial field on top of the global one (Sec. II.D): a
        # gradient along x, 0.02 from the centre to the edge, at 200 deg
        span = float(np.ptp(w.xy[:, 0])) / 2
        w.h_loc = workloads.spatial_gradient(w.xy, 0.02 / span, 200.0, 0.0)
    K = min(20 if args.steps is None else args.steps, w.n_steps)
    # every step re-gathers every row: the measured full-field pass
    sim = asi.Sim.from_workload(w, field_mode="full")
    if args.local_field == "wave":
        # a travelling wave evaluated in the pass (Sec. II.D): 0.02 along
        # 200 deg, wavelength 40 lattice units along x, period 500 steps
        sim.set_local_wave(w.xy, 0.02, 1.0 / 40.0, 0.0, 500.0, 0.0, 200.0)
    info = sim.info()
    E, N = info["n_edges"], info["n"]
    Wu = min(args.warmup, w.n_steps)
    if Wu > 0:
        sim.run(0, Wu)
    progress(f"{w.name}: {N} magnets, {E} pairs; warm-up {Wu} steps done")
    if args.no_full_protocol:
        # counter runs: only the first K steps, from the start state
        sim.set_state(w.spin0, -1)
        sim.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        flips = sim.run(0, K)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tm = sim.timing()
        sim.close()
        fa = tm["field_ms"] / max(1, tm["field_launches"]) / 1e3
        return {"metric": METRIC, "value": E * K / dt, "unit": "neighbour interactions/s",
                "steps": K, "flips": flips, "config": {"workload": w.name, "timed_steps": f"0..{K - 1}"},
                "field_pass": {"avg_us": fa * 1e6, "launches": tm["field_launches"],
                               "algorithmic_bytes": info["field_pass_bytes"]},
                "note": "--no-full-protocol: first K steps only (counter runs)"}
    # the whole protocol, timed once
    sim.set_state(w.spin0, -1)
    sim.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flips_all = sim.run(0, w.n_steps)
    torch.cuda.synchronize()
    dt_all = time.perf_counter() - t0
    tm_all = sim.timing()
    per_step = sim.step_flips()
    full = {"steps": w.n_steps, "seconds": dt_all, "flips": flips_all,
            "neighbour_interactions_per_s": E * w.n_steps / dt_all,
            "flips_per_s": flips_all / dt_all, "ms_per_step": dt_all / w.n_steps * 1e3,
            "field_pass_avg_us": tm_all["field_ms"] / max(1, tm_all["field_launches"]) * 1e3,
            "relax_ms": tm_all["relax_ms"],
            "relax_ns_per_flip": tm_all["relax_ms"] * 1e6 / max(1, flips_all),
            "mean_flips_per_step": float(np.mean(per_step)),
            "max_flips_per_step": int(np.max(per_step))}
    progress(f"whole protocol: {flips_all} flips in {dt_all:.2f} s")
    # the timed window, from the state an untimed prefix leaves
    a = representative_window(per_step, K)
    sim.set_state(w.spin0, -1)
    if a > 0:
        sim.run(0, a)
    spins_a = sim.state()[0]
    sim.set_state(spins_a, a - 1)      # the window's own flip log and checksum
    sim.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flips = sim.run(a, a + K)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tm = sim.timing()
    lg = sim.flip_log(cap=0)
    # the same window on the one-flip-at-a-time tree only (no speculation)
    t = sim.tuning()
    sim.set_tuning(t["relax_waves"], t["l1_shift"], 2 ** 62)
    sim.set_state(spins_a, a - 1)
    sim.set_timing(True)
    sim.run(a, a + K)
    tm_tree = sim.timing()
    tree_same = sim.flip_log(cap=0)["hash"] == lg["hash"]
    sim.close()
    field_avg_s = tm["field_ms"] / max(1, tm["field_launches"]) / 1e3
    achieved = info["field_pass_bytes"] / field_avg_s / 1e9
    lat = latency_reference(asi)
    ns_flip = tm["relax_ms"] * 1e6 / max(1, flips)
    ns_flip_tree = tm_tree["relax_ms"] * 1e6 / max(1, flips)
    traffic = (recorded_traffic() if w.name == "kagome577_rotating"
               and args.local_field == "none" else None)
    out = {
        "metric": METRIC,
        "value": E * K / dt,
        "unit": "neighbour interactions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wu,
        "ms_per_step": dt / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "magnets": N, "neighbour_pairs": E,
                   "max_degree": info["max_degree"], "neighbor_distance": w.neighbor_distance,
                   "thermal_std": w.thermal_std, "protocol_steps": w.n_steps,
                   "timed_steps": f"{a}..{a + K - 1}",
                   "field_pass": "full every step", "parallelism": "single instance, one GPU",
                   "local_field": args.local_field},
        "window": {"first_step": a, "steps": K, "flips": flips,
                   "mean_flips_per_step": flips / K,
                   "run_mean_flips_per_step": full["mean_flips_per_step"],
                   "how": "the K consecutive steps whose mean flips per step is nearest the "
                          "whole protocol's mean, reached by an untimed prefix"},
        "flips_per_s": flips / dt,
        "flips": flips,
        "field_calcs_per_s": N * K / dt,
        "full_protocol": full,
        "field_pass": {"avg_us": field_avg_s * 1e6, "launches": tm["field_launches"],
                       "algorithmic_bytes": info["field_pass_bytes"],
                       "neighbour_interactions_per_s": E / field_avg_s,
                       "field_calcs_per_s": N / field_avg_s},
        "relax": {"ms_total": tm["relax_ms"], "launches": tm["relax_launches"],
                  "ns_per_flip": ns_flip,
                  "flips_per_s_in_kernel": flips / max(1e-9, tm["relax_ms"] / 1e3),
                  "tree_only_ns_per_flip": ns_flip_tree,
                  "tree_only_flips_equal": bool(tree_same),
                  "latency_reference_ns": lat,
                  "ns_per_flip_over_l2_gather": ns_flip / lat["l2_4MiB_lanes64_ns"],
                  "tree_ns_per_flip_over_l2_gather": ns_flip_tree / lat["l2_4MiB_lanes64_ns"],
                  "ns_per_flip_over_hbm_load": ns_flip / lat["hbm_1GiB_lanes1_ns"],
                  "tree_ns_per_flip_over_hbm_load": ns_flip_tree / lat["hbm_1GiB_lanes1_ns"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "traffic_source": ({"profile": os.path.relpath(PROFILE, ROOT),
                                         "field_pass_source_sha256": field_pass_digest(),
                                         "measured_in_this_run": False,
                                         "note": "counter bytes per launch from the committed "
                                                 "rocprofv3 --pmc summary, used only while the "
                                                 "kernel source digest matches"}
                                        if traffic is not None else None),
                     "kernel": ("k_field_hd (full-field pass, a workgroup per 64-row slice)"
                                if info["max_degree"] >= HD_MIN_DEGREE
                                else "k_field (full-field pass, a lane per row)")},
        "paper_context": {"field_calcs_per_s": 1e8, "hardware": "NVIDIA Tesla V100 32GB",
                          "workload": "square ASI, 8-spin neighbourhood, saturated size"},
    }
    if not args.no_cpu_baseline and args.local_field != "wave":
        progress("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w, a, K, spins_a, {"flips": flips, "hash": lg["hash"]})
    return out


def bench_analysis(args, asi, workloads, torch):
    """The analyses after the path on paper-scale states: the net
    magnetisation and the spin-spin correlation of the 1M-magnet kagome,
    vertex maps of a 981,400-magnet closed square.  Wall time per call
    (each call copies its result to the host and synchronises); the kernel
    durations come from a kernel trace of this mode."""
    out = {"metric": "analysis calls/s", "unit": "calls/s", "n_gpus": 1, "data": "synthetic",
           "dtype": "f64", "higher_is_better": True, "vs_baseline": None}
    w = workloads.kagome_1m_rotating(n_steps=2)
    sim = asi.Sim.from_workload(w)
    rng = np.random.default_rng(3)
    sim.set_state(rng.choice([-1, 1], w.n).astype(np.int8), -1)
    reps = 50
    sim.magnetization()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.magnetization()
    t_mag = (time.perf_counter() - t0) / reps
    sim.spin_correlation(w.xy, 0.25, 13)
    t0 = time.perf_counter()
    for _ in range(5):
        sums, cnts = sim.spin_correlation(w.xy, 0.25, 13)
    t_corr = (time.perf_counter() - t0) / 5
    info = sim.info()
    sim.close()
    xy, theta = workloads.square_closed(700)
    n = len(theta)
    sq = workloads.Workload("square700", xy, theta, np.ones(n, np.int8), np.full(n, 0.2),
                            np.zeros((2, 2)), alpha=0.001, neighbor_distance=1.0, b=1, c=1,
                            beta=3, gamma=3)
    ptr, idx, _ = workloads.square_vertices(700)
    s2 = asi.Sim.from_workload(sq)
    s2.set_state(rng.choice([-1, 1], n).astype(np.int8), -1)
    s2.group_magnetization(ptr, idx)
    t0 = time.perf_counter()
    for _ in range(5):
        s2.group_magnetization(ptr, idx)
    t_vx = (time.perf_counter() - t0) / 5
    s2.close()
    out.update({"value": 1.0 / t_mag, "steps": reps, "warmup": 1, "ms_per_step": t_mag * 1e3,
                "scaling": "weak",
                "config": {"workload": "kagome577 (998,787 magnets) + square700 (981,400)",
                           "neighbour_pairs": info["n_edges"], "vertices": len(ptr) - 1},
                "magnetization_ms": t_mag * 1e3, "correlation_ms": t_corr * 1e3,
                "correlation_pairs": int(cnts.sum()), "vertex_map_ms": t_vx * 1e3})
    return out


def bench_batched(args, asi, workloads, torch):
    """Uneven sweep of instances: one batched run (one field launch and one
    relax launch per step, replayed from a captured graph) against the same
    instances run one after another with asi_run."""
    K = 500 if args.steps is None or args.mode == "all" else args.steps
    ws = workloads.batched_sweep(count=args.count, seed=4, n_steps=K)
    sims = [asi.Sim.from_workload(w) for w in ws]
    ntot = sum(w.n for w in ws)
    etot = sum(s.info()["n_edges"] for s in sims)
    # autotuned launch shapes per instance (state restored exactly), used by
    # both the sequential and the batched runs
    shapes = {}
    t_tune = 0.0
    if args.tune_steps > 0:
        t0 = time.perf_counter()
        for s in sims:
            r = s.tune(args.tune_steps)
            key = f"waves{r['relax_waves']}/l1s{r['l1_shift']}/spec_min{min(r['spec_min'], 10**9)}"
            shapes[key] = shapes.get(key, 0) + 1
        t_tune = time.perf_counter() - t0
        progress(f"tuned {len(sims)} instances in {t_tune:.1f}s: {shapes}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = []
    for k, s in enumerate(sims):
        s.run()
        plain.append(s.flip_log(cap=0))
        if k % 32 == 31:
            progress(f"plain {k + 1}/{len(sims)} {time.perf_counter() - t0:.1f}s")
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    plain_spins = [s.state()[0] for s in sims]
    for s, w in zip(sims, ws):
        s.set_state(w.spin0, -1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flips = asi.batch_run(sims, mode=args.batch_mode)
    torch.cuda.synchronize()
    t_bat = time.perf_counter() - t0
    same = all(s.flip_log(cap=0)["hash"] == p["hash"] and np.array_equal(s.state()[0], sp)
               for s, p, sp in zip(sims, plain, plain_spins))
    for s in sims:
        s.close()
    return {"metric": METRIC, "value": len(ws) / t_bat, "unit": "runs/s", "n_gpus": 1,
            "steps": K, "warmup": 0, "ms_per_step": t_bat / K * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"batched sweep of {len(ws)} square/pinwheel instances",
                       "batch_mode": args.batch_mode,
                       "magnets_total": ntot, "neighbour_pairs_total": etot,
                       "parallelism": "one launch per phase over all instances"},
            "batched_runs_per_s": len(ws) / t_bat, "plain_runs_per_s": len(ws) / t_seq,
            "speedup_vs_plain": t_seq / t_bat, "plain_seconds": t_seq, "batched_seconds": t_bat,
            "flips": int(flips.sum()), "bitwise_identical_to_plain": bool(same),
            "autotune": {"sample_steps": args.tune_steps, "seconds": t_tune, "shapes": shapes}}


def bench_served(args, asi, workloads, torch):
    """Poisson stream of jobs into the continuous-batching server, in real
    time; latency = completion - arrival.  The plain rate comes from a seeded
    uniform sample of the jobs, each re-run alone with asi_run (and checked
    bitwise against its served result)."""
    jobs = workloads.served_stream(count=args.jobs, seed=5, rate_per_s=args.rate,
                                   n_range=(1e3, args.max_n))
    progress(f"generating {len(jobs)} job inputs")
    wls = {j.job: j.workload() for j in jobs}
    srv = asi.Server(hbm_budget_bytes=int(args.budget_gb * (1 << 30)), max_slots=args.slots)
    ids = {}
    open_ids = {}
    lat = {}
    t0 = time.perf_counter()
    pending = list(jobs)
    active = 0
    last = t0
    while pending or active:
        if time.perf_counter() - last > 10:
            last = time.perf_counter()
            progress(f"served: {len(lat)}/{len(jobs)} done, {active} active, "
                     f"{last - t0:.1f}s")
        now = time.perf_counter() - t0
        while pending and pending[0].arrival_s <= now:
            j = pending.pop(0)
            ids[j.job] = open_ids[j.job] = srv.submit(wls[j.job])
        active = srv.step(args.burst_ms)
        for job, jid in list(open_ids.items()):
            if srv.poll(jid):
                lat[job] = time.perf_counter() - t0
                del open_ids[job]
        if not active and pending:
            time.sleep(max(0.0, pending[0].arrival_s - (time.perf_counter() - t0)))
    t_all = time.perf_counter() - t0
    res = {job: srv.take(jid) for job, jid in ids.items()}
    stats = srv.stats()
    srv.close()
    lats = np.array([lat[j.job] - j.arrival_s for j in jobs])
    for j in sorted(jobs, key=lambda j: res[j.job]["t_admit"] - res[j.job]["t_done"])[:5]:
        r = res[j.job]
        progress(f"slow job {j.job} {j.family} n={wls[j.job].n} d={j.d:g} steps={j.n_steps} "
                 f"flips={r['flips']} served={r['t_done'] - r['t_admit']:.3f}s")
    # plain rate from a seeded uniform sample, each job alone; the sample
    # stops early once the whole benchmark has used its time budget
    rng = np.random.default_rng(55)
    k = min(args.plain_sample, len(jobs))
    sample = sorted(rng.choice(len(jobs), size=k, replace=False).tolist())
    same = True
    times = []
    t1 = time.perf_counter()
    for c, q in enumerate(sample):
        if c >= 8 and time.perf_counter() - T_START > args.time_budget_s:
            progress(f"plain sample stopped at {c}/{k} jobs: time budget "
                     f"{args.time_budget_s:.0f}s reached")
            sample = sample[:c]
            break
        j = jobs[q]
        w = wls[j.job]
        torch.cuda.synchronize()
        ts = time.perf_counter()
        s = asi.Sim.from_workload(w, device="hip")
        s.run()
        lg = s.flip_log(cap=0)
        spins = s.state()[0]
        s.close()
        times.append(time.perf_counter() - ts)
        same &= lg["hash"] == res[j.job]["hash"] and np.array_equal(spins, res[j.job]["spins"])
        r = res[j.job]
        progress(f"job {j.job} {j.family} n={w.n} d={j.d:g} steps={j.n_steps} "
                 f"flips={lg['count']} plain={times[-1]:.3f}s "
                 f"served={r['t_done'] - r['t_admit']:.3f}s")
        if c % 10 == 9:
            progress(f"plain sample {c + 1}/{k} {time.perf_counter() - t1:.1f}s")
    mean_plain = float(np.mean(times))
    return {"metric": METRIC, "value": len(jobs) / t_all, "unit": "runs/s", "n_gpus": 1,
            "steps": int(sum(j.n_steps for j in jobs)), "warmup": 0,
            "ms_per_step": t_all / max(1, sum(j.n_steps for j in jobs)) * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"Poisson stream of {len(jobs)} jobs at {args.rate}/s, "
                                   f"1e3..{args.max_n:g} magnets, square/pinwheel/kagome",
                       "slots": args.slots, "hbm_budget_gb": args.budget_gb,
                       "burst_ms": args.burst_ms,
                       "parallelism": "continuous batching, one GPU"},
            "served_runs_per_s": len(jobs) / t_all, "served_seconds": t_all,
            "plain_runs_per_s": 1.0 / mean_plain,
            "plain_sample": {"jobs": len(times), "asked": k, "mean_s": mean_plain,
                             "max_s": float(np.max(times)), "seed": 55,
                             "how": "uniform sample, each job alone with asi_run"},
            "speedup_vs_plain": (len(jobs) / t_all) * mean_plain,
            "latency_s": {"p50": float(np.percentile(lats, 50)),
                          "p99": float(np.percentile(lats, 99)), "max": float(lats.max())},
            "bitwise_identical_to_plain": bool(same), "bitwise_checked_jobs": len(times),
            "server_stats": stats}


def _oracle_instance(spec):
    """One sweep instance's whole protocol on the single-threaded oracle
    (process-pool worker): (index, seconds, flips, neighbour pairs)."""
    k, K = spec
    from oracle import native
    from paper_2002_11401_amd import workloads
    w = workloads.batched_sweep(count=256, seed=4, n_steps=K)[k]
    t0 = time.perf_counter()
    o = native.Oracle.from_workload(w)
    o.set_spins(w.spin0)
    r = o.run(w.H, 0, w.n_steps, log_cap=1024)
    dt = time.perf_counter() - t0
    E = o.num_edges
    o.close()
    return k, dt, int(r["n_flips"]), E


def bench_oracle(args, asi, workloads, torch):
    """CPU baseline table: the single-threaded C++ oracle on this machine's
    host cores.  For the square 10 x 10, the 100 x 100 pinwheel and the 1M
    kagome: one full field evaluation (neighbour interactions/s, median of
    3) and the whole protocol (wall time, flips/s, printed in chunks of
    steps).  For the 256-instance sweep: every instance's whole protocol in
    a process pool over the host cores (per-instance single-core seconds
    and the pool's aggregate runs/s)."""
    import multiprocessing as mp
    from oracle import native
    out = {"metric": "oracle baseline (CPU, single-threaded per instance)", "host": host_info(),
           "configs": {}}
    try:
        import subprocess
        out["host"]["lscpu"] = [ln for ln in subprocess.run(
            ["lscpu"], capture_output=True, text=True, timeout=30).stdout.splitlines()
            if ln.split(":")[0] in ("Model name", "CPU(s)", "Thread(s) per core",
                                    "Core(s) per socket", "Socket(s)", "CPU max MHz",
                                    "L3 cache", "NUMA node(s)")]
    except Exception:  # noqa: BLE001 - informational only
        pass
    for name in ("square10_triangle", "pinwheel100_reversal", "kagome577_rotating"):
        w = workloads.NAMED[name]()
        t0 = time.perf_counter()
        o = native.Oracle.from_workload(w)
        t_build = time.perf_counter() - t0
        E = o.num_edges
        evals = []
        for _ in range(3):
            t0 = time.perf_counter()
            o.set_spins(w.spin0)
            o.fields(w.H, 0)
            evals.append(time.perf_counter() - t0)
        t_eval = float(np.median(evals))
        o.set_spins(w.spin0)
        flips, fnv = 0, native.FNV_OFFSET
        chunk = max(1, w.n_steps // 20)
        t0 = time.perf_counter()
        for a in range(0, w.n_steps, chunk):
            r = o.run(w.H, a, min(w.n_steps, a + chunk), log_cap=1024, fnv=fnv)
            flips += int(r["n_flips"])
            fnv = r["hash"]
            progress(f"oracle {name}: steps ..{min(w.n_steps, a + chunk)} flips {flips} "
                     f"{time.perf_counter() - t0:.1f}s")
        dt = time.perf_counter() - t0
        o.close()
        out["configs"][name] = {"magnets": w.n, "neighbour_pairs": E, "steps": w.n_steps,
                                "build_s": t_build, "full_evaluation_s": t_eval,
                                "neighbour_interactions_per_s": E / t_eval,
                                "field_calcs_per_s": w.n / t_eval,
                                "whole_run_s": dt, "flips": flips, "flips_per_s": flips / dt,
                                "flip_hash": str(fnv)}
    K = 500
    procs = min(args.oracle_procs, os.cpu_count() or 1)
    specs = [(k, K) for k in range(args.count)]
    t0 = time.perf_counter()
    per = {}
    with mp.get_context("fork").Pool(procs) as pool:
        for k, dt, nf, E in pool.imap_unordered(_oracle_instance, specs):
            per[k] = (dt, nf, E)
            if len(per) % 16 == 0:
                progress(f"oracle sweep {len(per)}/{len(specs)} {time.perf_counter() - t0:.1f}s")
    wall = time.perf_counter() - t0
    secs = np.array([per[k][0] for k in sorted(per)])
    out["configs"]["batched_sweep"] = {
        "instances": len(per), "steps": K, "processes": procs,
        "pool_wall_s": wall, "pool_runs_per_s": len(per) / wall,
        "single_core_sum_s": float(secs.sum()),
        "single_core_runs_per_s": len(per) / float(secs.sum()),
        "per_instance_s": {"min": float(secs.min()), "median": float(np.median(secs)),
                           "max": float(secs.max())},
        "flips": int(sum(v[1] for v in per.values())),
        "neighbour_pairs": int(sum(v[2] for v in per.values()))}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--mode", choices=["all", "plain", "batched", "served", "analysis", "oracle"],
                    default="all")
    ap.add_argument("--workload", default="kagome577_rotating")
    ap.add_argument("--local-field", default="none", choices=["none", "gradient", "wave"],
                    help="plain: add a static spatial field, or a travelling wave "
                         "evaluated on the device (no CPU baseline for the wave)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-full-protocol", action="store_true",
                    help="plain: time only the first K steps (for counter runs)")
    ap.add_argument("--count", type=int, default=256, help="batched: instances")
    ap.add_argument("--oracle-procs", type=int, default=16,
                    help="oracle: worker processes for the sweep (at most the host's cores)")
    ap.add_argument("--batch-mode", default="fused", choices=["lockstep", "graph", "fused"])
    ap.add_argument("--tune-steps", type=int, default=20,
                    help="batched: autotune each instance on this many steps (0: off)")
    ap.add_argument("--jobs", type=int, default=2000, help="served: jobs")
    ap.add_argument("--plain-sample", type=int, default=32, help="served: jobs re-run alone")
    ap.add_argument("--time-budget-s", type=float, default=480.0,
                    help="served: stop the plain sample (after at least 8 jobs) once the "
                         "benchmark has run this long")
    ap.add_argument("--rate", type=float, default=50.0, help="served: arrivals per second")
    ap.add_argument("--max-n", type=float, default=1e6, help="served: largest job")
    ap.add_argument("--slots", type=int, default=256, help="served: resident jobs")
    ap.add_argument("--budget-gb", type=float, default=240.0, help="served: HBM budget")
    ap.add_argument("--burst-ms", type=float, default=20.0, help="served: device time per step")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library drives one "
              "device per process; independent instances would shard across GPUs with no "
              "communication, but no multi-GPU path is implemented.", file=sys.stderr)
        sys.exit(2)

    from paper_2002_11401_amd import workloads
    if args.mode == "oracle":
        # host cores only: the GPU is not touched (the pool forks)
        print(json.dumps(bench_oracle(args, None, workloads, None)), flush=True)
        return
    import torch
    from paper_2002_11401_amd import asi

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.mode != "all":
        fn = {"plain": bench_plain, "batched": bench_batched, "served": bench_served,
              "analysis": bench_analysis, "oracle": bench_oracle}[args.mode]
        print(json.dumps(fn(args, asi, workloads, torch)), flush=True)
        return
    # the default: the 1M-magnet kagome (value and roofline), then the
    # batched sweep and the served stream, each against its plain runs
    t_all = time.perf_counter()
    out = bench_plain(args, asi, workloads, torch)
    progress(f"plain done at {time.perf_counter() - t_all:.1f}s")
    contract = ("metric", "n_gpus", "steps", "warmup", "higher_is_better", "scaling",
                "vs_baseline", "data")
    for mode, fn in (("batched", bench_batched), ("served", bench_served)):
        torch.cuda.empty_cache()     # the previous phase's memory back to the device
        r = fn(args, asi, workloads, torch)
        out[mode] = {k: v for k, v in r.items() if k not in contract}
        progress(f"{mode} done at {time.perf_counter() - t_all:.1f}s")
    out["bench_seconds"] = time.perf_counter() - t_all
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
