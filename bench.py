#!/usr/bin/env python3
"""Benchmark of the Independent-algorithm hot path on one MI355X.

A step is one complete simulate of the plain form on the spatially explicit
workload (256 x 256 torus, one individual per cell, Gaussian sigma = 2 on a
21 x 21 kernel, nu = 1e-3, all 65,536 individuals sampled): lineage init,
horizon rounds (event sampling, dispersal, culling, compaction), output and
richness -- every kernel of the path, on inputs already resident in HBM.  The
scenario tables are built once (they are the scenario, like model weights);
each step uses its own seed.

Before timing, the round kernels' performance knobs (launch form included) are
autotuned on this workload (results never depend on them).  Prints one JSON
line: lineage events/s (value), individuals/s, the round kernel's VALU roofline
fraction (HIP events on the library's stream) and its serial bound, and beside
them: the batched form (the 256-scenario mix in one run, knobs tuned on the mix,
median of several runs, its own roofline, vs one scenario per run), the served
form (a Poisson request stream through the continuous-batching server after a
warm-up: p50/p99 latency, throughput, HBM budget, the slowest request against
its run alone, vs the same requests one per run), the heterogeneous habitat
(per-deme tables gathered from HBM), and the CPU oracle: single-threaded on a
bounded sample of the plain workload and one process per host core on the mix.
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

METRIC = "lineage events/s & individuals/s vs CPU oracle; serve p50/p99 latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="bound on the oracle baseline's CPU time")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "k_run_c2_traffic.txt"),
                    help="HBM bytes per round launch from rocprofv3 FETCH_SIZE/WRITE_SIZE runs")
    ap.add_argument("--no-tune", action="store_true", help="use the library defaults instead of autotuning")
    ap.add_argument("--knobs", default=None, help="JSON dict of tuned knobs to use instead of autotuning")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched (C4) and served (C5) forms")
    ap.add_argument("--batch-plain-subset", type=int, default=32,
                    help="scenarios of the 256-scenario mix also run one per launch for the comparison")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="length of the served request stream")
    ap.add_argument("--serve-warmup", type=float, default=5.0,
                    help="served seconds before the measured stream (same rate, other requests; not measured)")
    ap.add_argument("--serve-hbm-frac", type=float, default=0.8, help="serving budget as a fraction of free HBM")
    ap.add_argument("--serve-plain", type=int, default=32, help="requests of the stream also run one per launch")
    ap.add_argument("--batch-runs", type=int, default=5, help="timed runs of the batched form (median)")
    ap.add_argument("--no-batch-tune", action="store_true", help="batched form on library defaults")
    ap.add_argument("--cpu-c4-seconds", type=float, default=15.0,
                    help="bound on the N-process oracle's wall time over the 256-scenario mix")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the heterogeneous-habitat workload (1024x1024 fractal map, per-deme tables, "
                         "10%% sample, nu = 1e-5)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (calibrates rocprofv3 FETCH/WRITE_SIZE)")
    ap.add_argument("--event-stream", action="store_true",
                    help="only run the event-stream form on the 256x256 torus and print its JSON (for profiling)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the batched form (256-scenario mix) once per --batch-runs and print its JSON "
                         "(for profiling; --batch-knobs fixes its knobs)")
    ap.add_argument("--batch-knobs", default=None, help="JSON dict of knobs for the batched form instead of tuning")
    ap.add_argument("--profile-summary", default=None, metavar="DB",
                    help="only summarise a rocprofv3 results database (no GPU): per-kernel trace statistics, and "
                         "per-dispatch counter sums of the kernels matching --profile-kernel")
    ap.add_argument("--profile-kernel", default="k_run|k_round", help="kernel-name regex for --profile-summary")
    return ap.parse_args()


def note(*a):
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def traffic_from_profile(path: str) -> float | None:
    """HBM bytes per round launch recorded from rocprofv3 FETCH_SIZE and WRITE_SIZE runs, or None when
    the kernel source has changed since they were taken."""
    import hashlib
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2108_05815_amd", "csrc", "necsim_hip.hip")
    with open(src, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    if fields.get("kernel_source_sha256") != digest:
        return None
    return float(fields["bytes_per_launch"])


def chain_events(ev, co) -> int:
    """The longest serial chain of the run, in events, read from the event stream: the most events
    on any sample's path to its speciation.  An event's predecessors are the arrival named by its
    prior event time and origin, and the arrivals of the lineages that coalesced there during
    that stay (the coalescences at its origin whose parent arrived at its prior event time); the
    stream is sorted by time, so one pass computes every event's depth."""
    from collections import defaultdict
    t, prior, origin, outcome = (ev["t"].tolist(), ev["t_prior"].tolist(), ev["origin"].tolist(),
                                 ev["outcome"].tolist())
    arrival = {(t[i], outcome[i]): i for i in range(len(t)) if outcome[i] != 0xFFFFFFFF}
    joined = defaultdict(list)
    for tc, tp, loc in zip(co["t"].tolist(), co["t_parent"].tolist(), co["loc"].tolist()):
        joined[(loc, tp)].append(tc)
    depth = [0] * len(t)
    best = 0
    for i in range(len(t)):
        d = depth[arrival[(prior[i], origin[i])]] if prior[i] > 0.0 else 0
        for tc in joined.get((origin[i], prior[i]), ()):
            d = max(d, depth[arrival[(tc, origin[i])]])
        depth[i] = d + 1
        if outcome[i] == 0xFFFFFFFF:
            best = max(best, depth[i])
    return best


def horizon_table(cfg, t_max: float) -> list:
    """The horizons of a single-job run, as the library builds them from the config (same defaults
    for unset fields): h[0] = 0, h[1] = horizon0, then steps of min(step_max, h (growth - 1));
    past the library's 1024 entries its last step repeats."""
    h0 = cfg.horizon0 if cfg.horizon0 > 0 else 0.5
    g = cfg.horizon_growth if cfg.horizon_growth > 1.0 else 1.25
    smax = cfg.horizon_step_max if cfg.horizon_step_max > 0 else 4096.0
    h = [0.0, h0]
    while h[-1] < t_max:
        step = min(smax, h[-1] * (g - 1.0)) if len(h) < 1024 else h[1023] - h[1022]
        h.append(h[-1] + step)
    return h


def window_maxima(ev, co, horizons) -> list:
    """Per horizon window (h[k], h[k+1]]: the most events one lineage entering the window commits
    inside it; the round of that window cannot end sooner.  A lineage's path is followed through
    the stream: after an arrival comes the event at that location whose prior event time is the
    arrival's time, or, for an arrival that coalesced there, the event of the lineage it joined.
    A window's entries are the events whose earliest prior event time lies before it."""
    t = ev["t"]
    tl, pl, ol, xl = t.tolist(), ev["t_prior"].tolist(), ev["origin"].tolist(), ev["outcome"].tolist()
    first = {(pl[i], ol[i]): i for i in range(len(tl))}
    joined = {(tc, loc): tp for tc, tp, loc in zip(co["t"].tolist(), co["t_parent"].tolist(), co["loc"].tolist())}
    h = np.asarray(horizons, dtype=np.float64)
    k = (np.searchsorted(h, t, side="left") - 1).tolist()
    cnt = [0] * len(tl)
    for i in range(len(tl) - 1, -1, -1):  # successors come later in time order
        c = 1
        if xl[i] != 0xFFFFFFFF:
            key = (tl[i], xl[i])
            j = first.get(key)
            if j is None:
                j = first[(joined[key], xl[i])]
            if k[j] == k[i]:
                c += cnt[j]
        cnt[i] = c
    m = [0] * ((max(k) + 1) if k else 0)
    for i in range(len(tl)):
        if pl[i] <= h[k[i]] and cnt[i] > m[k[i]]:
            m[k[i]] = cnt[i]
    return m


def lone_event_ns(B, scn, seed: int, stream) -> float:
    """Per-event latency of a lone lineage (nh_measure_event_latency, 20,000 events): the median of
    three walks, which move by several per cent from one to the next."""
    return float(np.median([B.measure_event_latency(scn, seed, 20000, stream) for _ in range(3)]))


def latency_bound(B, scn, samples, out, ws, cfg, stream, run_ms: float) -> dict:
    """The serial bound of the seed-42 simulate: the events on its longest sample path, each waiting
    on the previous one, times the per-event latency of a lone lineage (measured with the round
    kernel's group step); frac = bound / the run's stream time."""
    jobs = [(scn, 42, samples, out, None)]
    run_rounds = B.batch_run(jobs, ws, cfg, stream)[0]["rounds"]
    res = B.event_stream(jobs, ws, stream=stream)[0]
    path = chain_events(res["events"], res["coalescences"])
    ev = res["events"]
    windows = window_maxima(ev, res["coalescences"], horizon_table(cfg, float(ev["t"].max()) if len(ev) else 0.0))
    ns = lone_event_ns(B, scn, 42, stream)
    bound_ms = path * ns * 1e-6
    sched_ms = sum(windows) * ns * 1e-6
    return {"path_events": path, "event_ns": ns, "bound_ms": bound_ms, "run_ms": run_ms, "frac": bound_ms / run_ms,
            "what": "longest sample path in events x lone-lineage per-event latency, vs the seed-42 run",
            # the horizon rounds' own bound: each round waits for the busiest lineage of its window
            "schedule": {"rounds": len(windows), "run_rounds": run_rounds, "events": sum(windows), "bound_ms": sched_ms,
                         "frac": sched_ms / run_ms, "per_round_events": windows},
            # each event of the run once (no copies of coalesced lineages): independent of the knobs
            "distinct_events": res["n_events"], "distinct_events_per_s": res["n_events"] / (run_ms * 1e-3)}


def host_cpu() -> dict:
    """The host's CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.lower().startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def _mix_worker(k):
    import oracle
    from paper_2108_05815_amd import workloads as W
    w = W.config4()[k]
    osc = oracle.Scenario(w.capacity, w.weights, w.nu, mode=w.mode)
    _, ev, _ = osc.simulate_culled(w.seeds[0], w.samples, 2.0)
    return k, len(w.samples), ev


def cpu_baseline_mix(budget_s: float) -> dict:
    """The culled oracle over the 256-scenario mix in one process per usable core (scenarios are
    independent), smallest scenarios first, for a bounded wall time: the scenarios finished within
    it give the rate."""
    import multiprocessing as mp
    from paper_2108_05815_amd import workloads as W
    wls = W.config4()
    order = sorted(range(len(wls)), key=lambda k: len(wls[k].samples))
    n = host_cpu()["nproc"] or 1
    done, lineages, events = 0, 0, 0
    t0 = time.perf_counter()
    el = 0.0
    # fresh interpreters (this process holds the GPU; the workers never touch it)
    with mp.get_context("spawn").Pool(processes=n) as pool:
        it = pool.imap_unordered(_mix_worker, order, chunksize=1)
        for _ in order:
            try:
                _, nl, ev = it.next(timeout=max(0.01, budget_s - (time.perf_counter() - t0)))
            except mp.TimeoutError:
                break
            el = time.perf_counter() - t0
            done, lineages, events = done + 1, lineages + nl, events + ev
            if el >= budget_s:
                break
        pool.terminate()
    return {"value": lineages / el if el > 0 else 0.0, "unit": "individuals/s", "cores": n, "kind": "oracle",
            "events_per_s": events / el if el > 0 else 0.0, "individuals_per_s": lineages / el if el > 0 else 0.0,
            **host_cpu(),
            "sample": f"{done} of the 256 scenarios of the mix (smallest first, {lineages} lineages), culled "
                      f"oracle (horizon step 2.0), one process per core on {n} cores, {el:.1f} s"}


def cpu_baseline(wl, budget_s: float) -> dict:
    """The oracle's culled form on whole seeds of the same workload until the budget is spent."""
    import oracle
    sc = oracle.Scenario(wl.capacity, wl.weights, wl.nu, mode=wl.mode)
    events = 0
    runs = 0
    t0 = time.perf_counter()
    while True:
        _, ev, _ = sc.simulate_culled(42 + runs, wl.samples, 1.0)
        events += ev
        runs += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return {"value": events / el, "unit": "lineage events/s", "cores": 1, "kind": "oracle",
            "individuals_per_s": runs * len(wl.samples) / el, **host_cpu(),
            "sample": f"{runs} whole seeds (42..{41 + runs}) of the same 65,536-lineage workload, "
                      f"single-threaded culled oracle (horizon step 1.0), {el:.1f} s"}


def profile_summary(db: str, kernel_re: str) -> dict:
    """Kernel-trace statistics (per kernel name: calls, average/total/min/max duration) and counter
    sums per dispatch (rocprofv3 reports counters per shader engine; they are added up) from a
    rocprofv3 SQLite results database."""
    import re
    import sqlite3
    con = sqlite3.connect(db)
    tables = {r[0] for r in con.execute("select name from sqlite_master where type in ('table', 'view')")}

    def short(name):
        n = re.sub(r"\(anonymous namespace\)::", "", name)
        if "rocprim" in n:
            return "rocprim sort/scan kernels (all)"
        return re.sub(r"\(.*$", "", n).replace("void ", "")

    out = {"database": os.path.basename(db)}
    if "kernels" in tables:
        agg = {}
        for name, dur in con.execute("select name, duration from kernels"):
            agg.setdefault(short(name), []).append(dur / 1e3)
        out["trace"] = [{"kernel": k, "calls": len(v), "avg_us": sum(v) / len(v), "total_ms": sum(v) / 1e3,
                         "min_us": min(v), "max_us": max(v)}
                        for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))]
    if "counters_collection" in tables:
        per = {}
        for d, kname, c, v in con.execute("select dispatch_id, kernel_name, counter_name, sum(value) from "
                                          "counters_collection group by dispatch_id, counter_name "
                                          "order by dispatch_id"):
            if re.search(kernel_re, kname):
                per.setdefault(int(d), {"kernel": short(kname)})[c] = float(v)
        out["counters"] = per
    return out


def main():
    args = parse()
    if args.profile_summary:
        print(json.dumps(profile_summary(args.profile_summary, args.profile_kernel)))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the method shards by samples with no "
              "communication, and this benchmark measures a single GPU.", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30, "copies": 3}))
        return
    from paper_2108_05815_amd import binding as B
    from paper_2108_05815_amd import roofline as RL
    from paper_2108_05815_amd import workloads as W
    if args.event_stream:
        print(json.dumps(stream_form(B, W, torch, torch.cuda.current_stream())), flush=True)
        return
    if args.batched_only:
        print(json.dumps(batched_form(args, B, W, torch, compare=False)), flush=True)
        return

    wl = W.config2()
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    scn = B.Scenario.from_workload(wl)
    create_ms = (time.perf_counter() - t0) * 1e3
    n = len(wl.samples)
    samples = torch.from_numpy(wl.samples.astype(np.int64)).to(dev)
    out = torch.empty(n, dtype=torch.int64, device=dev)
    rich = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(B.workspace_bytes(n, 1), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    tuned = None
    if args.knobs:
        from paper_2108_05815_amd import autotune as AT
        tuned = json.loads(args.knobs)
        cfg = AT.to_config(tuned, event_timing=1)
    elif not args.no_tune:
        from paper_2108_05815_amd import autotune as AT

        def one(cfg):
            st = B.batch_run([(scn, 7, samples, out, rich)], ws, cfg, stream)[0]
            return st["device_ms"] / 1e3

        note("autotuning the plain form")
        tuned, tuned_s, _ = AT.tune(one, reps=2)
        cfg = AT.to_config(tuned, event_timing=1)
    else:
        cfg = B.make_config(event_timing=1)

    note("plain form (256x256 torus): warm-up and timed steps")
    for k in range(args.warmup):
        B.batch_run([(scn, 1000 + k, samples, out, rich)], ws, cfg, stream)
    torch.cuda.synchronize()
    totals = dict(events=0, philox_calls=0, exp_draws=0, round_kernels=0, round_kernel_ms=0.0, richness=0)
    t0 = time.perf_counter()
    run_ms = []
    for k in range(args.steps):
        st = B.batch_run([(scn, 42 + k, samples, out, rich)], ws, cfg, stream)[0]
        run_ms.append(st["device_ms"])
        for key in totals:
            totals[key] += st[key]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    latency = latency_bound(B, scn, samples, out, ws, cfg, stream, run_ms[0])

    events_per_s = totals["events"] / elapsed
    ops = RL.algorithmic_ops(totals["philox_calls"], totals["exp_draws"], totals["events"])
    round_s = totals["round_kernel_ms"] / 1e3
    achieved = ops / round_s / 1e12 if round_s > 0 else 0.0
    peak = RL.PEAK_LANE_OPS / 1e12
    # the rate the chip sustains for the same Philox + log mix with every lane busy (in-repo microbenchmark)
    mix_peak = B.measure_mix_peak(stream) / 1e12
    traffic = traffic_from_profile(args.traffic)
    line = {
        "metric": METRIC,
        "value": events_per_s,
        "unit": "lineage events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "form": "plain (one scenario per run)", "lineages": n, "torus": "256x256",
                   "capacity": 1, "sigma": 2.0, "kernel": "21x21", "nu": wl.nu, "lambda": 1.0, "delta_t": 1.0,
                   "seeds": f"42..{41 + args.steps}", "tuned": tuned},
        "individuals_per_s": args.steps * n / elapsed,
        "events_per_step": totals["events"] / args.steps,
        "mean_richness": totals["richness"] / args.steps,
        "scenario_create_ms": create_ms,
        "roofline": {
            "bound": "alu",
            "kernel": ("k_run (one persistent launch: every horizon round of the run, each event sampling, "
                       "dispersal, cull and compaction, with a grid barrier between rounds)"
                       if cfg.launch == B.NH_LAUNCH_PERSISTENT else
                       "k_round (one horizon round: event sampling, dispersal, cull, compaction)"),
            "achieved": achieved,
            "peak": peak,
            "unit": "T lane-ops/s",
            "frac": achieved / peak,
            "traffic": traffic,
            "mix_peak": mix_peak,
            "frac_of_mix_peak": achieved / mix_peak,
            "avg_launch_us": totals["round_kernel_ms"] * 1e3 / max(1, totals["round_kernels"]),
            "launches": totals["round_kernels"],
            "ops_per_launch": ops / max(1, totals["round_kernels"]),
            "philox_per_event": totals["philox_calls"] / max(1, totals["events"]),
            "draws_per_event": totals["exp_draws"] / max(1, totals["events"]),
            "latency": latency,
        },
    }
    if not args.no_extras:
        # the host-buffer entry point (nh_simulate, library default knobs): the same workload with
        # samples uploaded and species downloaded over PCIe each time; context only, never the value
        t0 = time.perf_counter()
        host_ev = 0
        for k in range(5):
            _, _, st_h = B.simulate(scn, 42 + k, wl.samples)
            host_ev += st_h["events"]
        host_s = time.perf_counter() - t0
        line["host_buffers"] = {"entry": "nh_simulate", "runs": 5, "ms_per_run": host_s * 200.0,
                                "events_per_s": host_ev / host_s}
        note("Poisson-count sampler")
        line["poisson_sampler"] = sampler_form(B, W, torch, cfg, stream)
        note("event stream")
        line["event_stream"] = stream_form(B, W, torch, stream)
        note("batched form (256-scenario mix): tuning, warm-up, timed runs")
        line["batched"] = batched_form(args, B, W, torch)
        line["serve"] = served_form(args, W, torch)
    if not args.no_c3:
        note("heterogeneous habitat (1024x1024)")
        line["c3"] = habitat_form(B, W, torch)
    if not args.no_cpu:
        note("CPU oracle, one thread")
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
        if not args.no_extras:
            note("CPU oracle, one process per core, on the mix")
            line["cpu_baseline_c4"] = cpu_baseline_mix(args.cpu_c4_seconds)
            b = line["batched"]
            line["cpu_baseline_c4"]["gpu_batched_individuals_per_s"] = b["individuals_per_s"]
            line["cpu_baseline_c4"]["gpu_over_cpu_individuals"] = (b["individuals_per_s"]
                                                                   / line["cpu_baseline_c4"]["individuals_per_s"])
    print(json.dumps(line), flush=True)


def sampler_form(B, W, torch, cfg, stream, steps: int = 10) -> dict:
    """The same torus with the Poisson-count event-time sampler (other bits, same law), timed like
    the headline runs: the comparison the paper makes between its two samplers."""
    import copy
    dev = torch.device("cuda:0")
    wl = copy.copy(W.config2())
    wl.sampler = 1
    scn = B.Scenario.from_workload(wl)
    n = len(wl.samples)
    samples = torch.from_numpy(wl.samples.astype(np.int64)).to(dev)
    out = torch.empty(n, dtype=torch.int64, device=dev)
    ws = torch.empty(B.workspace_bytes(n, 1), dtype=torch.uint8, device=dev)
    for k in range(2):
        B.batch_run([(scn, 1000 + k, samples, out, None)], ws, cfg, stream)
    torch.cuda.synchronize()
    ev = 0
    t0 = time.perf_counter()
    for k in range(steps):
        ev += B.batch_run([(scn, 42 + k, samples, out, None)], ws, cfg, stream)[0]["events"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"workload": wl.name + ", Poisson-count sampler", "steps": steps, "ms_per_step": el * 1e3 / steps,
            "events_per_s": ev / el, "individuals_per_s": steps * n / el}


def stream_form(B, W, torch, stream, reps: int = 5) -> dict:
    """The event stream of one run of the same torus (nh_event_stream into resident device buffers):
    the replay of every committed event, the radix sorts and the reduction, timed per call.  The run
    uses the library's default knobs, which commit fewer redundant events than the throughput-tuned
    ones (the replay re-derives every committed event)."""
    cfg = B.make_config()
    dev = torch.device("cuda:0")
    wl = W.config2()
    scn = B.Scenario.from_workload(wl)
    n = len(wl.samples)
    samples = torch.from_numpy(wl.samples.astype(np.int64)).to(dev)
    out = torch.empty(n, dtype=torch.int64, device=dev)
    ws = torch.empty(B.workspace_bytes(n, 1), dtype=torch.uint8, device=dev)
    jobs = [(scn, 42, samples, out, None)]
    st = B.batch_run(jobs, ws, cfg, stream)[0]
    co = [torch.empty(n * B.COALESCENCE_DTYPE.itemsize, dtype=torch.uint8, device=dev)]
    n_ev, n_co = B.event_stream_device(jobs, ws, [None], co, stream)[0]
    ev = [torch.empty(n_ev * B.EVENT_DTYPE.itemsize, dtype=torch.uint8, device=dev)]
    B.event_stream_device(jobs, ws, ev, co, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        B.event_stream_device(jobs, ws, ev, co, stream)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    return {"workload": wl.name + ", seed 42", "entry": "nh_event_stream", "reps": reps, "ms_per_stream": el * 1e3,
            "committed_events_replayed": st["events"], "distinct_events": n_ev, "coalescences": n_co,
            "distinct_events_per_s": n_ev / el, "records_per_s": (st["events"] + st["merged"]) / el,
            "simulate_ms": st["device_ms"]}


def habitat_form(B, W, torch) -> dict:
    """The heterogeneous-habitat workload: per-deme alias tables (about 10 GiB) gathered from HBM."""
    from paper_2108_05815_amd import roofline as RL
    dev = torch.device("cuda:0")
    wl = W.config3()
    t0 = time.perf_counter()
    scn = B.Scenario.from_workload(wl)
    create_s = time.perf_counter() - t0
    n = len(wl.samples)
    s = torch.from_numpy(wl.samples.astype(np.int64)).to(dev)
    out = torch.empty(n, dtype=torch.int64, device=dev)
    ws = torch.empty(B.workspace_bytes(n, 1), dtype=torch.uint8, device=dev)
    cfg = B.make_config(event_timing=1)
    B.batch_run([(scn, 41, s, out, None)], ws, cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = B.batch_run([(scn, wl.seeds[0], s, out, None)], ws, cfg)[0]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # each dispersal gathers a 16-byte alias entry (with the targets' capacities) and a row pointer pair (8 B)
    disp = st["events"] - st["speciated"]
    gather_bytes = disp * RL.BYTES_PER_DISPERSAL_PER_DEME
    rs = st["round_kernel_ms"] / 1e3
    # random 16-byte gathers from a table as large as the habitat's: the ceiling those gathers could reach
    ceiling = B.measure_gather(scn_table_sized(torch, dev, scn.table_bytes))
    return {"workload": wl.name, "lineages": n, "table_gib": scn.table_bytes / 2**30, "create_s": create_s,
            "seconds": el, "events": st["events"], "events_per_s": st["events"] / el, "individuals_per_s": n / el,
            "richness": st["richness"], "rounds": st["rounds"],
            "gather_gb_per_s": gather_bytes / rs / 1e9 if rs > 0 else None,
            "gather_frac_of_8tbs": gather_bytes / rs / 8e12 if rs > 0 else None,
            "gather_ceiling_gb_per_s": ceiling / 1e9,
            "gather_frac_of_ceiling": gather_bytes / rs / ceiling if rs > 0 else None}


def scn_table_sized(torch, dev, nbytes):
    return torch.empty(max(int(nbytes), 1 << 20), dtype=torch.uint8, device=dev)


# the batched form stays one persistent launch per run; these are its tuned knobs
BATCH_KNOBS = {"solo_max": [0, 64, 256], "horizon_step_max": [64.0, 256.0, 4096.0],
               "horizon_growth": [1.25, 1.5, 2.0], "horizon0": [0.5, 2.0], "blocks_per_cu": [2, 4]}


def batched_form(args, B, W, torch, compare: bool = True) -> dict:
    """The 256-scenario mix in one batched run: knobs tuned on the mix itself (one run per
    candidate), one warm-up run, then the median of args.batch_runs timed runs; the ALU roofline
    of its round kernel and the serial bound of its slowest scenario; and the mix against one
    scenario per run on a subset, compared in individuals/s (which no knob changes)."""
    from paper_2108_05815_amd import autotune as AT
    from paper_2108_05815_amd import roofline as RL
    import statistics
    dev = torch.device("cuda:0")
    wls = W.config4()
    scns = [B.Scenario.from_workload(w) for w in wls]
    samples = [torch.from_numpy(w.samples.astype(np.int64)).to(dev) for w in wls]
    outs = [torch.empty(len(w.samples), dtype=torch.int64, device=dev) for w in wls]
    n_total = sum(len(w.samples) for w in wls)
    ws = torch.empty(B.workspace_bytes(n_total, len(wls)), dtype=torch.uint8, device=dev)
    jobs = [(scns[k], wls[k].seeds[0], samples[k], outs[k], None) for k in range(len(wls))]

    def timed(cfg):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = B.batch_run(jobs, ws, cfg)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, st

    tuned = None
    start = dict(AT.DEFAULT, launch=0, solo_max=0)
    if args.batch_knobs:
        tuned = dict(start, **json.loads(args.batch_knobs))
    elif not args.no_batch_tune:
        tuned, _, _ = AT.tune(lambda cfg: timed(cfg)[0], knobs=BATCH_KNOBS, start=start, reps=1)
    knobs = tuned or start
    cfg = AT.to_config(knobs, event_timing=1)
    if compare:
        timed(cfg)  # warm-up
    runs = [timed(cfg) for _ in range(max(1, args.batch_runs))]
    secs = [r[0] for r in runs]
    el = statistics.median(secs)
    st = runs[secs.index(el)][1] if el in secs else runs[0][1]
    ev = sum(x["events"] for x in st)
    tot = st[0]
    ops = RL.algorithmic_ops(tot["philox_calls"], tot["exp_draws"], ev)
    round_s = tot["round_kernel_ms"] / 1e3
    achieved = ops / round_s if round_s > 0 else 0.0
    slow = max(range(len(wls)), key=lambda k: st[k]["rounds"])
    roof = {"bound": "alu", "kernel": "k_run" if knobs.get("launch", 0) == 0 else "k_round",
            "achieved": achieved / 1e12, "peak": RL.PEAK_LANE_OPS / 1e12, "unit": "T lane-ops/s",
            "frac": achieved / RL.PEAK_LANE_OPS, "round_kernel_s": round_s, "launches": tot["round_kernels"],
            "avg_launch_us": tot["round_kernel_ms"] * 1e3 / max(1, tot["round_kernels"]),
            "ops_per_launch": ops / max(1, tot["round_kernels"])}
    res = {"workload": "C4 mix: 256 scenarios, sides 64-512, capacity 1-4, sigma 1-6, nu 1e-6..1e-2",
           "lineages": n_total, "tuned": knobs, "runs": len(secs), "seconds": el, "seconds_all": secs,
           "events_per_s": ev / el, "individuals_per_s": n_total / el, "rounds": max(x["rounds"] for x in st),
           "slowest_scenario": wls[slow].name, "roofline": roof}
    if not compare:
        return res
    roof["latency"] = slowest_job_bound(B, torch, wls[slow], scns[slow], samples[slow], knobs)
    m = min(args.batch_plain_subset, len(wls))
    sub = jobs[:m]
    n_sub = sum(len(w.samples) for w in wls[:m])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.batch_run(sub, ws, cfg)
    torch.cuda.synchronize()
    el_b = time.perf_counter() - t0
    t0 = time.perf_counter()
    for j in sub:
        B.batch_run([j], ws, cfg)
    torch.cuda.synchronize()
    el_p = time.perf_counter() - t0
    res["subset"] = {"scenarios": m, "lineages": n_sub, "batched_s": el_b, "plain_s": el_p,
                     "batched_individuals_per_s": n_sub / el_b, "plain_individuals_per_s": n_sub / el_p,
                     "speedup": el_p / el_b}
    return res


def slowest_job_bound(B, torch, wl, scn, samples, knobs) -> dict:
    """Serial bound of the batch's slowest scenario (the job that finished last): its latest
    speciation time t_max, from the speciation-event reporter of a run of that scenario alone,
    times lambda is the expected number of events on the path that ends there (events come at
    rate lambda); times the lone-lineage latency per event it is the time no schedule can beat."""
    from paper_2108_05815_amd import autotune as AT
    dev = torch.device("cuda:0")
    n = len(wl.samples)
    out = torch.empty(n, dtype=torch.int64, device=dev)
    rep = {"spec_loc": torch.empty(n, dtype=torch.int32, device=dev),
           "spec_time": torch.empty(n, dtype=torch.float64, device=dev)}
    ws = torch.empty(B.workspace_bytes(n, 1), dtype=torch.uint8, device=dev)
    cfg = AT.to_config(knobs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.batch_run([(scn, wl.seeds[0], samples, out, None, rep)], ws, cfg)
    torch.cuda.synchronize()
    alone_s = time.perf_counter() - t0
    t_max = float(rep["spec_time"].max().item())
    ns = lone_event_ns(B, scn, wl.seeds[0], None)
    path = t_max * wl.lam
    return {"scenario": wl.name, "lineages": n, "t_max": t_max, "path_events_estimate": path, "event_ns": ns,
            "bound_s": path * ns * 1e-9, "alone_s": alone_s,
            "what": "latest speciation time x lambda (expected events on that path) x lone-lineage latency"}


def served_form(args, W, torch) -> dict:
    """Poisson request stream (200 req/s) through the continuous-batching server: args.serve_warmup
    seconds of warm-up requests, then args.serve_seconds measured, all on one server whose budget
    (lineage pool plus every live request's tables) is args.serve_hbm_frac of the free HBM; the
    slowest measured request again alone on the idle device; and the first measured requests one
    per run for comparison (individuals/s: no knob changes it)."""
    from paper_2108_05815_amd import binding as B
    from paper_2108_05815_amd import serve as S
    total = args.serve_warmup + args.serve_seconds
    arrivals, specs = W.config5_requests(duration=total)
    free, _ = torch.cuda.mem_get_info()
    budget = int(args.serve_hbm_frac * free)
    note(f"served form: {len(specs)} requests over {total:g} s")
    served = S.run_served(arrivals, specs, hbm_budget_bytes=budget, measure_from=args.serve_warmup, progress_s=10.0)
    note("served form: the first measured requests one per run")
    meas = served["measured"]
    m = min(args.serve_plain, len(meas))
    first = meas[:m]
    plain = S.run_plain(arrivals[first], [specs[k] for k in first])
    prefix = served["latencies_s"][first]
    # the slowest measured request again, alone on the idle device: the floor its serial tail sets
    # (the median of three runs: a lone lineage's per-event time moves by several per cent between runs)
    slow = max(meas, key=lambda k: served["latencies_s"][k])
    note("served form: the slowest request alone, three times")
    wl, scn = S._build(specs[slow])
    n = scn.individuals
    dev = torch.device("cuda:0")
    s_ids = torch.arange(n, dtype=torch.int64, device=dev)
    out_ids = torch.empty(n, dtype=torch.int64, device=dev)
    ws = torch.empty(B.workspace_bytes(n, 1), dtype=torch.uint8, device=dev)
    alone_runs = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = B.batch_run([(scn, wl.seeds[0], s_ids, out_ids, None)], ws)[0]
        torch.cuda.synchronize()
        alone_runs.append(time.perf_counter() - t0)
    alone_s = float(np.median(alone_runs))
    rounds, events, _, _ = served["per_request"][slow]
    served_ms = float(served["latencies_s"][slow] * 1e3)
    return {"workload": f"C5: Poisson 200 req/s, {args.serve_warmup:g} s warm-up then {args.serve_seconds:g} s "
                        "measured, half spatial (C4-like), half non-spatial J 1e3..1e6, all individuals sampled",
            "requests": served["requests"], "warmup_requests": served["warmup_requests"],
            "p50_ms": served["latency"]["p50_ms"], "p99_ms": served["latency"]["p99_ms"],
            "max_ms": served["latency"]["max_ms"], "mean_ms": served["latency"]["mean_ms"],
            "events_per_s": served["events_per_s"], "individuals_per_s": served["individuals_per_s"],
            "offered_requests_per_s": served["offered_requests_per_s"], "sustained": served["sustained"],
            "median_latency_first_third_ms": served["median_latency_first_third_ms"],
            "median_latency_last_third_ms": served["median_latency_last_third_ms"],
            "peak_pending": served["peak_pending"], "peak_active": served["peak_active"],
            "hbm": {"free_bytes": int(free), "budget_frac": args.serve_hbm_frac, "budget_bytes": budget,
                    "lineage_pool_bytes": served["lineage_pool_bytes"], "lineage_capacity": served["lineage_capacity"],
                    "table_budget_bytes": served["table_budget_bytes"],
                    "table_peak_bytes": served["table_peak_bytes"]},
            "plain_prefix": {"requests": m, "plain_p50_ms": plain["latency"]["p50_ms"],
                             "plain_p99_ms": plain["latency"]["p99_ms"],
                             "plain_individuals_per_s": plain["individuals_per_s"],
                             "served_p50_ms": float(np.percentile(prefix, 50) * 1e3),
                             "served_p99_ms": float(np.percentile(prefix, 99) * 1e3)},
            "slowest_request": {"spec": {k: v for k, v in specs[slow].items() if k != "name"},
                                "served_ms": served_ms, "events": events, "alone_ms": alone_s * 1e3,
                                "alone_ms_runs": [x * 1e3 for x in alone_runs],
                                "alone_events": st["events"], "served_over_alone": served_ms / (alone_s * 1e3)}}


if __name__ == "__main__":
    main()
