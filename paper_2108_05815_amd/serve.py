"""Served form of the Independent algorithm: a request stream through the
continuous-batching engine (nh_server_* in libnecsim_hip).

Each request is a scenario (landscape, dispersal kernel, nu) and a seed, with
every individual sampled.  Requests arrive on a Poisson clock; on arrival a
worker thread builds the scenario's tables (nh_scenario_create), the request is
submitted to the server, which admits it into the running device batch as soon
as a contiguous range of resident lineage slots (its HBM footprint) and a job
slot are free, and the request completes when its last lineage retires.
Latency = completion (richness on the host) minus arrival.

The plain comparison runs the same requests one at a time, each in its own
device run (nh_batch_run with one job), in arrival order: a request starts
when it has arrived and the previous one has finished.
"""
from __future__ import annotations

import concurrent.futures as cf
import sys
import time

import numpy as np

from . import binding as B
from . import workloads as W


def _build(spec_or_workload):
    wl = W.materialize(spec_or_workload) if isinstance(spec_or_workload, dict) else spec_or_workload
    return wl, B.Scenario.from_workload(wl)


def _percentiles(lat):
    a = np.asarray(lat, dtype=np.float64)
    if len(a) == 0:
        return {"p50_ms": None, "p99_ms": None, "mean_ms": None, "max_ms": None}
    return {"p50_ms": float(np.percentile(a, 50) * 1e3), "p99_ms": float(np.percentile(a, 99) * 1e3),
            "mean_ms": float(a.mean() * 1e3), "max_ms": float(a.max() * 1e3)}


def lineage_capacity_for_budget(budget_bytes: int, max_jobs: int) -> int:
    """Largest resident pool whose device footprint fits the byte budget."""
    lo, hi = 1, 1 << 30
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if B.server_bytes(mid, max_jobs) <= budget_bytes:
            lo = mid
        else:
            hi = mid
    return lo


# Served jobs share round boundaries, so one round lasts as long as the slowest
# lineage's events in it; a small cap on each round's horizon advance keeps
# rounds short for the jobs that just arrived (a long-lived job then takes more,
# cheap rounds).  A job down to its last few lineages (solo_max) leaves that
# schedule: its lineages run 8 lanes each at raised wave priority and advance
# solo_step per round (a short step keeps the rounds short too), and its last
# lineage leaves for the tail lane, so its serial tail is not paced by young
# jobs' rounds.  The batched form, which only cares about the total, prefers a
# large cap; the autotuner chooses per workload.
SERVE_DEFAULTS = {"horizon_step_max": 64.0, "solo_max": 256, "solo_step": 256.0}


def table_bytes_estimate(spec: dict) -> int:
    """Device bytes of a request's scenario tables before they are built: capacity (u32) and its
    prefix (u64) per cell, and one 16-byte alias entry per kernel cell (shared table)."""
    if spec["kind"] == "spatial":
        cells = spec["L"] * spec["L"]
        return 12 * cells + 8 + 16 * (2 * spec["R"] + 1) ** 2 + 4096
    return 4096


def run_served(arrivals, requests, *, hbm_budget_bytes: int | None = None, lineage_capacity: int | None = None,
               max_jobs: int = 2048, lookahead: int = 64, config=None, workers: int = 4, timeout_s: float = 900.0,
               collect: bool = False, measure_from: float = 0.0, table_frac: float = 0.02,
               progress_s: float = 0.0, tail_blocks: int = 32):
    """Serve the stream; returns latency percentiles, throughput and admission statistics.

    HBM admission: the budget (default half of the free HBM) holds the resident lineage pool (the
    server's workspace) and every live request's scenario tables.  table_frac of it is set aside for
    tables; a request whose tables would not fit waits, unbuilt, until completed requests release
    theirs, and a request is admitted into the running batch once its lineage slots are free.
    progress_s > 0: a line on stderr that often (requests done, active, waiting).
    tail_blocks: compute units of the server's tail lane (a job's last lineage walks there outside
    the rounds; 0 = none).
    measure_from: requests arriving before this time (s) warm the server up and are left out of
    the latency and throughput figures.  collect: also return each request's result as (richness,
    SHA-256 of its species array in sample order), read back on completion (for parity checks; it
    adds a device-to-host copy per request)."""
    import torch

    if config is None:
        config = B.make_config(**SERVE_DEFAULTS)
    dev = torch.device("cuda:0")
    if hbm_budget_bytes is None:
        free, _ = torch.cuda.mem_get_info()
        hbm_budget_bytes = int(0.5 * free)
    table_budget = int(table_frac * hbm_budget_bytes)
    if lineage_capacity is None:
        lineage_capacity = lineage_capacity_for_budget(hbm_budget_bytes - table_budget, max_jobs)
    pool_bytes = B.server_bytes(lineage_capacity, max_jobs)
    stream = torch.cuda.Stream()
    srv = B.Server(lineage_capacity, max_jobs=max_jobs, lookahead=lookahead, config=config, stream=stream,
                   tail_blocks=tail_blocks)
    pool = cf.ThreadPoolExecutor(max_workers=workers)
    n = len(requests)
    lat = np.full(n, np.nan)
    per_request = {}  # request index -> (rounds, events, lineages) from its completion
    results = {}      # request index -> (richness, species digest) when collecting
    tables = {}       # request index -> device bytes of its tables (reserved estimate, then actual)
    table_live = table_peak = 0
    building = {}
    waiting = []      # arrived requests whose tables do not fit yet, in arrival order
    nxt = done = 0
    peak_pending = peak_active = 0
    t0 = time.perf_counter()
    next_note = progress_s
    try:
        while done < n:
            now = time.perf_counter() - t0
            if progress_s > 0 and now >= next_note:
                print(f"[serve] {now:.0f} s: {done}/{n} done, {nxt} arrived, {len(waiting) + len(building)} waiting",
                      file=sys.stderr, flush=True)
                next_note += progress_s
            if now > timeout_s:
                raise TimeoutError(f"serving stream did not finish in {timeout_s} s ({done}/{n} done)")
            while nxt < n and arrivals[nxt] <= now:
                waiting.append(nxt)
                nxt += 1
            while waiting:
                idx = waiting[0]
                need = table_bytes_estimate(requests[idx])
                if table_live + need > table_budget and table_live > 0:
                    break
                waiting.pop(0)
                tables[idx] = need
                table_live += need
                building[idx] = pool.submit(_build, requests[idx])
            for idx in [k for k, f in building.items() if f.done()]:
                wl, scn = building.pop(idx).result()
                table_live += scn.table_bytes - tables[idx]
                tables[idx] = scn.table_bytes
                table_peak = max(table_peak, table_live)
                with torch.cuda.stream(stream):
                    N = scn.individuals
                    samples = torch.arange(N, dtype=torch.int64, device=dev)
                    out = torch.empty(N, dtype=torch.int64, device=dev)
                    rich = torch.empty(1, dtype=torch.int64, device=dev)
                srv.submit(idx, scn, wl.seeds[0], samples, out, rich)
            active, pending = srv.progress()
            peak_pending = max(peak_pending, pending + len(building) + len(waiting))
            peak_active = max(peak_active, active)
            for c in srv.poll():
                t_done = time.perf_counter() - t0
                idx = c["tag"]
                if c["status"] != 0:
                    raise RuntimeError(f"request {idx} failed with status {c['status']}")
                lat[idx] = t_done - arrivals[idx]
                per_request[idx] = (int(c["rounds"]), int(c["events"]), int(c["lineages"]), float(t_done))
                if collect:
                    import hashlib
                    species = c["held"][2].cpu().numpy().view(np.uint64)
                    results[idx] = (int(c["richness"]), hashlib.sha256(species.astype("<u8").tobytes()).hexdigest())
                c["held"][0].close()  # the request's tables go back to the budget
                table_live -= tables.pop(idx)
                done += 1
            if not building and not waiting and nxt < n and srv.progress()[0] == 0:
                time.sleep(min(0.0005, max(0.0, arrivals[nxt] - (time.perf_counter() - t0))))
        wall = time.perf_counter() - t0
    finally:
        pool.shutdown(wait=True)
        srv.close()
    meas = [k for k in range(n) if arrivals[k] >= measure_from]
    m_lat = lat[meas]
    events = sum(per_request[k][1] for k in meas)
    individuals = sum(per_request[k][2] for k in meas)
    # throughput of the measured requests: from the first measured arrival to the last measured completion
    span = (max(per_request[k][3] for k in meas) - float(arrivals[meas[0]])) if meas else wall
    third = max(1, len(meas) // 3)
    first, last = (np.median(m_lat[:third]), np.median(m_lat[-third:])) if meas else (np.nan, np.nan)
    return {"requests": len(meas), "warmup_requests": n - len(meas), "wall_s": wall, "events": int(events),
            "individuals": int(individuals), "events_per_s": events / span, "individuals_per_s": individuals / span,
            "offered_requests_per_s": (len(meas) / float(arrivals[meas[-1]] - arrivals[meas[0]])
                                       if len(meas) > 1 else None),
            "hbm_budget_bytes": int(hbm_budget_bytes), "lineage_pool_bytes": int(pool_bytes),
            "table_budget_bytes": table_budget, "table_peak_bytes": int(table_peak),
            "lineage_capacity": int(lineage_capacity), "max_jobs": max_jobs,
            "peak_pending": int(peak_pending), "peak_active": int(peak_active),
            "latency": _percentiles(m_lat), "latencies_s": lat, "measured": meas, "per_request": per_request,
            "results": results,
            # the stream is sustained if requests arriving late wait no longer than early ones
            "median_latency_first_third_ms": float(first * 1e3), "median_latency_last_third_ms": float(last * 1e3),
            "sustained": bool(last <= 2.0 * first + 0.05)}


def run_plain(arrivals, requests, *, config=None):
    """The same requests one per device run, in arrival order (each waits for the previous)."""
    import torch

    dev = torch.device("cuda:0")
    n = len(requests)
    lat = np.zeros(n)
    busy_until = 0.0
    events = individuals = 0
    service = 0.0
    for k, req in enumerate(requests):
        t_start = time.perf_counter()
        wl, scn = _build(req)
        N = scn.individuals
        samples = torch.arange(N, dtype=torch.int64, device=dev)
        out = torch.empty(N, dtype=torch.int64, device=dev)
        rich = torch.empty(1, dtype=torch.int64, device=dev)
        ws = torch.empty(B.workspace_bytes(N, 1), dtype=torch.uint8, device=dev)
        st = B.batch_run([(scn, wl.seeds[0], samples, out, rich)], ws, config)[0]
        torch.cuda.synchronize()
        dur = time.perf_counter() - t_start
        scn.close()
        start = max(float(arrivals[k]), busy_until)
        busy_until = start + dur
        lat[k] = busy_until - float(arrivals[k])
        events += st["events"]
        individuals += N
        service += dur
    span = busy_until - float(arrivals[0])
    return {"requests": n, "service_s": service, "events": int(events), "individuals": int(individuals),
            "events_per_s": events / span, "individuals_per_s": individuals / span, "requests_per_s": n / span,
            "latency": _percentiles(lat), "latencies_s": lat}
