"""Oracle species of a whole configuration, computed by the culled oracle in a
pool of worker processes; prints one JSON line per task with its richness and
the SHA-256 of its species array (u64, sample order).  Test infrastructure only:
a GPU test runs it as a separate process (which never touches the GPU, so its
workers may fork) and compares the digests with the library's output.

  --config 4   the 256-scenario mix: one task per scenario (key k = scenario index)
  --config 3   the 1024 x 1024 habitat: its samples split into --split contiguous
               parts, one task each (key k = part); a run's species do not depend on
               how the samples are partitioned (the Independent algorithm's
               partition independence), so the parts' arrays concatenated are the
               whole run's, and richness is computed over the concatenation
  --config 5   the served request stream of --serve-seconds: one task per request
               (key k = request index), every individual of the request sampled

    python tests/oracle_pool.py --config 4 [--dw 2.0] [--workers 16]
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import resource
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)

_TASKS = None  # list of (workload, samples or None for all individuals)


def _digest(species):
    return hashlib.sha256(species.astype("<u8").tobytes()).hexdigest()


def _culled(k_dw_whole):
    """One task: the species array itself (whole=True) or its richness and digest."""
    import numpy as np
    import oracle
    k, dw, whole = k_dw_whole
    w, samples = _TASKS[k]
    osc = oracle.Scenario(w.capacity, w.weights, w.nu, mode=w.mode)
    if samples is None:
        samples = np.arange(osc.individuals, dtype=np.uint64)
    species, events, _ = osc.simulate_culled(w.seeds[0], samples, dw)
    rss_gib = resource.getrusage(resource.RUSAGE_SELF).ru_maxrss / 2**20
    res = species if whole else (oracle.richness(species), _digest(species))
    return k, res, events, rss_gib


def _size(task):
    w, samples = task
    return len(samples) if samples is not None else int(w.capacity.astype(np.uint64).sum())


def main():
    global _TASKS
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=4, choices=(3, 4, 5))
    ap.add_argument("--dw", type=float, default=2.0, help="horizon step of the culled oracle")
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--split", type=int, default=4, help="config 3: parts of the sample set")
    ap.add_argument("--serve-seconds", type=float, default=5.0, help="config 5: length of the request stream")
    args = ap.parse_args()
    from paper_2108_05815_amd import workloads as W
    if args.config == 4:
        _TASKS = [(w, w.samples) for w in W.config4()]
    elif args.config == 3:
        wl = W.config3()
        _TASKS = [(wl, part) for part in np.array_split(wl.samples, args.split)]
    else:
        _, specs = W.config5_requests(duration=args.serve_seconds)
        _TASKS = [(W.materialize(s), None) for s in specs]
    whole = args.config == 3
    order = sorted(range(len(_TASKS)), key=lambda k: -_size(_TASKS[k]))  # largest first
    n = max(1, min(args.workers, os.cpu_count() or 1, len(_TASKS)))
    parts = {}
    with mp.get_context("fork").Pool(processes=n) as pool:
        for k, res, events, rss_gib in pool.imap_unordered(_culled, [(k, args.dw, whole) for k in order],
                                                           chunksize=1):
            line = {"k": k, "events": int(events), "worker_max_rss_gib": round(rss_gib, 2)}
            if whole:
                parts[k] = res
                line = {"part": k, **{x: line[x] for x in ("events", "worker_max_rss_gib")}}
            else:
                line.update(richness=res[0], sha256=res[1])
            print(json.dumps(line), flush=True)
    if whole:
        import oracle
        species = np.concatenate([parts[k] for k in range(len(_TASKS))])
        print(json.dumps({"k": 0, "richness": oracle.richness(species), "sha256": _digest(species)}), flush=True)


if __name__ == "__main__":
    main()
