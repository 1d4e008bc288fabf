"""Autotuner for the round kernels' performance knobs.

None of the knobs changes a result (the GPU tests check that species ids are
identical under every setting), so the tuner is free to pick whatever runs
fastest on the workload at hand:

* cull period: the horizon schedule (first horizon, growth per round) --
  short rounds merge coalesced lineages sooner, long rounds pay fewer
  round boundaries;
* lanes per lineage: the queue length below which a lineage gets a group of
  8 lanes (its independent Philox blocks side by side) instead of one lane;
* launch form: one persistent launch for the whole run (grid barrier between
  rounds) or one launch per round replayed from captured graphs;
* occupancy and launch shape: workgroups per CU, workgroup size, round kernels
  per captured graph;
* solo tails (runs of several jobs): the live-lineage count below which a job
  runs its lineages 8 lanes each on blocks of their own;
* table placement: a shared dispersal table staged in LDS or read from global
  memory (L1/L2).

Search: coordinate descent from the library defaults, each candidate timed as
the median device time of `reps` runs.
"""
from __future__ import annotations

import statistics

from . import binding as B

# The launch form is a knob too ("launch": [0, 1], with "rounds_per_graph": [4, 8, 16] for the graph
# form), searched only when asked for: the default search keeps one persistent launch per run.
KNOBS = {
    "horizon0": [0.25, 0.5, 1.0, 2.0],
    "horizon_growth": [1.15, 1.25, 1.5, 2.0],
    "horizon_step_max": [64.0, 256.0, 4096.0],
    "coop_divisor": [0, 32, 16, 8],   # coop_max = launch lanes / divisor + 1; 0 keeps one lane per lineage
    "blocks_per_cu": [2, 4, 8],
    "block_size": [128, 256],
    "table_placement": [0, 1],
}

DEFAULT = {"launch": 0, "horizon0": 0.5, "horizon_growth": 1.25, "horizon_step_max": 4096.0, "coop_divisor": 16,
           "blocks_per_cu": 4, "block_size": 256, "rounds_per_graph": 8, "table_placement": 0}


def n_compute_units() -> int:
    import torch
    return torch.cuda.get_device_properties(0).multi_processor_count


def to_config(knobs: dict, n_cu: int | None = None, **extra) -> B.nh_config:
    n_cu = n_cu or n_compute_units()
    lanes = n_cu * knobs["blocks_per_cu"] * knobs["block_size"]
    div = knobs["coop_divisor"]
    return B.make_config(horizon0=knobs["horizon0"], horizon_growth=knobs["horizon_growth"],
                         horizon_step_max=knobs.get("horizon_step_max", 4096.0),
                         blocks_per_cu=knobs["blocks_per_cu"], block_size=knobs["block_size"],
                         rounds_per_graph=knobs["rounds_per_graph"], table_placement=knobs["table_placement"],
                         coop_max=(lanes // div + 1) if div else 1, launch=knobs.get("launch", 0),
                         solo_max=knobs.get("solo_max", 0), solo_step=knobs.get("solo_step", 0.0),
                         endgame=knobs.get("endgame", 0), **extra)


def tune(run, knobs=None, start=None, reps: int = 3, passes: int = 1, log=None):
    """Coordinate descent.  run(config) -> seconds for one run of the workload being tuned.
    Returns (best knob dict, best seconds, trial log)."""
    knobs = knobs or KNOBS
    best = dict(start or DEFAULT)
    n_cu = n_compute_units()
    trials = []

    def measure(k):
        cfg = to_config(k, n_cu)
        times = [run(cfg) for _ in range(reps)]
        t = statistics.median(times)
        trials.append((dict(k), t))
        if log:
            log(f"autotune {k} -> {t * 1e3:.3f} ms")
        return t

    best_t = measure(best)
    for _ in range(passes):
        for name, values in knobs.items():
            measured = best[name]  # the current setting was just measured
            for val in values:
                if val == measured:
                    continue
                cand = dict(best)
                cand[name] = val
                t = measure(cand)
                if t < best_t:
                    best, best_t = cand, t
    return best, best_t, trials
