"""Host-only logic around the GPU path: autotuner search, pool sizing for an HBM budget,
the request stream, and the traffic record's staleness check."""
import hashlib
import importlib.util
import os

import numpy as np
import pytest

from paper_2108_05815_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_autotune_coordinate_descent_finds_separable_minimum(monkeypatch):
    from paper_2108_05815_amd import autotune as AT
    monkeypatch.setattr(AT, "n_compute_units", lambda: 256)
    target = {"horizon0": 1.0, "horizon_growth": 1.5, "horizon_step_max": 256.0, "coop_divisor": 8,
              "blocks_per_cu": 2, "block_size": 128, "rounds_per_graph": 8, "table_placement": 1}
    seen = []

    def run(cfg):
        seen.append(cfg)
        # cost = number of knobs away from the target, read back from the config the tuner built
        knobs = {"horizon0": cfg.horizon0, "horizon_growth": cfg.horizon_growth,
                 "horizon_step_max": cfg.horizon_step_max, "blocks_per_cu": cfg.blocks_per_cu,
                 "block_size": cfg.block_size, "rounds_per_graph": cfg.rounds_per_graph,
                 "table_placement": cfg.table_placement}
        cost = sum(knobs[k] != target[k] for k in knobs)
        lanes = 256 * cfg.blocks_per_cu * cfg.block_size
        cost += cfg.coop_max != lanes // 8 + 1
        return float(cost)

    best, t, trials = AT.tune(run, reps=1)
    assert t == 0.0
    for k in target:
        assert best[k] == target[k], k
    assert len(trials) == 1 + sum(len(v) - 1 for v in AT.KNOBS.values())
    # the launch form is searched when asked for
    knobs = dict(AT.KNOBS, launch=[0, 1])
    best, t, _ = AT.tune(lambda cfg: float(cfg.launch != 1), knobs=knobs, reps=1)
    assert best["launch"] == 1 and t == 0.0


def test_autotune_config_mapping(monkeypatch):
    from paper_2108_05815_amd import autotune as AT
    cfg = AT.to_config(dict(AT.DEFAULT, coop_divisor=0), n_cu=256)
    assert cfg.coop_max == 1  # one lane per lineage always
    cfg = AT.to_config(dict(AT.DEFAULT), n_cu=256, event_timing=1)
    assert cfg.coop_max == 256 * 4 * 256 // 16 + 1 and cfg.event_timing == 1


def test_pool_sizing_respects_budget():
    from paper_2108_05815_amd import binding as B
    from paper_2108_05815_amd import serve as S
    for budget in (1 << 26, 1 << 30, 64 << 30):
        cap = S.lineage_capacity_for_budget(budget, 1024)
        assert B.server_bytes(cap, 1024) <= budget < B.server_bytes(cap + 1, 1024) or cap == (1 << 30) - 1


def test_request_stream_is_seeded_and_mixed():
    a1, s1 = W.config5_requests(duration=2.0)
    a2, s2 = W.config5_requests(duration=2.0)
    assert np.array_equal(a1, a2) and s1 == s2
    assert np.all(np.diff(a1) >= 0) and 300 < len(a1) < 500
    kinds = [s["kind"] for s in s1]
    assert 0.35 < kinds.count("spatial") / len(kinds) < 0.65
    wl = W.materialize(s1[0])
    assert wl.individuals == W.spec_individuals(s1[0])
    for s in s1[:50]:
        assert 1e-6 <= s["nu"] <= 1e-2
        if s["kind"] == "spatial":
            assert 64 <= s["L"] <= 512 and 1 <= s["cap"] <= 4 and 2 * s["R"] + 1 <= s["L"]


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_record_goes_stale_with_the_kernel(tmp_path):
    bench = _bench()
    src = os.path.join(ROOT, "paper_2108_05815_amd", "csrc", "necsim_hip.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    good = tmp_path / "t.txt"
    good.write_text(f"# test\nkernel_source_sha256: {digest}\nbytes_per_launch: 1234.5\n")
    assert bench.traffic_from_profile(str(good)) == 1234.5
    stale = tmp_path / "s.txt"
    stale.write_text("kernel_source_sha256: 00\nbytes_per_launch: 1\n")
    assert bench.traffic_from_profile(str(stale)) is None
    assert bench.traffic_from_profile(str(tmp_path / "missing.txt")) is None


@pytest.mark.parametrize("case", range(3))
def test_chain_events_is_the_longest_sample_path(case):
    """bench.py's serial-chain length, read from an event stream, equals the most events any
    sample's lineage goes through (the oracle tracing each sample alone)."""
    import numpy as np
    import bench
    import oracle
    from paper_2108_05815_amd import workloads as W
    cap, w, nu, seed = [(np.ones((16, 16), np.uint32), W.gaussian_kernel(1.5, 3), 0.02, 3),
                        (np.full((10, 10), 2, np.uint32), np.ones((3, 3)), 0.01, 5),
                        (np.array([[50]], np.uint32), np.ones((1, 1)), 0.01, 7)][case]
    sc = oracle.Scenario(cap, w, nu)
    s = np.arange(sc.individuals, dtype=np.uint64)
    ev, co = sc.event_stream(seed, s)
    e = np.zeros(len(ev["t"]), dtype=[("t", "<f8"), ("t_prior", "<f8"), ("origin", "<u4"), ("outcome", "<u4")])
    e["t"], e["t_prior"], e["origin"], e["outcome"] = ev["t"], ev["prior"], ev["origin"], ev["outcome"]
    c = np.zeros(len(co["t"]), dtype=[("t", "<f8"), ("t_parent", "<f8"), ("loc", "<u4"), ("reserved", "<u4")])
    c["t"], c["t_parent"], c["loc"] = co["t"], co["parent"], co["loc"]
    _, _, events = sc.simulate_naive(seed, s)
    assert bench.chain_events(e, c) == int(events.max())


@pytest.mark.parametrize("case", range(3))
def test_window_maxima_are_the_busiest_sample_path_of_each_window(case):
    """bench.py's per-window maxima, read from an event stream, equal the most events that any
    sample's own path (the oracle tracing it alone) has inside each horizon window, for several
    horizon schedules."""
    import types

    import numpy as np
    import bench
    import oracle
    from paper_2108_05815_amd import workloads as W
    cap, w, nu, seed = [(np.ones((16, 16), np.uint32), W.gaussian_kernel(1.5, 3), 0.02, 3),
                        (np.full((10, 10), 2, np.uint32), np.ones((3, 3)), 0.01, 5),
                        (np.array([[50]], np.uint32), np.ones((1, 1)), 0.01, 7)][case]
    sc = oracle.Scenario(cap, w, nu)
    s = np.arange(sc.individuals, dtype=np.uint64)
    ev, co = sc.event_stream(seed, s)
    e = np.zeros(len(ev["t"]), dtype=[("t", "<f8"), ("t_prior", "<f8"), ("origin", "<u4"), ("outcome", "<u4")])
    e["t"], e["t_prior"], e["origin"], e["outcome"] = ev["t"], ev["prior"], ev["origin"], ev["outcome"]
    c = np.zeros(len(co["t"]), dtype=[("t", "<f8"), ("t_parent", "<f8"), ("loc", "<u4"), ("reserved", "<u4")])
    c["t"], c["t_parent"], c["loc"] = co["t"], co["parent"], co["loc"]
    traces = []
    for x in s:
        times, _, _, _, done = sc.trace(seed, int(x))
        assert done
        traces.append(times)
    for h0, g, smax in [(0.5, 1.25, 4096.0), (2.0, 2.0, 8.0), (1.0, 3.0, 4096.0)]:
        h = bench.horizon_table(types.SimpleNamespace(horizon0=h0, horizon_growth=g, horizon_step_max=smax),
                                float(e["t"].max()))
        assert h[:2] == [0.0, h0] and all(b - a <= smax + 1e-12 for a, b in zip(h, h[1:]))
        got = bench.window_maxima(e, c, h)
        want = np.zeros(len(got), np.int64)
        for times in traces:
            k = np.searchsorted(np.asarray(h), times, side="left") - 1
            want = np.maximum(want, np.bincount(k, minlength=len(got)))
        assert got == want.tolist() and sum(got) >= bench.chain_events(e, c)
