"""GPU tests of the continuous-batching engine (nh_server_*): jobs submitted while others
run are admitted as lineage slots free up, and each result is bitwise the same as the
job run alone (and as the oracle), on a hand-picked mix and on the served request
stream of config 5 (every request against the culled oracle)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2108_05815_amd import workloads as W
from reporters_check import check_reporters

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-serving]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2108_05815_amd import binding as B
    return B, torch


def _mix():
    wl = [W.nonspatial(1000, 0.1, [s], name=f"C1 seed {s}") for s in range(6)]
    wl += [W.spatial_torus(24, 2, 1.5, 4, 0.02, [5], name="torus 24"),
           W.spatial_torus(37, 3, 2.5, 9, 0.004, [6], name="torus 37"),
           W.Workload("fractal 61", W.fractal_capacity(61, 12, base_period=16), W.gaussian_kernel(3.0, 8), 0.003, 1,
                      None, [2**63 + 11]),
           W.nonspatial(20000, 1e-3, [77], name="nonspatial J=20000"),
           W.spatial_torus(64, 1, 2.0, 10, 1e-3, [8], name="torus 64 C2-like")]
    for w in wl:
        if w.samples is None:
            w.samples = np.arange(int(w.capacity.astype(np.uint64).sum()), dtype=np.uint64)
    return wl


SOLO = [None, (256, 64.0), (1 << 30, 8.0), (256, 64.0, 4), (16, 512.0, 1)]


@pytest.mark.parametrize("solo", SOLO, ids=["default", "solo 256 step 64", "all solo step 8",
                                             "solo 256 step 64 tail lane 4", "solo 16 tail lane 1"])
def test_served_results_equal_alone_and_oracle(env, solo):
    B, torch = env
    dev = torch.device("cuda:0")
    wls = _mix()
    scns = [B.Scenario.from_workload(w) for w in wls]
    biggest = max(len(w.samples) for w in wls)
    cfg = None if solo is None else B.make_config(solo_max=solo[0], solo_step=solo[1])
    say("solo setting", solo)
    # a pool that holds the biggest job but not everything at once: admissions must wait
    srv = B.Server(lineage_capacity=biggest + 3000, max_jobs=8, lookahead=4, config=cfg,
                   tail_blocks=solo[2] if solo is not None and len(solo) > 2 else 0)
    outs, submitted = {}, 0
    order = list(range(len(wls)))
    done = {}
    step = 0
    while len(done) < len(wls):
        # stagger: submit one more job every few progress calls
        if submitted < len(order) and step % 3 == 0:
            k = order[submitted]
            s = torch.from_numpy(wls[k].samples.astype(np.int64)).to(dev)
            o = torch.empty(len(wls[k].samples), dtype=torch.int64, device=dev)
            r = torch.zeros(1, dtype=torch.int64, device=dev)
            rep = None
            if k % 2 == 0:  # every other job also asks for the reporters
                n = len(wls[k].samples)
                rep = {"spec_loc": torch.empty(n, dtype=torch.int32, device=dev),
                       "spec_time": torch.empty(n, dtype=torch.float64, device=dev),
                       "abundance_ids": torch.empty(n, dtype=torch.int64, device=dev),
                       "abundance_counts": torch.empty(n, dtype=torch.int32, device=dev)}
            srv.submit(k, scns[k], wls[k].seeds[0], s, o, r, reporters=rep)
            outs[k] = (o, r, rep)
            submitted += 1
        srv.progress()
        for c in srv.poll():
            done[c["tag"]] = c
        step += 1
        assert step < 10_000_000
    srv.drain(60.0)
    for k, w in enumerate(wls):
        c = done[k]
        assert c["status"] == 0 and c["lineages"] == len(w.samples)
        got = outs[k][0].cpu().numpy().view(np.uint64)
        alone, rich, _ = B.simulate(scns[k], w.seeds[0], w.samples)
        assert np.array_equal(got, alone), w.name
        assert int(outs[k][1].item()) == rich == c["richness"]
        if outs[k][2] is not None:
            check_reporters(got, rich, outs[k][2], w.seeds[0])
        say(w.name, "rounds", c["rounds"], "richness", rich)
    # every job against the oracle
    for k, w in enumerate(wls):
        ref, _, _ = oracle.Scenario(w.capacity, w.weights, w.nu, mode=w.mode).simulate_culled(w.seeds[0], w.samples,
                                                                                              2.0)
        assert np.array_equal(outs[k][0].cpu().numpy().view(np.uint64), ref), w.name
    srv.close()


def test_server_isolates_bad_and_empty_jobs(env):
    B, torch = env
    dev = torch.device("cuda:0")
    w = W.spatial_torus(24, 2, 1.5, 4, 0.02, [5])
    scn = B.Scenario.from_workload(w)
    srv = B.Server(lineage_capacity=10_000, max_jobs=4)
    good = torch.from_numpy(w.samples.astype(np.int64)).to(dev)
    out_good = torch.empty(len(w.samples), dtype=torch.int64, device=dev)
    bad = torch.tensor([0, scn.individuals + 5, 3], dtype=torch.int64, device=dev)
    out_bad = torch.empty(3, dtype=torch.int64, device=dev)
    empty = torch.zeros(0, dtype=torch.int64, device=dev)
    out_empty = torch.zeros(0, dtype=torch.int64, device=dev)
    rich_empty = torch.full((1,), 7, dtype=torch.int64, device=dev)
    srv.submit(1, scn, 5, good, out_good)
    srv.submit(2, scn, 5, bad, out_bad)
    srv.submit(3, scn, 5, empty, out_empty, rich_empty)
    srv.drain(60.0)
    res = {c["tag"]: c for c in srv.poll()}
    assert res[1]["status"] == 0 and res[2]["status"] == B.NH_EINVAL and res[3]["status"] == 0
    assert int(rich_empty.item()) == 0 and res[3]["richness"] == 0
    alone, _, _ = B.simulate(scn, 5, w.samples)
    assert np.array_equal(out_good.cpu().numpy().view(np.uint64), alone)
    with pytest.raises(B.NecsimError):
        too_big = torch.zeros(20_000, dtype=torch.int64, device=dev)
        srv.submit(9, scn, 5, too_big, torch.empty(20_000, dtype=torch.int64, device=dev))
    srv.close()


def test_served_config5_stream_equals_the_oracle(env):
    """The first 5 s of the config-5 request stream (Poisson 200 req/s; half config-4-like tori, half
    non-spatial demes with J up to 10^6; nu down to 10^-6), served through the continuous-batching
    server exactly as the benchmark serves it: every request's species array (by SHA-256) and
    richness equal the culled oracle's, computed meanwhile in a host process pool."""
    B, torch = env
    from paper_2108_05815_amd import serve as S
    here = os.path.dirname(os.path.abspath(__file__))
    pool = subprocess.Popen([sys.executable, os.path.join(here, "oracle_pool.py"), "--config", "5",
                             "--serve-seconds", "5", "--workers", "16"],
                            stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
    try:
        arrivals, specs = W.config5_requests(duration=5.0)
        big_slow = [k for k, sp in enumerate(specs) if sp["kind"] == "nonspatial" and sp["J"] >= 1e5 and sp["nu"] <= 1e-5]
        say(f"config 5: {len(specs)} requests, {len(big_slow)} non-spatial with J >= 1e5 and nu <= 1e-5")
        assert big_slow, "the stream has no large slow non-spatial request"
        free, _ = torch.cuda.mem_get_info()
        served = S.run_served(arrivals, specs, hbm_budget_bytes=int(0.8 * free), collect=True)
        say(f"config 5: served p50 {served['latency']['p50_ms']:.1f} ms, p99 {served['latency']['p99_ms']:.1f} ms")
        say("config 5: waiting for the oracle pool")
        out, err = pool.communicate(timeout=900)
    finally:
        if pool.poll() is None:
            pool.kill()
            pool.wait()
    assert pool.returncode == 0, err[-2000:]
    ref = {d["k"]: d for d in (json.loads(line) for line in out.splitlines() if line.startswith("{"))}
    assert sorted(ref) == list(range(len(specs))) == sorted(served["results"])
    bad = [k for k in range(len(specs))
           if served["results"][k] != (ref[k]["richness"], ref[k]["sha256"])]
    assert not bad, f"{len(bad)} served requests differ from the oracle, e.g. {[specs[k]['name'] for k in bad[:5]]}"
    say("config 5: all", len(specs), "served requests equal the oracle")
