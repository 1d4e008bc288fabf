"""GPU parity: species identities from the HIP library (through the C ABI)
must equal the CPU oracle's bit for bit, on the same seeded inputs.

Small and ragged cases are compared in full, and so are the full-size
workloads: configs 1 and 2 directly, the 1024 x 1024 habitat (config 3) and the
256-scenario mix (config 4) by a digest of each species array against the
culled oracle run meanwhile in host processes (tests/oracle_pool.py), together
with properties that hold at any size (richness = distinct ids, duplicates
agree, results independent of batching, launch form and tuning)."""
import os
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2108_05815_amd import workloads as W
from reporters_check import check_reporters

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-parity]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2108_05815_amd import binding
    return binding


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def _run(B, wl, seed, samples=None):
    scn = B.Scenario.from_workload(wl)
    s = wl.samples if samples is None else samples
    return B.simulate(scn, seed, s)


# --------------------------------------------------------------------------- #
# Config 1: non-spatial J = 1000, nu = 0.1, 1000 seeds                        #
# --------------------------------------------------------------------------- #

def test_config1_all_seeds_batched_and_plain(B, torch_mod):
    torch = torch_mod
    wl = W.config1(1000)
    osc = oracle.Scenario(wl.capacity, wl.weights, wl.nu)
    scn = B.Scenario.from_workload(wl)
    dev = torch.device("cuda:0")
    samples = torch.from_numpy(wl.samples.astype(np.int64)).to(dev)
    outs = [torch.empty(len(wl.samples), dtype=torch.int64, device=dev) for _ in wl.seeds]
    rich = torch.zeros(len(wl.seeds), dtype=torch.int64, device=dev)
    jobs = [(scn, seed, samples, outs[k], rich[k:k + 1]) for k, seed in enumerate(wl.seeds)]
    ws = torch.empty(B.workspace_bytes(len(wl.samples) * len(wl.seeds), len(jobs)), dtype=torch.uint8, device=dev)
    say("config 1: 1000 seeds in one batch")
    stats = B.batch_run(jobs, ws)
    torch.cuda.synchronize()
    got_rich = rich.cpu().numpy()
    richs = []
    for k, seed in enumerate(wl.seeds):
        ref, _, _ = osc.simulate_naive(seed, wl.samples)
        got = outs[k].cpu().numpy().view(np.uint64)
        assert np.array_equal(got, ref), f"seed {seed}"
        r = oracle.richness(ref)
        assert got_rich[k] == r and stats[k]["richness"] == r
        richs.append(r)
    # the GPU results obey the closed form too (Ewens mean, theta = J nu / (1 - nu))
    th = 1000 * 0.1 / 0.9
    expected = sum(th / (th + i) for i in range(1000))
    richs = np.array(richs, float)
    assert abs(richs.mean() - expected) < 4 * richs.std(ddof=1) / np.sqrt(len(richs))
    say("config 1: plain form, 25 seeds")
    for seed in range(25):
        got, r, st = B.simulate(scn, seed, wl.samples)
        assert np.array_equal(got, outs[seed].cpu().numpy().view(np.uint64))
        assert r == got_rich[seed] and st["lineages"] == 1000


# --------------------------------------------------------------------------- #
# Small and ragged workloads, compared in full                                 #
# --------------------------------------------------------------------------- #

SMALL = [
    W.nonspatial(300, 0.05, [4], name="nonspatial J=300"),
    W.nonspatial(1, 0.01, [5], name="nonspatial J=1"),
    W.spatial_torus(24, 2, 1.5, 4, 0.02, [5], name="torus 24x24 cap2 R4"),
    W.spatial_torus(37, 3, 2.5, 9, 0.004, [6], name="torus 37x37 cap3 R9"),
    W.Workload("fractal 24 per-deme", W.fractal_capacity(24, 11, base_period=8), W.gaussian_kernel(2.0, 5), 0.02, 1,
               None, [6]),
    W.Workload("fractal 61 per-deme", W.fractal_capacity(61, 12, base_period=16), W.gaussian_kernel(3.0, 8), 0.003,
               1, None, [2**64 - 1]),
    W.Workload("3x3 cap1 flat", np.ones((3, 3), np.uint32), np.ones((3, 3)), 0.1, 0, None, [0]),
    W.spatial_torus(16, 1, 1.0, 0, 0.05, [7], name="no dispersal"),
    W.spatial_torus(20, 2, 1.0, 2, 1.0, [8], name="nu = 1"),
]


@pytest.mark.parametrize("wl", SMALL, ids=[w.name for w in SMALL])
def test_small_workloads_full(B, wl):
    osc = oracle.Scenario(wl.capacity, wl.weights, wl.nu, mode=wl.mode)
    samples = np.arange(osc.individuals, dtype=np.uint64)
    seed = wl.seeds[0]
    say(wl.name, "n =", len(samples))
    ref, _, _ = osc.simulate_culled(seed, samples, 2.0)
    got, rich, st = _run(B, wl, seed, samples)
    assert np.array_equal(got, ref)
    assert rich == oracle.richness(ref) == st["richness"]
    assert st["speciated"] + st["merged"] == len(samples)
    # the same through device buffers, every round in 8-lanes-per-lineage groups, and one lane per lineage
    import torch
    dev = torch.device("cuda:0")
    scn = B.Scenario.from_workload(wl)
    d_s = torch.from_numpy(samples.astype(np.int64)).to(dev)
    ws = torch.empty(B.workspace_bytes(len(samples), 1), dtype=torch.uint8, device=dev)
    for coop, launch in ((1 << 30, B.NH_LAUNCH_PERSISTENT), (1, B.NH_LAUNCH_PERSISTENT),
                         (1 << 30, B.NH_LAUNCH_GRAPHS), (1, B.NH_LAUNCH_GRAPHS)):
        out = torch.empty(len(samples), dtype=torch.int64, device=dev)
        st2 = B.batch_run([(scn, seed, d_s, out, None)], ws, B.make_config(coop_max=coop, launch=launch))[0]
        assert np.array_equal(out.cpu().numpy().view(np.uint64), ref), (coop, launch)
        assert st2["events"] == st["events"] or coop == 1


def test_subsets_permutations_duplicates(B):
    wl = SMALL[3]
    scn = B.Scenario.from_workload(wl)
    osc = oracle.Scenario(wl.capacity, wl.weights, wl.nu)
    n = osc.individuals
    full, _, _ = B.simulate(scn, 9, np.arange(n, dtype=np.uint64))
    rng = np.random.default_rng(1)
    for size in (1, 2, 63, 64, 65, 1000, 5000):
        sub = rng.choice(n, size=size, replace=True).astype(np.uint64)
        say("subset", size)
        got, rich, _ = B.simulate(scn, 9, sub)
        assert np.array_equal(got, full[sub.astype(np.int64)])
        assert rich == len(np.unique(got))
    ref, _, _ = osc.simulate_naive(9, np.arange(0, n, 97, dtype=np.uint64))
    assert np.array_equal(full[::97], ref)


def test_empty_sample_list(B):
    scn = B.Scenario.from_workload(SMALL[0])
    got, rich, st = B.simulate(scn, 1, np.zeros(0, np.uint64))
    assert got.shape == (0,) and rich == 0


def test_rejects_out_of_range_sample_on_device(B, torch_mod):
    torch = torch_mod
    wl = SMALL[2]
    scn = B.Scenario.from_workload(wl)
    dev = torch.device("cuda:0")
    bad = torch.tensor([0, 5, scn.individuals], dtype=torch.int64, device=dev)
    out = torch.empty(3, dtype=torch.int64, device=dev)
    ws = torch.empty(B.workspace_bytes(3, 1), dtype=torch.uint8, device=dev)
    with pytest.raises(B.NecsimError) as e:
        B.batch_run([(scn, 1, bad, out, None)], ws)
    assert e.value.code == B.NH_EINVAL
    # the library is still usable afterwards
    got, _, _ = B.simulate(scn, 1, np.array([0, 5], np.uint64))
    ref, _, _ = oracle.Scenario(wl.capacity, wl.weights, wl.nu).simulate_naive(1, np.array([0, 5], np.uint64))
    assert np.array_equal(got, ref)


def test_rejects_small_workspace(B, torch_mod):
    torch = torch_mod
    scn = B.Scenario.from_workload(SMALL[0])
    dev = torch.device("cuda:0")
    s = torch.arange(10, dtype=torch.int64, device=dev)
    out = torch.empty(10, dtype=torch.int64, device=dev)
    ws = torch.empty(B.workspace_bytes(10, 1) - 256, dtype=torch.uint8, device=dev)
    with pytest.raises(B.NecsimError) as e:
        B.batch_run([(scn, 1, s, out, None)], ws)
    assert e.value.code == B.NH_ENOMEM


# --------------------------------------------------------------------------- #
# Config 2: 256 x 256 torus, 65,536 lineages, compared in full                 #
# --------------------------------------------------------------------------- #

def test_config2_full_bitexact(B):
    wl = W.config2(seeds=(42, 43, 44))
    scn = B.Scenario.from_workload(wl)
    osc = oracle.Scenario(wl.capacity, wl.weights, wl.nu)
    for seed in wl.seeds:
        say("config 2 seed", seed)
        got, rich, st = B.simulate(scn, seed, wl.samples)
        ref, ev, _ = osc.simulate_culled(seed, wl.samples, 1.0)
        assert np.array_equal(got, ref)
        assert rich == oracle.richness(ref)
        assert st["speciated"] + st["merged"] == 65536


def test_tuning_never_changes_results(B, torch_mod):
    """Horizon schedule, block size, occupancy, graph length and the lanes-per-lineage switch are
    performance knobs only."""
    torch = torch_mod
    wl = W.config2()
    scn = B.Scenario.from_workload(wl)
    dev = torch.device("cuda:0")
    samples = torch.from_numpy(wl.samples.astype(np.int64)).to(dev)
    ws = torch.empty(B.workspace_bytes(len(wl.samples), 1), dtype=torch.uint8, device=dev)
    base = None
    for cfg in (dict(), dict(horizon0=0.125, horizon_growth=1.05), dict(horizon0=8.0, horizon_growth=2.0),
                dict(block_size=64, blocks_per_cu=1, rounds_per_graph=1), dict(block_size=128, blocks_per_cu=8),
                dict(horizon_step_max=1.0, rounds_per_graph=32), dict(coop_max=1), dict(coop_max=1 << 30),
                dict(coop_max=1 << 30, block_size=64, horizon0=2.0), dict(launch=B.NH_LAUNCH_GRAPHS),
                dict(launch=B.NH_LAUNCH_GRAPHS, block_size=64, blocks_per_cu=1, rounds_per_graph=1),
                dict(launch=B.NH_LAUNCH_GRAPHS, horizon_step_max=1.0, rounds_per_graph=32)):
        say("config 2 tuning", cfg)
        out = torch.empty(len(wl.samples), dtype=torch.int64, device=dev)
        B.batch_run([(scn, 42, samples, out, None)], ws, B.make_config(**cfg))
        got = out.cpu().numpy()
        if base is None:
            base = got
        assert np.array_equal(got, base)


def test_repeat_runs_are_identical(B):
    wl = W.config2()
    scn = B.Scenario.from_workload(wl)
    a, ra, sa = B.simulate(scn, 7, wl.samples)
    b, rb, sb = B.simulate(scn, 7, wl.samples[::-1].copy())
    assert np.array_equal(a, b[::-1]) and ra == rb
    assert sa["events"] == sb["events"]


# --------------------------------------------------------------------------- #
# Config 3: 1024 x 1024 fractal habitat, per-deme tables, sampled outputs       #
# --------------------------------------------------------------------------- #

def _start_pool(*args):
    """The culled oracle of a whole configuration in a separate host process pool (tests/oracle_pool.py)."""
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    return subprocess.Popen([sys.executable, os.path.join(here, "oracle_pool.py"), *args],
                            stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)


def _pool_results(pool, timeout):
    import json
    try:
        out, err = pool.communicate(timeout=timeout)
    finally:
        if pool.poll() is None:
            pool.kill()
            pool.wait()
    assert pool.returncode == 0, err[-2000:]
    return [json.loads(line) for line in out.splitlines() if line.startswith("{")]


def _digest(a):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a).astype("<u8").tobytes()).hexdigest()


def test_config3_full_parity(B):
    """All 330,302 samples of the 1024 x 1024 habitat (per-deme tables, about 10 GiB) against the
    culled oracle over the same samples, run meanwhile in a host process (about a minute, about
    11 GB of lazily built per-deme tables), compared by the SHA-256 of the species array."""
    pool = _start_pool("--config", "3", "--split", "1", "--workers", "1")
    try:
        wl = W.config3()
        say("config 3: building per-deme tables")
        t0 = time.time()
        scn = B.Scenario.from_workload(wl)
        say(f"config 3: tables {scn.table_bytes / 2**30:.2f} GiB in {time.time() - t0:.1f} s; simulating",
            len(wl.samples))
        got, rich, st = B.simulate(scn, wl.seeds[0], wl.samples)
        say("config 3:", st)
        assert rich == len(np.unique(got))
        assert st["speciated"] + st["merged"] == len(wl.samples)
        scn.close()
        say("config 3: waiting for the oracle (all samples, culled)")
        lines = _pool_results(pool, 900)
    finally:
        if pool.poll() is None:
            pool.kill()
            pool.wait()
    ref = [d for d in lines if "sha256" in d]
    say("config 3: oracle", [d for d in lines if "part" in d])
    assert len(ref) == 1
    if _digest(got) != ref[0]["sha256"]:  # name the first differing samples, traced one by one
        osc = oracle.Scenario(wl.capacity, wl.weights, wl.nu, mode=1)
        pick = np.random.default_rng(3).choice(len(wl.samples), size=20, replace=False)
        exp, _, _ = osc.simulate_naive(wl.seeds[0], wl.samples[pick])
        raise AssertionError(f"config 3 species differ from the oracle; sampled mismatches: "
                             f"{np.flatnonzero(exp != got[pick]).tolist()}")
    assert rich == ref[0]["richness"]


# --------------------------------------------------------------------------- #
# Config 4: 256 scenarios in one batch                                         #
# --------------------------------------------------------------------------- #

def test_config4_full_parity_and_alone_equals_mix(B, torch_mod):
    """All 256 scenarios of the mix (38.6 M samples) in one batch: every species id equals the
    culled oracle's (run meanwhile in a separate process pool on the host's cores, compared by a
    digest of each scenario's species array), and a few scenarios run alone equal the mix."""
    torch = torch_mod
    pool = _start_pool("--config", "4", "--workers", "16")
    try:
        wls = W.config4()
        dev = torch.device("cuda:0")
        say("config 4: creating 256 scenarios")
        scns = [B.Scenario.from_workload(w) for w in wls]
        samples = [torch.from_numpy(w.samples.astype(np.int64)).to(dev) for w in wls]
        outs = [torch.empty(len(w.samples), dtype=torch.int64, device=dev) for w in wls]
        rich = torch.zeros(len(wls), dtype=torch.int64, device=dev)
        jobs = [(scns[k], wls[k].seeds[0], samples[k], outs[k], rich[k:k + 1]) for k in range(len(wls))]
        n_total = sum(len(w.samples) for w in wls)
        ws = torch.empty(B.workspace_bytes(n_total, len(jobs)), dtype=torch.uint8, device=dev)
        say("config 4: batch run of", n_total, "lineages")
        t0 = time.time()
        stats = B.batch_run(jobs, ws)
        torch.cuda.synchronize()
        say(f"config 4: {time.time() - t0:.2f} s, events {sum(s['events'] for s in stats)}")
        got_rich = rich.cpu().numpy()
        got = [outs[k].cpu().numpy().view(np.uint64) for k in range(len(wls))]
        for k in range(len(wls)):
            assert got_rich[k] == len(np.unique(got[k])) == stats[k]["richness"]
        say("config 4: waiting for the oracle pool")
        lines = _pool_results(pool, 600)
    finally:
        if pool.poll() is None:
            pool.kill()
            pool.wait()
    ref = {d["k"]: d for d in lines}
    assert sorted(ref) == list(range(len(wls)))
    bad = [k for k in range(len(wls)) if _digest(got[k]) != ref[k]["sha256"] or got_rich[k] != ref[k]["richness"]]
    if bad:  # name the first differing samples of the first bad scenario
        k = bad[0]
        osc = oracle.Scenario(wls[k].capacity, wls[k].weights, wls[k].nu, mode=wls[k].mode)
        exp, _, _ = osc.simulate_culled(wls[k].seeds[0], wls[k].samples, 2.0)
        diff = np.flatnonzero(exp != got[k])[:5]
        raise AssertionError(f"{len(bad)} scenarios differ; scenario {k} ({wls[k].name}) at samples {diff.tolist()}")
    say("config 4: all", len(wls), "scenarios equal the oracle")
    # batch-alone == batch-mix for a few scenarios of different sizes
    for k in (0, 1, 2, int(np.argmin([w.individuals for w in wls]))):
        say("config 4 alone:", wls[k].name)
        alone, r, _ = B.simulate(scns[k], wls[k].seeds[0], wls[k].samples)
        assert np.array_equal(alone, got[k])
        assert r == got_rich[k]


def test_solo_tails_never_change_results(B, torch_mod):
    """Routing nearly finished jobs to the solo queue (8 lanes per lineage, own horizon step) is a
    performance knob only: a batch of mixed scenarios gives the same ids under every setting."""
    torch = torch_mod
    dev = torch.device("cuda:0")
    wls = W.config4()[:24] + [SMALL[k] for k in (0, 2, 4, 5)]
    for w in wls:
        if w.samples is None:
            w.samples = np.arange(int(w.capacity.astype(np.uint64).sum()), dtype=np.uint64)
    scns = [B.Scenario.from_workload(w) for w in wls]
    samples = [torch.from_numpy(w.samples.astype(np.int64)).to(dev) for w in wls]
    n_total = sum(len(w.samples) for w in wls)
    ws = torch.empty(B.workspace_bytes(n_total, len(wls)), dtype=torch.uint8, device=dev)
    base = None
    for cfg in (dict(), dict(solo_max=64), dict(solo_max=4096, solo_step=8.0), dict(solo_max=64, solo_step=1e5),
                dict(solo_max=1 << 30, solo_step=64.0, coop_max=1), dict(endgame=4096),
                dict(endgame=64, solo_max=64), dict(endgame=1, launch=B.NH_LAUNCH_GRAPHS)):
        say("solo setting", cfg, "lineages", n_total)
        outs = [torch.empty(len(w.samples), dtype=torch.int64, device=dev) for w in wls]
        rich = torch.zeros(len(wls), dtype=torch.int64, device=dev)
        jobs = [(scns[k], wls[k].seeds[0], samples[k], outs[k], rich[k:k + 1]) for k in range(len(wls))]
        st = B.batch_run(jobs, ws, B.make_config(**cfg))
        got = [o.cpu().numpy() for o in outs] + [rich.cpu().numpy()]
        assert all(s["speciated"] + s["merged"] == len(w.samples) for s, w in zip(st, wls))
        if base is None:
            base = got
        else:
            for a, b in zip(got, base):
                assert np.array_equal(a, b)


@pytest.mark.parametrize("launch", [0, 1], ids=["persistent", "graphs"])
def test_checkpoint_resume_equals_uninterrupted(B, torch_mod, launch):
    """A run suspended between rounds, its workspace copied to the host, the device copy destroyed
    and the bytes restored (in place, then into another buffer) finishes with bitwise the same ids,
    richness and event counts as an uninterrupted run; a multi-job batch also resumes under other
    tuning knobs (and the other launch form)."""
    torch = torch_mod
    mk = lambda **kw: B.make_config(launch=launch, **kw)  # noqa: E731
    dev = torch.device("cuda:0")
    wl = W.config2()
    scn = B.Scenario.from_workload(wl)
    n = len(wl.samples)
    s = torch.from_numpy(wl.samples.astype(np.int64)).to(dev)
    nbytes = B.workspace_bytes(n, 1)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    ref = torch.empty(n, dtype=torch.int64, device=dev)
    rich_ref = torch.zeros(1, dtype=torch.int64, device=dev)
    st_ref = B.batch_run([(scn, 42, s, ref, rich_ref)], ws, mk())[0]
    assert not st_ref["suspended"]
    out = torch.empty(n, dtype=torch.int64, device=dev)
    rich = torch.zeros(1, dtype=torch.int64, device=dev)
    job = [(scn, 42, s, out, rich)]
    cap = mk(max_rounds=3)
    st = B.batch_run(job, ws, cap)[0]
    say("checkpoint: suspended after", st["rounds"], "rounds")
    assert st["suspended"] and 3 <= st["rounds"] < st_ref["rounds"]
    host = ws.cpu()
    ws.fill_(0xA5)  # the device copy is gone
    ws.copy_(host.to(dev))
    st = B.batch_resume(job, ws, cap)[0]
    assert st["suspended"] and st["rounds"] < st_ref["rounds"]
    host = ws.cpu()
    ws.fill_(0x5A)
    ws2 = torch.empty(nbytes + 512, dtype=torch.uint8, device=dev)[256:256 + nbytes]  # another buffer
    assert ws2.data_ptr() != ws.data_ptr() and ws2.data_ptr() % 256 == 0
    ws2.copy_(host.to(dev))
    st = B.batch_resume(job, ws2, mk())[0]
    assert not st["suspended"] and st["rounds"] == st_ref["rounds"]
    torch.cuda.synchronize()
    assert torch.equal(out, ref) and int(rich.item()) == int(rich_ref.item())
    assert st["events"] == st_ref["events"] and st["merged"] == st_ref["merged"]
    # several jobs, resumed with other knobs (knobs never change results)
    wls = W.config4()[:6] + [SMALL[k] for k in (0, 4)]
    for w in wls:
        if w.samples is None:
            w.samples = np.arange(int(w.capacity.astype(np.uint64).sum()), dtype=np.uint64)
    scns = [B.Scenario.from_workload(w) for w in wls]
    ss = [torch.from_numpy(w.samples.astype(np.int64)).to(dev) for w in wls]
    n_total = sum(len(w.samples) for w in wls)
    wsb = torch.empty(B.workspace_bytes(n_total, len(wls)), dtype=torch.uint8, device=dev)
    outs_a = [torch.empty(len(w.samples), dtype=torch.int64, device=dev) for w in wls]
    B.batch_run([(scns[k], wls[k].seeds[0], ss[k], outs_a[k], None) for k in range(len(wls))], wsb)
    outs_b = [torch.empty(len(w.samples), dtype=torch.int64, device=dev) for w in wls]
    jobs_b = [(scns[k], wls[k].seeds[0], ss[k], outs_b[k], None) for k in range(len(wls))]
    st = B.batch_run(jobs_b, wsb, mk(max_rounds=5, rounds_per_graph=1))
    assert st[0]["suspended"]
    st = B.batch_resume(jobs_b, wsb, B.make_config(block_size=128, blocks_per_cu=2, solo_max=64, launch=1 - launch))
    assert not st[0]["suspended"]
    for a, b in zip(outs_a, outs_b):
        assert torch.equal(a, b)


@pytest.mark.parametrize("launch", [0, 1], ids=["persistent", "graphs"])
def test_timed_out_run_fails_cleanly_and_reruns_bitwise(B, torch_mod, launch):
    """A run stopped by its wall-clock limit (forced from the host: every kernel still finishes its
    round) reports NH_ETIMEOUT; the same call afterwards gives the uninterrupted result."""
    torch = torch_mod
    dev = torch.device("cuda:0")
    wl = W.config2()
    scn = B.Scenario.from_workload(wl)
    n = len(wl.samples)
    s = torch.from_numpy(wl.samples.astype(np.int64)).to(dev)
    ws = torch.empty(B.workspace_bytes(n, 1), dtype=torch.uint8, device=dev)
    out = torch.empty(n, dtype=torch.int64, device=dev)
    with pytest.raises(B.NecsimError) as e:
        B.batch_run([(scn, 9, s, out, None)], ws, B.make_config(timeout_s=1e-9, launch=launch))
    assert e.value.code == B.NH_ETIMEOUT
    B.batch_run([(scn, 9, s, out, None)], ws, B.make_config(launch=launch))
    ref, _, _ = B.simulate(scn, 9, wl.samples)
    assert np.array_equal(out.cpu().numpy().view(np.uint64), ref)


def test_barrier_wait_limit_stops_the_run_and_the_kernel_exits(B, torch_mod):
    """A persistent run whose grid barrier wait limit is shorter than a round (forced from the host: a
    first horizon past the whole run makes one round of several milliseconds, the limit is 1 ms)
    stops with NH_EDEVICE; every workgroup leaves, and the next call gives the normal result."""
    torch = torch_mod
    dev = torch.device("cuda:0")
    wl = W.config2()
    scn = B.Scenario.from_workload(wl)
    n = len(wl.samples)
    s = torch.from_numpy(wl.samples.astype(np.int64)).to(dev)
    ws = torch.empty(B.workspace_bytes(n, 1), dtype=torch.uint8, device=dev)
    out = torch.empty(n, dtype=torch.int64, device=dev)
    with pytest.raises(B.NecsimError) as e:
        B.batch_run([(scn, 9, s, out, None)], ws, B.make_config(horizon0=1e7, coop_max=1, barrier_wait_ms=1))
    assert e.value.code == B.NH_EDEVICE and "barrier" in str(e.value)
    B.batch_run([(scn, 9, s, out, None)], ws)
    ref, _, _ = B.simulate(scn, 9, wl.samples)
    assert np.array_equal(out.cpu().numpy().view(np.uint64), ref)


def _reporters(torch, n, dev):
    return {"spec_loc": torch.empty(n, dtype=torch.int32, device=dev),
            "spec_time": torch.empty(n, dtype=torch.float64, device=dev),
            "abundance_ids": torch.empty(n, dtype=torch.int64, device=dev),
            "abundance_counts": torch.empty(n, dtype=torch.int32, device=dev)}


def test_reporters_match_the_oracle_and_the_species(B, torch_mod):
    """Speciation-event and abundance reporters in one batch of mixed scenarios."""
    torch = torch_mod
    dev = torch.device("cuda:0")
    wls = [SMALL[k] for k in (0, 1, 2, 3, 4, 5, 8)]
    samples = [np.arange(int(w.capacity.astype(np.uint64).sum()), dtype=np.uint64) for w in wls]
    scns = [B.Scenario.from_workload(w) for w in wls]
    ss = [torch.from_numpy(x.astype(np.int64)).to(dev) for x in samples]
    outs = [torch.empty(len(x), dtype=torch.int64, device=dev) for x in samples]
    rich = torch.zeros(len(wls), dtype=torch.int64, device=dev)
    reps = [_reporters(torch, len(x), dev) for x in samples]
    jobs = [(scns[k], wls[k].seeds[0], ss[k], outs[k], rich[k:k + 1], reps[k]) for k in range(len(wls))]
    n_total = sum(len(x) for x in samples)
    ws = torch.empty(B.workspace_bytes(n_total, len(wls)), dtype=torch.uint8, device=dev)
    B.batch_run(jobs, ws)
    torch.cuda.synchronize()
    for k, w in enumerate(wls):
        say("reporters:", w.name)
        sp = outs[k].cpu().numpy().view(np.uint64)
        osc = oracle.Scenario(w.capacity, w.weights, w.nu, mode=w.mode)
        ref, _, _ = osc.simulate_culled(w.seeds[0], samples[k], 2.0)
        assert np.array_equal(sp, ref)
        check_reporters(sp, int(rich[k].item()), reps[k], w.seeds[0], osc, samples[k])
    # pairs must be both or neither
    bad = dict(reps[0])
    bad["spec_time"] = None
    with pytest.raises(B.NecsimError):
        B.batch_run([(scns[0], 1, ss[0], outs[0], None, bad)], ws)


def _poisson(w):
    import copy
    x = copy.copy(w)
    x.sampler = 1
    if x.samples is None:
        x.samples = np.arange(int(x.capacity.astype(np.uint64).sum()), dtype=np.uint64)
    return x


POISSON = [_poisson(SMALL[k]) for k in (0, 2, 3, 5, 8)] + [
    _poisson(W.spatial_torus(24, 2, 1.5, 4, 0.02, [5], name="torus 24 lambda 4 dt 0.5")),
    _poisson(W.nonspatial(400, 0.05, [9], name="nonspatial J=400 lambda 0.25 dt 8"))]
POISSON[-2].lam, POISSON[-2].dt = 4.0, 0.5
POISSON[-1].lam, POISSON[-1].dt = 0.25, 8.0


@pytest.mark.parametrize("wl", POISSON, ids=[w.name for w in POISSON])
def test_poisson_sampler_bitexact(B, torch_mod, wl):
    """The Poisson-count event-time sampler: GPU == oracle for the plain entry point and for both
    lane layouts forced, with the speciation events of the reporters equal to the oracle's."""
    torch = torch_mod
    dev = torch.device("cuda:0")
    osc = oracle.Scenario(wl.capacity, wl.weights, wl.nu, mode=wl.mode, lam=wl.lam, dt=wl.dt, sampler=1)
    ref, _, _ = osc.simulate_culled(wl.seeds[0], wl.samples, 2.0)
    scn = B.Scenario.from_workload(wl)
    got, rich, _ = B.simulate(scn, wl.seeds[0], wl.samples)
    assert np.array_equal(got, ref) and rich == oracle.richness(ref)
    n = len(wl.samples)
    s = torch.from_numpy(wl.samples.astype(np.int64)).to(dev)
    ws = torch.empty(B.workspace_bytes(n, 1), dtype=torch.uint8, device=dev)
    for coop in (1 << 30, 1):
        out = torch.empty(n, dtype=torch.int64, device=dev)
        r1 = torch.zeros(1, dtype=torch.int64, device=dev)
        rep = _reporters(torch, n, dev)
        B.batch_run([(scn, wl.seeds[0], s, out, r1, rep)], ws, B.make_config(coop_max=coop))
        got = out.cpu().numpy().view(np.uint64)
        assert np.array_equal(got, ref), coop
        check_reporters(got, int(r1.item()), rep, wl.seeds[0], osc if n <= 2000 else None, wl.samples)


def test_poisson_sampler_torus_full_and_mixed_batch(B, torch_mod):
    """The 256x256 torus under the Poisson sampler, bit-exact; a batch mixing both samplers equals
    each job alone."""
    torch = torch_mod
    dev = torch.device("cuda:0")
    wl = _poisson(W.config2())
    osc = oracle.Scenario(wl.capacity, wl.weights, wl.nu, sampler=1)
    ref, _, _ = osc.simulate_culled(42, wl.samples, 16.0)
    scn_p = B.Scenario.from_workload(wl)
    got, _, _ = B.simulate(scn_p, 42, wl.samples)
    assert np.array_equal(got, ref)
    wl_e = W.config2()
    scn_e = B.Scenario.from_workload(wl_e)
    n = len(wl.samples)
    s = torch.from_numpy(wl.samples.astype(np.int64)).to(dev)
    outs = [torch.empty(n, dtype=torch.int64, device=dev) for _ in range(4)]
    jobs = [(scn_p, 42, s, outs[0], None), (scn_e, 42, s, outs[1], None), (scn_p, 43, s, outs[2], None),
            (scn_e, 43, s, outs[3], None)]
    ws = torch.empty(B.workspace_bytes(4 * n, 4), dtype=torch.uint8, device=dev)
    B.batch_run(jobs, ws, B.make_config(solo_max=64))
    assert np.array_equal(outs[0].cpu().numpy().view(np.uint64), ref)
    for k, (scn, seed) in enumerate([(scn_p, 42), (scn_e, 42), (scn_p, 43), (scn_e, 43)]):
        alone, _, _ = B.simulate(scn, seed, wl.samples)
        assert np.array_equal(outs[k].cpu().numpy().view(np.uint64), alone), k


IMPLICIT = [(3, 4, 0.3, 0.2, 0), (50, 400, 0.1, 0.01, 0), (1000, 20000, 0.02, 1e-3, 0), (200, 200, 1.0, 0.05, 0),
            (300, 3000, 0.05, 0.005, 1)]


@pytest.mark.parametrize("J,Jm,m,nu,sampler", IMPLICIT, ids=[f"J{c[0]}_Jm{c[1]}_m{c[2]}_s{c[4]}" for c in IMPLICIT])
def test_spatially_implicit_bitexact(B, torch_mod, J, Jm, m, nu, sampler):
    """The spatially implicit scenario: GPU == oracle for the local community's samples (and one
    run that also samples the metacommunity), both lane layouts, with the reporters."""
    torch = torch_mod
    dev = torch.device("cuda:0")
    osc = oracle.Scenario.implicit(J, Jm, m, nu, sampler=sampler)
    scn = B.Scenario.implicit(J, Jm, m, nu, sampler=sampler)
    for samples in (np.arange(J, dtype=np.uint64), np.arange(0, J + Jm, max(1, (J + Jm) // 500), dtype=np.uint64)):
        ref, _, _ = osc.simulate_culled(11, samples, 4.0)
        got, rich, _ = B.simulate(scn, 11, samples)
        assert np.array_equal(got, ref) and rich == oracle.richness(ref)
    samples = np.arange(J, dtype=np.uint64)
    ref, _, _ = osc.simulate_culled(11, samples, 4.0)
    s = torch.from_numpy(samples.astype(np.int64)).to(dev)
    ws = torch.empty(B.workspace_bytes(J, 1), dtype=torch.uint8, device=dev)
    for coop in (1 << 30, 1):
        out = torch.empty(J, dtype=torch.int64, device=dev)
        r1 = torch.zeros(1, dtype=torch.int64, device=dev)
        rep = _reporters(torch, J, dev)
        B.batch_run([(scn, 11, s, out, r1, rep)], ws, B.make_config(coop_max=coop))
        got = out.cpu().numpy().view(np.uint64)
        assert np.array_equal(got, ref), coop
        check_reporters(got, int(r1.item()), rep, 11, osc if J <= 300 else None, samples)


def test_spatially_implicit_in_a_mixed_batch(B, torch_mod):
    torch = torch_mod
    dev = torch.device("cuda:0")
    scns = [B.Scenario.implicit(400, 5000, 0.05, 2e-3), B.Scenario.from_workload(SMALL[2]),
            B.Scenario.implicit(100, 100, 0.5, 0.02, sampler=1), B.Scenario.from_workload(SMALL[0])]
    ns = [400, SMALL[2].individuals, 100, SMALL[0].individuals]
    ss = [torch.arange(n, dtype=torch.int64, device=dev) for n in ns]
    outs = [torch.empty(n, dtype=torch.int64, device=dev) for n in ns]
    ws = torch.empty(B.workspace_bytes(sum(ns), 4), dtype=torch.uint8, device=dev)
    B.batch_run([(scns[k], 5 + k, ss[k], outs[k], None) for k in range(4)], ws, B.make_config(solo_max=32))
    for k in range(4):
        alone, _, _ = B.simulate(scns[k], 5 + k, np.arange(ns[k], dtype=np.uint64))
        assert np.array_equal(outs[k].cpu().numpy().view(np.uint64), alone), k


def _protracted(w, tau, lam=None, dt=None, sampler=0):
    import copy
    x = copy.copy(w)
    x.tau, x.sampler = tau, sampler
    x.lam = x.lam if lam is None else lam
    x.dt = x.dt if dt is None else dt
    x.name = f"{w.name} tau={tau} lambda={x.lam} dt={x.dt} sampler={sampler}"
    if x.samples is None:
        x.samples = np.arange(int(x.capacity.astype(np.uint64).sum()), dtype=np.uint64)
    return x


# lambda = 0.3 is not a power of two, so tau / lambda is inexact and the threshold time the
# library derives must still decide exactly as lambda * t < tau does
PROTRACTED = [_protracted(SMALL[0], 10.0), _protracted(SMALL[2], 5.0), _protracted(SMALL[3], 40.0, lam=0.3),
              _protracted(SMALL[4], 3.0, lam=0.3), _protracted(SMALL[5], 25.0, sampler=1),
              _protracted(SMALL[2], 2.5, lam=4.0, dt=0.5, sampler=1), _protracted(SMALL[8], 1.0)]


@pytest.mark.parametrize("wl", PROTRACTED, ids=[w.name for w in PROTRACTED])
def test_protracted_speciation_bitexact(B, torch_mod, wl):
    """Protracted speciation: GPU == oracle for the plain entry point and both lane layouts, with
    every reported speciation at least tau generations old and equal to the oracle's event."""
    torch = torch_mod
    dev = torch.device("cuda:0")
    say(wl.name, "n =", len(wl.samples))
    osc = oracle.Scenario(wl.capacity, wl.weights, wl.nu, mode=wl.mode, lam=wl.lam, dt=wl.dt,
                          sampler=wl.sampler, tau=wl.tau)
    ref, _, _ = osc.simulate_culled(wl.seeds[0], wl.samples, 2.0)
    scn = B.Scenario.from_workload(wl)
    got, rich, _ = B.simulate(scn, wl.seeds[0], wl.samples)
    assert np.array_equal(got, ref) and rich == oracle.richness(ref)
    n = len(wl.samples)
    s = torch.from_numpy(wl.samples.astype(np.int64)).to(dev)
    ws = torch.empty(B.workspace_bytes(n, 1), dtype=torch.uint8, device=dev)
    for coop in (1 << 30, 1):
        out = torch.empty(n, dtype=torch.int64, device=dev)
        r1 = torch.zeros(1, dtype=torch.int64, device=dev)
        rep = _reporters(torch, n, dev)
        B.batch_run([(scn, wl.seeds[0], s, out, r1, rep)], ws, B.make_config(coop_max=coop))
        got = out.cpu().numpy().view(np.uint64)
        assert np.array_equal(got, ref), coop
        check_reporters(got, int(r1.item()), rep, wl.seeds[0], osc if n <= 2000 else None, wl.samples)
        assert (wl.lam * rep["spec_time"].cpu().numpy() >= wl.tau).all()


def test_protracted_speciation_torus_full_implicit_and_mixed_batch(B, torch_mod):
    """The 256x256 torus with tau = 20 generations, bit-exact; the spatially implicit scenario with
    tau; a batch mixing point and protracted speciation equals each job alone."""
    torch = torch_mod
    dev = torch.device("cuda:0")
    wl = _protracted(W.config2(), 20.0)
    say(wl.name)
    osc = oracle.Scenario(wl.capacity, wl.weights, wl.nu, tau=20.0)
    ref, _, _ = osc.simulate_culled(42, wl.samples, 16.0)
    scn_p = B.Scenario.from_workload(wl)
    got, rich_p, _ = B.simulate(scn_p, 42, wl.samples)
    assert np.array_equal(got, ref)
    scn_e = B.Scenario.from_workload(W.config2())
    _, rich_e, _ = B.simulate(scn_e, 42, wl.samples)
    assert rich_p < rich_e  # young species no longer count
    J, Jm = 300, 3000
    oimp = oracle.Scenario.implicit(J, Jm, 0.05, 0.005, tau=4.0)
    gimp = B.Scenario.implicit(J, Jm, 0.05, 0.005, tau=4.0)
    samples = np.arange(J, dtype=np.uint64)
    assert np.array_equal(B.simulate(gimp, 11, samples)[0], oimp.simulate_culled(11, samples, 4.0)[0])
    n = len(wl.samples)
    s = torch.from_numpy(wl.samples.astype(np.int64)).to(dev)
    si = torch.from_numpy(samples.astype(np.int64)).to(dev)
    outs = [torch.empty(n, dtype=torch.int64, device=dev) for _ in range(3)] + [
        torch.empty(J, dtype=torch.int64, device=dev)]
    jobs = [(scn_p, 42, s, outs[0], None), (scn_e, 42, s, outs[1], None), (scn_p, 43, s, outs[2], None),
            (gimp, 11, si, outs[3], None)]
    ws = torch.empty(B.workspace_bytes(3 * n + J, 4), dtype=torch.uint8, device=dev)
    B.batch_run(jobs, ws, B.make_config(solo_max=64))
    assert np.array_equal(outs[0].cpu().numpy().view(np.uint64), ref)
    for k, (scn, seed, smp) in enumerate([(scn_p, 42, wl.samples), (scn_e, 42, wl.samples),
                                          (scn_p, 43, wl.samples), (gimp, 11, samples)]):
        alone, _, _ = B.simulate(scn, seed, smp)
        assert np.array_equal(outs[k].cpu().numpy().view(np.uint64), alone), k


def _rates(w, lam, dt):
    import copy
    x = copy.copy(w)
    x.lam, x.dt = lam, dt
    x.name = f"{w.name} lambda={lam} dt={dt}"
    if x.samples is None:
        x.samples = np.arange(int(x.capacity.astype(np.uint64).sum()), dtype=np.uint64)
    return x


# lambda dt from 1/64 (most searches find no event in the next five intervals) to 64 (every
# interval needs far more than four draws): both ends leave the group step for its slow search
RATES = [_rates(SMALL[2], 1.0, 16.0), _rates(SMALL[2], 1.0, 1.0 / 64), _rates(SMALL[2], 64.0, 1.0),
         _rates(SMALL[4], 4.0, 0.5), _rates(SMALL[0], 0.25, 8.0), _rates(SMALL[3], 2.0, 4.0)]


@pytest.mark.parametrize("wl", RATES, ids=[w.name for w in RATES])
def test_exponential_sampler_rate_and_interval_extremes(B, torch_mod, wl):
    """The exponential-sum sampler away from lambda dt = 1, bit-exact in both lane layouts."""
    torch = torch_mod
    dev = torch.device("cuda:0")
    say(wl.name, "n =", len(wl.samples))
    osc = oracle.Scenario(wl.capacity, wl.weights, wl.nu, mode=wl.mode, lam=wl.lam, dt=wl.dt)
    ref, _, _ = osc.simulate_culled(wl.seeds[0], wl.samples, 2.0 / wl.lam)
    scn = B.Scenario.from_workload(wl)
    n = len(wl.samples)
    s = torch.from_numpy(wl.samples.astype(np.int64)).to(dev)
    ws = torch.empty(B.workspace_bytes(n, 1), dtype=torch.uint8, device=dev)
    for coop in (1 << 30, 1):
        out = torch.empty(n, dtype=torch.int64, device=dev)
        B.batch_run([(scn, wl.seeds[0], s, out, None)], ws, B.make_config(coop_max=coop))
        assert np.array_equal(out.cpu().numpy().view(np.uint64), ref), coop


def test_batch_with_empty_and_duplicate_jobs_and_device_entry_point(B, torch_mod):
    """Empty jobs inside a batch, the same job twice, and nh_simulate_device agree with the plain form."""
    import ctypes as C
    torch = torch_mod
    dev = torch.device("cuda:0")
    wl = SMALL[2]
    scn = B.Scenario.from_workload(wl)
    n = len(wl.samples)
    s = torch.from_numpy(wl.samples.astype(np.int64)).to(dev)
    empty = torch.zeros(0, dtype=torch.int64, device=dev)
    outs = [torch.empty(n, dtype=torch.int64, device=dev) for _ in range(2)]
    rich = torch.full((4,), -1, dtype=torch.int64, device=dev)
    jobs = [(scn, 3, empty, torch.zeros(0, dtype=torch.int64, device=dev), rich[0:1]),
            (scn, 3, s, outs[0], rich[1:2]),
            (scn, 3, empty, torch.zeros(0, dtype=torch.int64, device=dev), rich[2:3]),
            (scn, 3, s, outs[1], rich[3:4])]
    ws = torch.empty(B.workspace_bytes(2 * n, 4), dtype=torch.uint8, device=dev)
    B.batch_run(jobs, ws)
    torch.cuda.synchronize()
    alone, r, _ = B.simulate(scn, 3, wl.samples)
    assert np.array_equal(outs[0].cpu().numpy().view(np.uint64), alone)
    assert np.array_equal(outs[1].cpu().numpy().view(np.uint64), alone)
    assert rich.cpu().tolist() == [0, r, 0, r]
    # nh_simulate_device: the library allocates its own workspace on the stream
    out = torch.empty(n, dtype=torch.int64, device=dev)
    r1 = torch.zeros(1, dtype=torch.int64, device=dev)
    st = B.nh_stats()
    rc = B.nh_simulate_device(scn.handle, 3, C.c_void_p(s.data_ptr()), n, C.c_void_p(out.data_ptr()),
                              C.c_void_p(r1.data_ptr()), None, C.byref(st),
                              C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint64), alone) and int(r1.item()) == r


def test_measurement_helpers_report_plausible_rates(B, torch_mod):
    """The mix-peak and gather-ceiling microbenchmarks run and give rates within physical bounds."""
    torch = torch_mod
    mix = B.measure_mix_peak()
    assert 1e12 < mix < 2e14, mix  # algorithmic lane-ops/s; the VALU issues 3.9e13 instructions/s
    table = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
    g = B.measure_gather(table)
    assert 1e9 < g < 8e12, g
    # a lone lineage's event: two Philox blocks, a logarithm and the dispersal in sequence, each
    # hundreds of clocks at 2.4 GHz; neither the LDS-staged nor the global-table form leaves that range
    for scn in (B.Scenario.from_workload(W.config2()), B.Scenario.from_workload(SMALL[4])):
        ns = B.measure_event_latency(scn, 1, 4000)
        assert 100.0 < ns < 20000.0, ns


def test_concurrent_threads_on_their_own_streams(B, torch_mod):
    """Two host threads, each with its own stream and workspace, run batches at the same time
    (ctypes releases the interpreter lock during the library call); every result equals the
    sequential run's."""
    import threading
    torch = torch_mod
    dev = torch.device("cuda:0")
    wls = [W.config2(), SMALL[4]]
    scns = [B.Scenario.from_workload(w) for w in wls]
    samples = [w.samples if w.samples is not None else np.arange(w.individuals, dtype=np.uint64) for w in wls]
    ref = [[B.simulate(scns[k], 100 + r, samples[k])[0] for r in range(3)] for k in range(2)]
    got = [[None] * 3 for _ in range(2)]
    errors = []

    def worker(k):
        try:
            st = torch.cuda.Stream(device=dev)
            n = len(samples[k])
            with torch.cuda.stream(st):
                s = torch.from_numpy(samples[k].astype(np.int64)).to(dev)
                ws = torch.empty(B.workspace_bytes(n, 1), dtype=torch.uint8, device=dev)
                for r in range(3):
                    out = torch.empty(n, dtype=torch.int64, device=dev)
                    B.batch_run([(scns[k], 100 + r, s, out, None)], ws, None, st)
                    st.synchronize()
                    got[k][r] = out.cpu().numpy().view(np.uint64)
        except Exception as e:  # reported below
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=90)
    assert not any(t.is_alive() for t in threads), "a worker did not finish"
    assert not errors, errors
    for k in range(2):
        for r in range(3):
            assert np.array_equal(got[k][r], ref[k][r]), (k, r)
