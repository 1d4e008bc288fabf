"""GPU event stream (sections "Sorting Events using the Water-Level Algorithm" and
"Reporting Coalescence Events Independently"): nh_event_stream after a batch run must
equal the oracle's reduced stream (every sample traced alone, all events sorted, copies
of shared events reduced) record for record, bit for bit; at the 256x256 torus it is
checked on sampled records against the oracle's event definition and on properties that
hold at any size."""
import sys

import numpy as np
import pytest

import oracle
from paper_2108_05815_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-events]", *a, file=sys.stderr, flush=True)


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


W3 = np.array([[1.0, 2.0, 1.0], [2.0, 4.0, 2.0], [1.0, 2.0, 1.0]])

# (name, oracle scenario factory, binding scenario factory, samples, seed)
CASES = [
    ("nonspatial J=300", dict(capacity=np.array([[300]], np.uint32), weights=np.ones((1, 1)), nu=0.05),
     np.arange(300), 4),
    ("torus 24x24 cap2 R4", dict(capacity=np.full((24, 24), 2, np.uint32), weights=W.gaussian_kernel(1.5, 4),
                                 nu=0.02), np.arange(24 * 24 * 2), 5),
    ("torus 37x37 cap3 R9 subset", dict(capacity=np.full((37, 37), 3, np.uint32), weights=W.gaussian_kernel(2.5, 9),
                                        nu=0.004), np.arange(0, 37 * 37 * 3, 5), 6),
    ("fractal 24 per-deme", dict(capacity=W.fractal_capacity(24, 11, base_period=8), weights=W.gaussian_kernel(2.0, 5),
                                 nu=0.02, mode=1), None, 6),
    ("3x3 cap1 flat", dict(capacity=np.ones((3, 3), np.uint32), weights=np.ones((3, 3)), nu=0.1), np.arange(9), 0),
    ("no dispersal", dict(capacity=np.ones((16, 16), np.uint32), weights=np.ones((1, 1)), nu=0.05), np.arange(256), 7),
    ("nu = 1", dict(capacity=np.full((20, 20), 2, np.uint32), weights=W.gaussian_kernel(1.0, 2), nu=1.0),
     np.arange(800), 8),
    ("protracted tau 6 lambda 0.3", dict(capacity=np.full((16, 16), 2, np.uint32), weights=W3, nu=0.03, lam=0.3,
                                         tau=6.0), np.arange(512), 9),
    ("Poisson sampler lambda 4 dt 0.5", dict(capacity=np.full((20, 20), 1, np.uint32), weights=W3, nu=0.02, lam=4.0,
                                             dt=0.5, sampler=1), np.arange(400), 10),
    ("duplicate and unsorted samples", dict(capacity=np.ones((12, 12), np.uint32), weights=W3, nu=0.05),
     np.array([7, 3, 7, 143, 0, 3, 100, 99, 7]), 11),
]


def _scenarios(B, kw):
    kw = dict(kw)
    cap, w, nu = kw.pop("capacity"), kw.pop("weights"), kw.pop("nu")
    return oracle.Scenario(cap, w, nu, **kw), B.Scenario(cap, w, nu, **kw)


def _samples(osc, samples):
    if samples is None:
        return np.arange(osc.individuals, dtype=np.uint64)
    return np.asarray(samples, dtype=np.uint64)


def _assert_same_stream(got, ref_ev, ref_co, name=""):
    e, c = got["events"], got["coalescences"]
    assert got["n_events"] == len(ref_ev["t"]) and got["n_coalescences"] == len(ref_co["t"]), name
    assert np.array_equal(e["t"], ref_ev["t"]) and np.array_equal(e["t_prior"], ref_ev["prior"]), name
    assert np.array_equal(e["origin"], ref_ev["origin"]) and np.array_equal(e["outcome"], ref_ev["outcome"]), name
    assert np.array_equal(c["t"], ref_co["t"]) and np.array_equal(c["t_parent"], ref_co["parent"]), name
    assert np.array_equal(c["loc"], ref_co["loc"]), name


def _run(B, torch, jobs_spec, config=None):
    """jobs_spec: list of (binding scenario, seed, samples); returns (jobs, workspace, outs)."""
    dev = torch.device("cuda:0")
    jobs, outs = [], []
    for scn, seed, samples in jobs_spec:
        s = torch.from_numpy(samples.astype(np.int64)).to(dev)
        out = torch.empty(max(len(samples), 1), dtype=torch.int64, device=dev)[:len(samples)]
        jobs.append((scn, seed, s, out, None))
        outs.append(out)
    ws = torch.empty(B.workspace_bytes(sum(len(x[2]) for x in jobs_spec), len(jobs)), dtype=torch.uint8, device=dev)
    st = B.batch_run(jobs, ws, config)
    return jobs, ws, outs, st


@pytest.mark.parametrize("k", range(len(CASES)), ids=[c[0] for c in CASES])
def test_event_stream_equals_the_oracle(B, torch_mod, k):
    name, kw, samples, seed = CASES[k]
    osc, scn = _scenarios(B, kw)
    samples = _samples(osc, samples)
    say(name, "n =", len(samples))
    ref_ev, ref_co = osc.event_stream(seed, samples)
    for coop in (1 << 30, 1):
        jobs, ws, _, _ = _run(B, torch_mod, [(scn, seed, samples)], B.make_config(coop_max=coop))
        got = B.event_stream(jobs, ws)[0]
        _assert_same_stream(got, ref_ev, ref_co, f"{name} coop_max={coop}")


@pytest.mark.parametrize("endgame", [0, 64, 4096], ids=["no endgame", "endgame 64", "endgame 4096"])
def test_event_stream_of_a_mixed_batch_and_a_short_buffer(B, torch_mod, endgame):
    """Lineages finished by the endgame (walked on without merging) leave the same reduced stream."""
    picks = [0, 1, 7, 8, 9]
    spec, refs = [], []
    for j, k in enumerate(picks):
        name, kw, samples, seed = CASES[k]
        osc, scn = _scenarios(B, kw)
        samples = _samples(osc, samples)
        spec.append((scn, seed + 100 * j, samples))
        refs.append(osc.event_stream(seed + 100 * j, samples))
    say("mixed batch of", len(spec))
    jobs, ws, _, _ = _run(B, torch_mod, spec, B.make_config(solo_max=32, endgame=endgame))
    for got, (ref_ev, ref_co) in zip(B.event_stream(jobs, ws), refs):
        _assert_same_stream(got, ref_ev, ref_co)
    # room for half of each job's events: the first half is written and the counts are whole
    caps = [len(r[0]["t"]) // 2 for r in refs]
    for got, (ref_ev, ref_co), cap in zip(B.event_stream(jobs, ws, events_cap=caps), refs, caps):
        assert got["n_events"] == len(ref_ev["t"]) and len(got["events"]) == cap
        assert np.array_equal(got["events"]["t"], ref_ev["t"][:cap])
        assert np.array_equal(got["events"]["outcome"], ref_ev["outcome"][:cap])
        assert np.array_equal(got["coalescences"]["t"], ref_co["t"])


def test_event_stream_implicit_empty_job_and_reporters(B, torch_mod):
    """The spatially implicit scenario (with protracted speciation), an empty job between two others,
    and the speciation events of the stream against the per-sample speciation reporter."""
    torch = torch_mod
    dev = torch.device("cuda:0")
    J, Jm = 200, 2000
    oimp = oracle.Scenario.implicit(J, Jm, 0.05, 0.01, tau=2.0)
    gimp = B.Scenario.implicit(J, Jm, 0.05, 0.01, tau=2.0)
    name, kw, samples, seed = CASES[1]
    osc, scn = _scenarios(B, kw)
    samples = _samples(osc, samples)
    local = np.arange(J, dtype=np.uint64)
    spec = [(gimp, 3, local), (scn, seed, np.zeros(0, np.uint64)), (scn, seed, samples)]
    jobs, ws, outs, _ = _run(B, torch, spec)
    got = B.event_stream(jobs, ws)
    _assert_same_stream(got[0], *oimp.event_stream(3, local), "implicit")
    assert got[1]["n_events"] == 0 and got[1]["n_coalescences"] == 0
    _assert_same_stream(got[2], *osc.event_stream(seed, samples), "after the empty job")
    # the reporter's speciation event of every sample is one of the stream's speciation events
    n = len(samples)
    rep = dict(spec_loc=torch.zeros(n, dtype=torch.int32, device=dev),
               spec_time=torch.zeros(n, dtype=torch.float64, device=dev))
    s = torch.from_numpy(samples.astype(np.int64)).to(dev)
    out = torch.empty(n, dtype=torch.int64, device=dev)
    ws1 = torch.empty(B.workspace_bytes(n, 1), dtype=torch.uint8, device=dev)
    job = [(scn, seed, s, out, None, rep)]
    B.batch_run(job, ws1)
    ev = B.event_stream(job, ws1)[0]["events"]
    sp = ev["outcome"] == B.NH_EVENT_SPECIATION
    events = set(zip(ev["origin"][sp].tolist(), ev["t"][sp].tolist()))
    reported = set(zip(rep["spec_loc"].cpu().numpy().view(np.uint32).tolist(), rep["spec_time"].cpu().numpy().tolist()))
    assert reported == events


def test_event_stream_needs_the_finished_run_of_the_same_jobs(B, torch_mod):
    name, kw, samples, seed = CASES[1]
    osc, scn = _scenarios(B, kw)
    samples = _samples(osc, samples)
    jobs, ws, _, st = _run(B, torch_mod, [(scn, seed, samples)], B.make_config(max_rounds=3))
    assert st[0]["suspended"]
    with pytest.raises(B.NecsimError) as e:
        B.event_stream(jobs, ws)
    assert e.value.code == B.NH_EINVAL
    B.batch_resume(jobs, ws)
    ref_ev, ref_co = osc.event_stream(seed, samples)
    _assert_same_stream(B.event_stream(jobs, ws)[0], ref_ev, ref_co, "resumed")
    other = [(scn, seed + 1) + tuple(jobs[0][2:])]
    with pytest.raises(B.NecsimError) as e:
        B.event_stream(other, ws)
    assert e.value.code == B.NH_EINVAL


def test_event_stream_of_the_256_torus(B, torch_mod):
    """The 256x256 torus (all 65,536 individuals, sigma 2, R 10, nu 1e-3): conservation, the
    species, the order, and sampled events and coalescences against the oracle's definitions."""
    wl = W.config2()
    osc = oracle.Scenario(wl.capacity, wl.weights, wl.nu)
    scn = B.Scenario.from_workload(wl)
    seed = 42
    say("256x256 torus")
    jobs, ws, outs, st = _run(B, torch_mod, [(scn, seed, wl.samples)])
    got = B.event_stream(jobs, ws)[0]
    ev, co = got["events"], got["coalescences"]
    species = outs[0].cpu().numpy().view(np.uint64)
    spec = ev["outcome"] == B.NH_EVENT_SPECIATION
    assert len(wl.samples) == spec.sum() + len(co)
    assert spec.sum() == len(np.unique(species)) == st[0]["richness"]
    assert got["n_events"] <= st[0]["events"]
    ids = {oracle.species_id(seed, int(l), float(t)) for l, t in zip(ev["origin"][spec], ev["t"][spec])}
    assert ids == set(int(x) for x in species)
    order = np.lexsort((ev["origin"], ev["t"]))
    assert np.array_equal(order, np.arange(len(ev)))
    assert not np.any((np.diff(ev["t"]) == 0) & (np.diff(ev["origin"].astype(np.int64)) == 0))
    corder = np.lexsort((co["t_parent"], co["loc"], co["t"]))
    assert np.array_equal(corder, np.arange(len(co)))
    rng = np.random.default_rng(5)
    for i in rng.choice(len(ev), 400, replace=False):
        t, prior, origin, outcome = float(ev["t"][i]), float(ev["t_prior"][i]), int(ev["origin"][i]), int(
            ev["outcome"][i])
        assert osc.next_event_time(seed, origin, prior) == t
        assert osc.event_outcome(seed, origin, t) == outcome
    arrivals = set(zip(ev["t"][~spec].tolist(), ev["outcome"][~spec].tolist()))
    for i in rng.choice(len(co), 400, replace=False):
        t, parent, loc = float(co["t"][i]), float(co["t_parent"][i]), int(co["loc"][i])
        assert 0.0 <= parent < t and (t, loc) in arrivals
        assert parent == 0.0 or (parent, loc) in arrivals


@pytest.mark.parametrize("knobs", [dict(), dict(horizon0=2.0, horizon_growth=2.0),
                                   dict(horizon0=0.25, horizon_growth=1.5, horizon_step_max=16.0),
                                   dict(launch=1), dict(launch=1, horizon0=0.25, horizon_growth=1.5,
                                                        horizon_step_max=16.0)],
                         ids=["default", "2x2", "capped", "graphs", "graphs-capped"])
def test_one_round_per_horizon_window(B, torch_mod, knobs):
    """A single-job run takes one round per horizon window up to the window of its last event,
    with the horizons bench.py derives from the config, so the per-window maxima it reports
    describe the run's own rounds."""
    import bench
    name, kw, samples, seed = CASES[2]
    osc, scn = _scenarios(B, kw)
    samples = _samples(osc, samples)
    cfg = B.make_config(**knobs)
    jobs, ws, _, st = _run(B, torch_mod, [(scn, seed, samples)], cfg)
    got = B.event_stream(jobs, ws)[0]
    ev, co = got["events"], got["coalescences"]
    m = bench.window_maxima(ev, co, bench.horizon_table(cfg, float(ev["t"].max())))
    say(name, knobs, "rounds", st[0]["rounds"], "windows", len(m))
    assert len(m) == st[0]["rounds"]
    assert m[-1] > 0 and sum(m) >= bench.chain_events(ev, co)
