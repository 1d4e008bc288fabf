"""Enqueue-only runs (nh_simulate_async, one persistent launch per run): the call
returns while the run is still on the device; runs enqueued back to back on one
stream and synchronised once are bit-exact to the oracle; device-side failures
come back through the richness; and the persistent launch that the blocking
entry points use by default gives the same bits as the graph-replayed rounds."""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2108_05815_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-async]", *a, file=sys.stderr, flush=True)


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


def _dev_samples(torch, samples):
    return torch.from_numpy(np.ascontiguousarray(samples).astype(np.int64)).to(torch.device("cuda:0"))


def test_two_runs_enqueued_then_one_sync_bitexact(B, torch_mod):
    torch = torch_mod
    dev = torch.device("cuda:0")
    wl2 = W.config2()
    wl_small = W.Workload("fractal 61 per-deme", W.fractal_capacity(61, 12, base_period=16),
                          W.gaussian_kernel(3.0, 8), 0.003, 1, None, [5])
    osc2 = oracle.Scenario(wl2.capacity, wl2.weights, wl2.nu)
    oscs = oracle.Scenario(wl_small.capacity, wl_small.weights, wl_small.nu, mode=wl_small.mode)
    samples_small = np.arange(oscs.individuals, dtype=np.uint64)
    scn2, scns = B.Scenario.from_workload(wl2), B.Scenario.from_workload(wl_small)
    s2, ss = _dev_samples(torch, wl2.samples), _dev_samples(torch, samples_small)
    out2 = torch.empty(len(wl2.samples), dtype=torch.int64, device=dev)
    outs = torch.empty(len(samples_small), dtype=torch.int64, device=dev)
    rich = torch.zeros(2, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    say("enqueue: config 2 seed 42, then a 61x61 per-deme habitat; one synchronize")
    B.simulate_async(scn2, 42, s2, out2, rich[0:1])
    B.simulate_async(scns, 5, ss, outs, rich[1:2])
    torch.cuda.synchronize()
    ref2, _, _ = osc2.simulate_culled(42, wl2.samples, 1.0)
    refs, _, _ = oscs.simulate_culled(5, samples_small, 2.0)
    assert np.array_equal(out2.cpu().numpy().view(np.uint64), ref2)
    assert np.array_equal(outs.cpu().numpy().view(np.uint64), refs)
    r = rich.cpu().numpy()
    assert r[0] == oracle.richness(ref2) and r[1] == oracle.richness(refs)


def test_the_call_returns_before_the_run_finishes(B, torch_mod):
    torch = torch_mod
    dev = torch.device("cuda:0")
    wl = W.config2()
    scn = B.Scenario.from_workload(wl)
    s = _dev_samples(torch, wl.samples)
    out = torch.empty(len(wl.samples), dtype=torch.int64, device=dev)
    rich = torch.zeros(1, dtype=torch.int64, device=dev)
    B.simulate_async(scn, 43, s, out, rich)  # first call: the library's per-device set-up
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    B.simulate_async(scn, 44, s, out, rich)
    B.simulate_async(scn, 45, s, out, rich)
    t_call = time.perf_counter() - t0
    pending = not stream.query()
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    say(f"two enqueue calls took {t_call * 1e3:.3f} ms; the runs finished after {t_all * 1e3:.3f} ms")
    assert pending, "the device had already finished when the calls returned"
    assert t_call < t_all
    ref, _, _ = B.simulate(scn, 45, wl.samples)
    assert np.array_equal(out.cpu().numpy().view(np.uint64), ref)


def test_device_side_failures_read_as_richness_all_ones(B, torch_mod):
    torch = torch_mod
    dev = torch.device("cuda:0")
    wl = W.spatial_torus(24, 2, 1.5, 4, 0.02, [5], name="torus 24x24 cap2 R4")
    scn = B.Scenario.from_workload(wl)
    out = torch.empty(3, dtype=torch.int64, device=dev)
    rich = torch.zeros(1, dtype=torch.int64, device=dev)
    bad = torch.tensor([0, 5, scn.individuals], dtype=torch.int64, device=dev)
    say("a sample id >= N")
    B.simulate_async(scn, 1, bad, out, rich)
    torch.cuda.synchronize()
    assert int(rich.item()) == -1
    wl2 = W.config2()
    scn2 = B.Scenario.from_workload(wl2)
    s2 = _dev_samples(torch, wl2.samples)
    out2 = torch.empty(len(wl2.samples), dtype=torch.int64, device=dev)
    rich.zero_()
    say("a run stopped by its time limit (forced from the host: the kernel exits after its first round)")
    B.simulate_async(scn2, 9, s2, out2, rich, config=B.make_config(timeout_s=1e-9))
    torch.cuda.synchronize()
    assert int(rich.item()) == -1
    # the library and the device are fine afterwards
    B.simulate_async(scn2, 9, s2, out2, rich)
    torch.cuda.synchronize()
    ref, r, _ = B.simulate(scn2, 9, wl2.samples)
    assert np.array_equal(out2.cpu().numpy().view(np.uint64), ref) and int(rich.item()) == r


def test_empty_run_and_rejected_calls(B, torch_mod):
    torch = torch_mod
    dev = torch.device("cuda:0")
    scn = B.Scenario.from_workload(W.nonspatial(300, 0.05, [4]))
    e = torch.empty(0, dtype=torch.int64, device=dev)
    rich = torch.full((1,), 7, dtype=torch.int64, device=dev)
    B.simulate_async(scn, 1, e, e, rich)
    torch.cuda.synchronize()
    assert int(rich.item()) == 0
    s = torch.arange(10, dtype=torch.int64, device=dev)
    out = torch.empty(10, dtype=torch.int64, device=dev)
    for cfg in (dict(max_rounds=3), dict(launch=B.NH_LAUNCH_GRAPHS), dict(block_size=320)):
        with pytest.raises(B.NecsimError) as err:
            B.simulate_async(scn, 1, s, out, rich, config=B.make_config(**cfg))
        assert err.value.code == B.NH_EINVAL


@pytest.mark.parametrize("wl", [W.config2(), W.Workload("fractal 61 per-deme", W.fractal_capacity(61, 12, base_period=16),
                                                         W.gaussian_kernel(3.0, 8), 0.003, 1, None, [2**64 - 1])],
                         ids=["config2", "fractal61"])
def test_persistent_and_graph_launches_agree(B, torch_mod, wl):
    """The same run as one persistent launch and as graph-replayed round launches: same species,
    richness, events and rounds."""
    torch = torch_mod
    dev = torch.device("cuda:0")
    scn = B.Scenario.from_workload(wl)
    samples = wl.samples if wl.samples is not None else np.arange(scn.individuals, dtype=np.uint64)
    s = _dev_samples(torch, samples)
    ws = torch.empty(B.workspace_bytes(len(samples), 1), dtype=torch.uint8, device=dev)
    res = []
    for launch in (B.NH_LAUNCH_PERSISTENT, B.NH_LAUNCH_GRAPHS):
        out = torch.empty(len(samples), dtype=torch.int64, device=dev)
        rich = torch.zeros(1, dtype=torch.int64, device=dev)
        st = B.batch_run([(scn, wl.seeds[0], s, out, rich)], ws, B.make_config(launch=launch))[0]
        say(wl.name, "launch", launch, "rounds", st["rounds"], "events", st["events"], f"{st['device_ms']:.2f} ms")
        res.append((out.cpu().numpy(), int(rich.item()), st))
    (a, ra, sa), (b, rb, sb) = res
    assert np.array_equal(a, b) and ra == rb
    assert sa["rounds"] == sb["rounds"] and sa["events"] == sb["events"] and sa["merged"] == sb["merged"]
