"""The allocation-free entry point (nh_simulate_noalloc) against the existing
device-buffer entry point (nh_simulate_device): bit-identical species and
richness on two calls in a row, the second smaller, through the C ABI; the
device's free memory does not move; a run too large for the scratch is
refused before any device work."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2108_05815_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-noalloc]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2108_05815_amd import binding
    return binding


def _device_call(B, torch, scn, seed, s, out, rich):
    """nh_simulate_device through the C ABI (blocking)."""
    st = B.nh_stats()
    rc = B.nh_simulate_device(scn.handle, seed, s.data_ptr(), s.numel(), out.data_ptr(), rich.data_ptr(), None,
                              C.byref(st), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == B.NH_OK, B.nh_last_error().decode()


def _noalloc_call(B, torch, scn, seed, s, out, rich):
    rc = B.nh_simulate_noalloc(scn.handle, seed, s.data_ptr(), s.numel(), out.data_ptr(), rich.data_ptr(), None,
                               C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == B.NH_OK, B.nh_last_error().decode()


def test_noalloc_equals_the_device_entry_point_twice_second_smaller(B):
    import torch
    dev = torch.device("cuda:0")
    big = W.config2()                                                 # 65,536 samples, shared table
    small = W.Workload("fractal 61 per-deme", W.fractal_capacity(61, 12, base_period=16),
                       W.gaussian_kernel(3.0, 8), 0.003, 1, None, [11])  # per-deme tables, fewer samples
    cases = []
    for wl, seed in ((big, 42), (small, 11)):
        scn = B.Scenario.from_workload(wl)
        samples = wl.samples if wl.samples is not None else np.arange(scn.individuals, dtype=np.uint64)
        s = torch.from_numpy(samples.astype(np.int64)).to(dev)
        cases.append((wl.name, scn, seed, s))
    assert cases[1][3].numel() < cases[0][3].numel()
    refs = []
    for name, scn, seed, s in cases:
        out = torch.empty(s.numel(), dtype=torch.int64, device=dev)
        rich = torch.zeros(1, dtype=torch.int64, device=dev)
        _device_call(B, torch, scn, seed, s, out, rich)
        refs.append((out.cpu().numpy(), int(rich.item())))
    outs = [torch.full((s.numel(),), -7, dtype=torch.int64, device=dev) for _, _, _, s in cases]
    richs = [torch.full((1,), -7, dtype=torch.int64, device=dev) for _ in cases]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for (name, scn, seed, s), out, rich in zip(cases, outs, richs):
        say(name, "n =", s.numel())
        _noalloc_call(B, torch, scn, seed, s, out, rich)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    for (name, _, _, _), out, rich, (ref, ref_rich) in zip(cases, outs, richs, refs):
        assert np.array_equal(out.cpu().numpy(), ref), name
        assert int(rich.item()) == ref_rich, name
    assert free1 == free0, f"device free memory moved by {free0 - free1} bytes"


def test_noalloc_refuses_a_run_beyond_its_scratch(B):
    import torch
    dev = torch.device("cuda:0")
    scn = B.Scenario.from_workload(W.nonspatial(1000, 0.1, [1]))
    n = 1
    while B.workspace_bytes(n, 1) <= 64 << 20:
        n *= 2
    s = torch.zeros(1, dtype=torch.int64, device=dev)  # never read: the size check comes first
    out = torch.zeros(1, dtype=torch.int64, device=dev)
    rc = B.nh_simulate_noalloc(scn.handle, 1, s.data_ptr(), n, out.data_ptr(), None, None,
                               C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == B.NH_EINVAL
    assert "scratch" in B.nh_last_error().decode()
