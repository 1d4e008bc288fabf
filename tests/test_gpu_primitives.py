"""Device-level unit tests of the path's building blocks (nh_eval_primitives):
Philox4x32-10 against its published known-answer vectors and the oracle, the
logarithm of the event-time search on millions of draws, the one-lane and 8-lane
next-event searches, event outcomes and one group step, all bit for bit against the
oracle on random inputs, with the table in LDS and in global memory."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2108_05815_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print("[gpu-primitives]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2108_05815_amd import binding
    return binding


@pytest.fixture(scope="module")
def torus(B):
    wl = W.config2()
    return wl, B.Scenario.from_workload(wl)


def _kat():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers_and_random_counters(B, torus):
    _, scn = torus
    for ctr, key, expected in _kat():
        seed = key[0] | (key[1] << 32)
        got = B.eval_primitives(scn, seed, ctr=np.array([ctr], np.uint32))["philox"][0]
        assert [int(x) for x in got] == expected
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 2**32, size=(1 << 20, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0x9E3779B97F4A7C15
    got = B.eval_primitives(scn, seed, ctr=ctr)["philox"]
    ref = oracle.philox_array(ctr, np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint32))
    assert np.array_equal(got, ref)


def test_logarithm_of_draws_is_bitwise_the_oracles(B, torus):
    _, scn = torus
    rng = np.random.default_rng(4)
    r = rng.integers(0, 2**64, size=1 << 23, dtype=np.uint64)
    # the ends and the binade edges of u = ((r >> 11) + 1) 2^-53, and both sides of sqrt(1/2)
    q = np.array([0, 1, 2, 3, (1 << 52) - 1, 1 << 52, (1 << 53) - 1, 0x16A09E667F3BCC, 0x16A09E667F3BCD,
                  0x16A09E667F3BCE] + [(1 << k) - 1 for k in range(1, 54)] + [1 << k for k in range(0, 53)],
                 dtype=np.uint64)
    r = np.concatenate([r, q << np.uint64(11), (q << np.uint64(11)) | np.uint64(0x7FF)])
    say("log draws", len(r))
    got = B.eval_primitives(scn, 1, r=r)["log"]
    assert np.array_equal(got.view(np.uint64), oracle.log_u53o_array(r).view(np.uint64))


def _scenarios(B):
    c2 = W.config2()
    habitat = W.Workload("fractal 61 per-deme", W.fractal_capacity(61, 12, base_period=16), W.gaussian_kernel(3.0, 8),
                         0.003, 1, None, [2])
    out = []
    for wl, lam, dt, sampler, tau in [(c2, 1.0, 1.0, 0, 0.0), (c2, 4.0, 0.5, 0, 0.0), (c2, 1.0, 1.0 / 64, 0, 0.0),
                                      (c2, 1.0, 16.0, 0, 0.0), (c2, 1.0, 1.0, 1, 0.0), (habitat, 1.0, 1.0, 0, 0.0),
                                      (habitat, 0.3, 2.0, 1, 5.0)]:
        kw = dict(mode=wl.mode, lam=lam, dt=dt, sampler=sampler, tau=tau)
        name = f"{wl.name} lambda={lam} dt={dt} sampler={sampler} tau={tau}"
        out.append((name, oracle.Scenario(wl.capacity, wl.weights, wl.nu, **kw),
                    B.Scenario(wl.capacity, wl.weights, wl.nu, **kw)))
    out.append(("implicit", oracle.Scenario.implicit(300, 3000, 0.05, 0.005), B.Scenario.implicit(300, 3000, 0.05,
                                                                                                  0.005)))
    return out


@pytest.mark.parametrize("use_lds", [True, False])
def test_event_primitives_are_bitwise_the_oracles(B, use_lds):
    rng = np.random.default_rng(5)
    for name, osc, scn in _scenarios(B):
        seed = int(rng.integers(0, 2**63))
        n = 1 << 16
        ids = rng.integers(0, osc.individuals, size=n, dtype=np.uint64)
        loc = np.array([osc.sample_location(int(i)) for i in ids], dtype=np.uint32)
        t = rng.uniform(0.0, 2000.0, size=n)
        t[:64] = np.floor(t[:64])  # interval boundaries
        t[64:128] = 0.0
        say(name, "lds" if use_lds else "global", n)
        got = B.eval_primitives(scn, seed, loc=loc, t=t, use_lds=use_lds)
        nxt = osc.next_event_time_array(seed, loc, t)
        assert np.array_equal(got["next"], nxt), name
        assert np.array_equal(got["next_group"], nxt), name
        out = osc.event_outcome_array(seed, loc, t)
        assert np.array_equal(got["outcome"], out), name
        spec = out == oracle.EVENT_SPECIATION
        assert np.array_equal(got["step_loc"], out), name
        step_t = np.where(spec, t, osc.next_event_time_array(seed, np.where(spec, loc, out), t))
        assert np.array_equal(got["step_t"], step_t), name


def test_invalid_items_touch_no_table(B, torus):
    wl, scn = torus
    loc = np.array([0, 65535, 65536, 0xFFFFFFFF, 5], np.uint32)
    t = np.array([1.0, 2.0, 3.0, 4.0, -1.0])
    got = B.eval_primitives(scn, 1, loc=loc, t=t)
    assert np.isfinite(got["next"][:2]).all() and np.isnan(got["next"][2:]).all()
    assert (got["outcome"][2:] == 0xFFFFFFFF).all()
