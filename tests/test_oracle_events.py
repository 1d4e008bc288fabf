"""Pins for the oracle's event stream (sections "Sorting Events using the Water-Level
Algorithm" and "Reporting Coalescence Events Independently"): every event of the
samples' lineages once, sorted, and the coalescences read off the copies of shared
events.  Checked against what the model fixes: lineage conservation (each coalescence
or speciation removes one lineage), the species set, the event-point definition of
every event, trace consistency, and, for a fully sampled deme, the jump times of the
lineage-count death process (closed-form means of every order statistic)."""
import math

import numpy as np
import pytest

import oracle

W3 = np.array([[1.0, 2.0, 1.0], [2.0, 4.0, 2.0], [1.0, 2.0, 1.0]])


def _scenarios():
    return [
        ("deme J=40", oracle.Scenario(np.array([[40]], np.uint32), np.ones((1, 1)), 0.05), np.arange(40)),
        ("torus 10x10 cap 2", oracle.Scenario(np.full((10, 10), 2, np.uint32), W3, 0.03), np.arange(0, 200, 3)),
        ("per-deme habitat", oracle.Scenario(np.array([[2, 0, 1, 3], [1, 1, 0, 2], [0, 2, 2, 1], [3, 1, 1, 0]],
                                                      np.uint32), W3, 0.04, mode=1), np.arange(20)),
        ("implicit", oracle.Scenario.implicit(30, 200, 0.1, 0.05), np.arange(30)),
        ("protracted + Poisson", oracle.Scenario(np.ones((12, 12), np.uint32), W3, 0.05, tau=4.0, sampler=1),
         np.arange(144)),
        ("duplicates", oracle.Scenario(np.ones((8, 8), np.uint32), W3, 0.05), np.array([5, 9, 5, 63, 9, 0])),
    ]


@pytest.mark.parametrize("k", range(6))
def test_stream_is_consistent_with_the_model(k):
    name, sc, samples = _scenarios()[k]
    samples = samples.astype(np.uint64)
    seed = 17 + k
    ev, co = sc.event_stream(seed, samples)
    sp, _, _ = sc.simulate_naive(seed, samples)
    distinct = len(np.unique(samples))
    spec = ev["outcome"] == oracle.EVENT_SPECIATION
    # conservation: every lineage ends in exactly one speciation or one coalescence
    assert distinct == spec.sum() + len(co["t"]), name
    # the speciation events are the species
    ids = {oracle.species_id(seed, int(l), float(t)) for l, t in zip(ev["origin"][spec], ev["t"][spec])}
    assert ids == set(int(x) for x in sp) and len(ids) == oracle.richness(sp)
    # sorted by (t, origin), each event once
    key = list(zip(ev["t"], ev["origin"]))
    assert all(a < b for a, b in zip(key, key[1:]))
    # each event is the next event point at its origin after its prior event time, with its outcome
    for t, prior, origin, outcome in zip(ev["t"], ev["prior"], ev["origin"], ev["outcome"]):
        assert sc.next_event_time(seed, int(origin), float(prior)) == t
        assert sc.event_outcome(seed, int(origin), float(t)) == outcome
    # coalescences: sorted; the child's arrival and the parent's arrival (or the present) exist
    ck = list(zip(co["t"], co["loc"], co["parent"]))
    assert all(a <= b for a, b in zip(ck, ck[1:]))
    arrivals = set(zip(ev["t"][~spec].tolist(), ev["outcome"][~spec].tolist()))
    starts = {sc.sample_location(int(s)) for s in samples}
    for t, parent, loc in zip(co["t"], co["parent"], co["loc"]):
        assert 0.0 <= parent < t
        assert (float(t), int(loc)) in arrivals
        assert (parent == 0.0 and int(loc) in starts) or (float(parent), int(loc)) in arrivals


def test_stream_contains_every_trace():
    sc = oracle.Scenario(np.full((10, 10), 2, np.uint32), W3, 0.03)
    samples = np.arange(0, 200, 7, dtype=np.uint64)
    ev, _ = sc.event_stream(4, samples)
    index = {(float(t), int(o)): (float(p), int(x)) for t, p, o, x in
             zip(ev["t"], ev["prior"], ev["origin"], ev["outcome"])}
    for s in samples:
        times, locs, _, _, done = sc.trace(4, int(s))
        assert done
        prior = 0.0
        for j, (t, l) in enumerate(zip(times, locs)):
            p, out = index[(float(t), int(l))]
            assert p <= prior  # the stream keeps the smallest prior of an event's copies
            assert out == (int(locs[j + 1]) if j + 1 < len(times) else oracle.EVENT_SPECIATION)
            prior = float(t)


@pytest.mark.parametrize("J,nu", [(8, 0.1), (5, 0.3)])
def test_lineage_count_jump_times(J, nu):
    """All J individuals of one deme sampled: the times at which the number of distinct lineages
    drops (coalescences and speciations together) are the jumps of a death process with rate
    k (nu + (1 - nu) (k - 1) / J) at k lineages (one event per lineage per generation; a parent is
    one of the other k - 1 lineages' slots with probability (k - 1) / J)."""
    sc = oracle.Scenario(np.array([[J]], np.uint32), np.ones((1, 1)), nu)
    samples = np.arange(J, dtype=np.uint64)
    rates = [k * (nu + (1.0 - nu) * (k - 1) / J) for k in range(J, 0, -1)]
    expected = np.cumsum([1.0 / r for r in rates])
    runs = 6000
    jumps = np.zeros((runs, J))
    for seed in range(runs):
        ev, co = sc.event_stream(seed, samples)
        spec_t = ev["t"][ev["outcome"] == oracle.EVENT_SPECIATION]
        jumps[seed] = np.sort(np.concatenate([co["t"], spec_t]))
    mean = jumps.mean(axis=0)
    se = jumps.std(axis=0, ddof=1) / math.sqrt(runs)
    assert (np.abs(mean - expected) < 5 * se).all(), (mean, expected, se)


def test_protracted_stream_has_no_young_speciation():
    sc = oracle.Scenario(np.ones((12, 12), np.uint32), W3, 0.05, lam=2.0, tau=6.0)
    ev, co = sc.event_stream(9, np.arange(144, dtype=np.uint64))
    spec = ev["outcome"] == oracle.EVENT_SPECIATION
    assert (2.0 * ev["t"][spec] >= 6.0).all()
    young = (2.0 * ev["t"] < 6.0) & ~spec
    assert young.any()
