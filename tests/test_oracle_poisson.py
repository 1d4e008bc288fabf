"""Pins for the oracle's second event-time sampler (section "Homogeneous Poisson
Point Process" of the Independent Algorithm chapter): per repriming interval a
Poisson(lambda dt) count of events placed uniformly in the interval.  It draws
different bits from the exponential sums, so it is pinned on its own: the
fixed-point-set alignment property, Exp(lambda) gaps across intervals, Poisson
counts, uniform positions, the Ewens mean, the exact chain on a tiny landscape,
and culled == naive."""
import math

import numpy as np
import pytest
from scipy import special, stats

import exact_chain as E
import oracle
from paper_2108_05815_amd import workloads as W


def _torus(lam=1.0, dt=1.0, nu=0.01):
    return oracle.Scenario(np.ones((8, 8), np.uint32), W.gaussian_kernel(1.0, 1), nu, lam=lam, dt=dt, sampler=1)


def test_rejects_unknown_sampler_and_huge_interval_rate():
    with pytest.raises(ValueError):
        oracle.Scenario(np.ones((4, 4), np.uint32), np.ones((3, 3)), 0.1, sampler=2)
    with pytest.raises(ValueError):
        oracle.Scenario(np.ones((4, 4), np.uint32), np.ones((3, 3)), 0.1, lam=1024.0, dt=1.0, sampler=1)
    oracle.Scenario(np.ones((4, 4), np.uint32), np.ones((3, 3)), 0.1, lam=512.0, dt=1.0, sampler=1)


def test_next_event_is_the_next_point_of_a_fixed_point_set():
    """Aligning colliding individuals still holds: the events at one slot are one fixed set of
    points, and a lineage arriving anywhere between two of them finds the later one (bitwise)."""
    sc = _torus()
    rng = np.random.default_rng(7)
    for loc in (0, 9, 63):
        for seed in (3, 2**63 + 1):
            pts, t = [], 0.0
            while t < 40.0:
                t = sc.next_event_time(seed, loc, t)
                pts.append(t)
            pts = np.array(pts)
            assert np.all(np.diff(pts) > 0)
            probes = list(rng.uniform(0, 38.0, size=200)) + [float(k) for k in range(38)] + list(pts[:-1])
            probes += [math.nextafter(p, 0) for p in pts[:-1]]
            for tq in probes:
                assert sc.next_event_time(seed, loc, tq) == pts[np.searchsorted(pts, tq, side="right")]


def _points(sc, seed, loc, t_end):
    pts, t = [], 0.0
    while True:
        t = sc.next_event_time(seed, loc, t)
        if t >= t_end:
            return np.array(pts)
        pts.append(t)


@pytest.mark.parametrize("lam,dt", [(1.0, 1.0), (4.0, 0.5), (0.5, 2.0), (3.0, 1.0), (16.0, 4.0)])
def test_gaps_are_exponential_counts_poisson_positions_uniform(lam, dt):
    """Gaps between consecutive events are Exp(lambda) across interval boundaries (KS); counts per
    interval are Poisson(lambda dt) (chi-square); positions inside an interval are uniform (KS)."""
    sc = _torus(lam=lam, dt=dt)
    n_int = int(4000 / (lam * dt)) + 200
    gaps, counts, frac = [], [], []
    for loc in range(4):
        pts = _points(sc, 5, loc, n_int * dt)
        gaps.extend(np.diff(np.concatenate([[0.0], pts]))[1:])
        k = np.floor(pts / dt).astype(np.int64)
        counts.extend(np.bincount(k, minlength=n_int)[:n_int])
        frac.extend(pts / dt - k)
    assert stats.kstest(np.array(gaps) * lam, "expon").pvalue > 1e-3
    assert stats.kstest(np.array(frac), "uniform").pvalue > 1e-3
    counts = np.array(counts)
    mu = lam * dt
    top = int(mu + 6 * math.sqrt(mu) + 3)
    obs = np.bincount(np.minimum(counts, top), minlength=top + 1)
    pmf = stats.poisson.pmf(np.arange(top + 1), mu)
    pmf[top] = stats.poisson.sf(top - 1, mu)
    keep = pmf * len(counts) >= 5
    exp_ = pmf[keep] * len(counts)
    o = obs[keep]
    chi2 = float(((o - exp_) ** 2 / exp_).sum()) + 0.0
    p = stats.chi2.sf(chi2, max(1, keep.sum() - 1))
    assert p > 1e-4, (lam, dt, p)


def test_ewens_mean_richness_non_spatial():
    """J = 1000, nu = 0.1: mean richness over 500 seeds equals theta (psi(theta+J) - psi(theta))."""
    J, nu = 1000, 0.1
    sc = oracle.Scenario(np.array([[J]], np.uint32), np.ones((1, 1)), nu, sampler=1)
    s = np.arange(J, dtype=np.uint64)
    rich = np.array([oracle.richness(sc.simulate_naive(seed, s)[0]) for seed in range(500)], dtype=np.float64)
    th = J * nu / (1.0 - nu)
    expected = th * (special.digamma(th + J) - special.digamma(th))
    se = rich.std(ddof=1) / math.sqrt(len(rich))
    assert abs(rich.mean() - expected) < 4 * se, (rich.mean(), expected, se)


def test_tiny_landscape_matches_exact_chain():
    cap = np.array([[1, 2, 0], [0, 1, 3], [2, 0, 1]], np.uint32)
    w = W.gaussian_kernel(1.0, 1)
    sc = oracle.Scenario(cap, w, 0.2, mode=1, sampler=1)
    n = sc.individuals
    samples = np.arange(n, dtype=np.uint64)
    exact = E.expected_richness(cap, w, 1, 0.2, range(n))
    N = 8000
    r = np.array([oracle.richness(sc.simulate_naive(seed, samples)[0]) for seed in range(N)], dtype=np.float64)
    se = r.std(ddof=1) / math.sqrt(N)
    assert abs(r.mean() - exact) < 4.5 * se, (r.mean(), exact, se)


@pytest.mark.parametrize("dW", [0.5, 8.0])
def test_culled_equals_naive(dW):
    wl = W.spatial_torus(20, 2, 1.5, 3, 0.02, [4])
    sc = oracle.Scenario(wl.capacity, wl.weights, wl.nu, sampler=1)
    s = np.arange(sc.individuals, dtype=np.uint64)
    a, _, _ = sc.simulate_naive(4, s)
    b, _, _ = sc.simulate_culled(4, s, dW)
    assert np.array_equal(a, b)


def test_differs_from_the_exponential_sampler():
    """Same scenario and seed, other sampler: other event times (the flag changes the bits)."""
    wl = W.spatial_torus(16, 1, 1.0, 2, 0.05, [2])
    a = oracle.Scenario(wl.capacity, wl.weights, wl.nu)
    b = oracle.Scenario(wl.capacity, wl.weights, wl.nu, sampler=1)
    assert a.next_event_time(2, 5, 0.0) != b.next_event_time(2, 5, 0.0)
