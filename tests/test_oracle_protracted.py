"""Pins for the oracle's protracted speciation (appendix "Protracted Speciation"): a
speciation counts only once tau generations have passed since it, so going back from
the present the speciation draws of the first tau generations (lambda t < tau) are
ignored and those events are ordinary dispersals.  Exact: a two-phase reverse-time
chain on tiny landscapes (pure dispersal and coalescence for tau generations, then the
point-speciation chain), itself checked against a lineage-count form for a single deme
and against Ewens' closed form at tau = 0."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import exact_chain as E
import oracle


def _count_chain(J: int, nu: float, tau: float) -> float:
    """Single deme of J, all J sampled: during the first tau generations k lineages coalesce at
    rate k (k - 1) / J (each moves once per generation and picks one of the other k - 1 slots
    with probability (k - 1) / J); afterwards, from k lineages, E[S] = sum_{i=1..k} nu / (nu +
    (1 - nu) (i - 1) / J) (the i-th lineage from the bottom is removed by speciation before
    coalescing with that probability)."""
    Q = np.zeros((J + 1, J + 1))
    for k in range(2, J + 1):
        Q[k, k - 1] = k * (k - 1) / J
        Q[k, k] = -Q[k, k - 1]
    p = expm(Q * tau)[J]
    s = np.cumsum([0.0] + [nu / (nu + (1.0 - nu) * (i - 1) / J) for i in range(1, J + 1)])
    return float((p * s).sum())


def _mean_richness(sc, samples, seeds: int):
    r = np.array([oracle.richness(sc.simulate_naive(seed, samples)[0]) for seed in range(seeds)], np.float64)
    return r.mean(), r.std(ddof=1) / math.sqrt(seeds)


@pytest.mark.parametrize("J,nu,tau", [(6, 0.3, 1.5), (5, 0.2, 3.0), (4, 0.45, 0.4)])
def test_the_exact_chain_matches_the_lineage_count_form(J, nu, tau):
    D = E.dispersal_law(np.array([[J]], np.uint32), np.ones((1, 1)), 0)
    got = E.protracted_expected_richness_law(D, np.full(J, nu), tau, range(J))
    assert got == pytest.approx(_count_chain(J, nu, tau), rel=1e-10)
    assert E.protracted_expected_richness_law(D, np.full(J, nu), 0.0, range(J)) == pytest.approx(
        E.ewens_mean(J, nu), rel=1e-12)


@pytest.mark.parametrize("J,nu,tau,lam,dt", [(6, 0.3, 1.5, 1.0, 1.0), (5, 0.2, 3.0, 2.0, 1.0),
                                             (4, 0.45, 0.4, 0.5, 2.0)])
def test_single_deme_matches_the_exact_chain(J, nu, tau, lam, dt):
    # tau counts generations (1 / lambda time units each), so lambda changes nothing here
    exact = _count_chain(J, nu, tau)
    sc = oracle.Scenario(np.array([[J]], np.uint32), np.ones((1, 1)), nu, lam=lam, dt=dt, tau=tau)
    mean, se = _mean_richness(sc, np.arange(J, dtype=np.uint64), 12000)
    assert abs(mean - exact) < 4.5 * se, (mean, exact, se)


def test_ignored_speciations_disperse():
    # The reading that an ignored speciation leaves the lineage in place makes the coalescence
    # phase effectively tau (1 - nu) generations long; that value lies far outside the tolerance.
    J, nu, tau = 6, 0.3, 1.5
    exact, wrong = _count_chain(J, nu, tau), _count_chain(J, nu, tau * (1.0 - nu))
    sc = oracle.Scenario(np.array([[J]], np.uint32), np.ones((1, 1)), nu, tau=tau)
    mean, se = _mean_richness(sc, np.arange(J, dtype=np.uint64), 12000)
    assert abs(mean - exact) < 4.5 * se and abs(mean - wrong) > 10 * se, (mean, exact, wrong, se)


@pytest.mark.parametrize("cap,mode,nu,tau,sampler", [
    ([[1, 1, 1], [1, 1, 1], [1, 1, 1]], 0, 0.25, 0.8, 0),
    ([[2, 1, 0], [1, 0, 1], [0, 1, 0]], 1, 0.3, 1.2, 0),
    ([[1, 1, 1], [1, 1, 1], [1, 1, 1]], 0, 0.25, 0.8, 1),
])
def test_tiny_torus_matches_the_exact_chain(cap, mode, nu, tau, sampler):
    capacity = np.array(cap, np.uint32)
    weights = np.array([[0.5, 1.0, 0.5], [1.0, 2.0, 1.0], [0.5, 1.0, 0.5]])
    D = E.dispersal_law(capacity, weights, mode)
    n = D.shape[0]
    exact = E.protracted_expected_richness_law(D, np.full(n, nu), tau, range(n))
    sc = oracle.Scenario(capacity, weights, nu, mode=mode, sampler=sampler, tau=tau)
    mean, se = _mean_richness(sc, np.arange(n, dtype=np.uint64), 12000)
    assert abs(mean - exact) < 4.5 * se, (mean, exact, se)


def test_spatially_implicit_matches_the_exact_chain():
    J, Jm, m, nu, tau = 3, 3, 0.4, 0.3, 1.0
    D, start = E.implicit_law(J, Jm, m)
    exact = E.protracted_expected_richness_law(D, np.array([0.0] * J + [nu] * Jm), tau, start)
    sc = oracle.Scenario.implicit(J, Jm, m, nu, tau=tau)
    mean, se = _mean_richness(sc, np.arange(J, dtype=np.uint64), 12000)
    assert abs(mean - exact) < 4.5 * se, (mean, exact, se)


def test_speciations_are_at_least_tau_generations_old_and_zero_tau_is_point_speciation():
    cap = np.ones((12, 12), np.uint32)
    w = np.array([[1.0, 2.0, 1.0], [2.0, 4.0, 2.0], [1.0, 2.0, 1.0]])
    s = np.arange(144, dtype=np.uint64)
    for lam, tau in [(1.0, 5.0), (4.0, 5.0), (0.25, 0.75)]:
        sp, ts, _ = oracle.Scenario(cap, w, 0.05, lam=lam, tau=tau).simulate_naive(3, s)
        assert (lam * ts >= tau).all()
        sp0, ts0, _ = oracle.Scenario(cap, w, 0.05, lam=lam).simulate_naive(3, s)
        young = lam * ts0 < tau
        assert young.any()
        # a sample whose point speciation is old enough has the same history up to it
        assert (sp[~young] == sp0[~young]).all() and (ts[~young] == ts0[~young]).all()
    a = oracle.Scenario(cap, w, 0.05, tau=0.0).simulate_naive(3, s)
    b = oracle.Scenario(cap, w, 0.05).simulate_naive(3, s)
    assert all((x == y).all() for x, y in zip(a, b))


def test_culled_equals_naive_with_tau():
    cap = np.ones((16, 16), np.uint32)
    w = np.array([[1.0, 2.0, 1.0], [2.0, 4.0, 2.0], [1.0, 2.0, 1.0]])
    s = np.arange(256, dtype=np.uint64)
    for sampler in (0, 1):
        sc = oracle.Scenario(cap, w, 0.02, tau=7.5, sampler=sampler)
        for seed in (1, 2):
            assert (sc.simulate_culled(seed, s, 4.0)[0] == sc.simulate_naive(seed, s)[0]).all()


@pytest.mark.parametrize("tau", [-1.0, float("nan"), float("inf")])
def test_invalid_tau_is_rejected(tau):
    with pytest.raises(ValueError):
        oracle.Scenario(np.ones((2, 2), np.uint32), np.ones((1, 1)), 0.1, tau=tau)
