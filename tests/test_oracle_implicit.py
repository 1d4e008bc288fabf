"""Pins for the oracle's spatially implicit scenario (background section "Spatially
Implicit"): a local community of J with migration probability m per event into a
non-spatial metacommunity of J_m (simulated alongside) that alone speciates, with
probability nu_m.  Exact: the reverse-time jump chain on tiny communities.
Closed form: Etienne's expected richness for an infinite static metacommunity,
which a large dynamic one approaches (as the paper's own comparison found)."""
import math

import numpy as np
import pytest
from scipy import special

import exact_chain as E
import oracle


@pytest.mark.parametrize("J,Jm,m,nu", [(3, 4, 0.3, 0.2), (2, 5, 0.6, 0.1), (4, 2, 0.15, 0.4), (3, 3, 1.0, 0.25)])
def test_tiny_communities_match_the_exact_chain(J, Jm, m, nu):
    D, start = E.implicit_law(J, Jm, m)
    nu_slot = np.array([0.0] * J + [nu] * Jm)
    exact = E.expected_richness_law(D, nu_slot, start)
    sc = oracle.Scenario.implicit(J, Jm, m, nu)
    s = np.arange(J, dtype=np.uint64)
    N = 12000
    r = np.array([oracle.richness(sc.simulate_naive(seed, s)[0]) for seed in range(N)], dtype=np.float64)
    se = r.std(ddof=1) / math.sqrt(N)
    assert abs(r.mean() - exact) < 4.5 * se, (r.mean(), exact, se)


def _etienne(J, m, theta):
    """E[S] = theta sum_j P(K = j) (psi(theta + j) - psi(theta)), K ~ Ewens(I) ancestors of J
    local individuals, P(K = j) = |s(J, j)| I^j / (I)_J, with I = J m / (1 - m) (a local parent
    may be the lineage's own slot, as in the non-spatial closed form)."""
    I = J * m / (1.0 - m)
    # P(K = j) by the recursion of unsigned Stirling numbers, in probability space
    p = np.zeros(J + 1)
    p[0] = 1.0
    for n in range(J):  # add the (n+1)-th individual: new ancestor w.p. I / (I + n)
        q = np.zeros(J + 1)
        q[1:] += p[:-1] * I / (I + n)
        q += p * n / (I + n)
        p = q
    j = np.arange(J + 1)
    return float(theta * (p * (special.digamma(theta + j) - special.digamma(theta))).sum())


def test_large_metacommunity_approaches_etienne():
    J, Jm, m, nu = 60, 200000, 0.05, 2.5e-4
    theta = Jm * nu / (1.0 - nu)
    expected = _etienne(J, m, theta)
    sc = oracle.Scenario.implicit(J, Jm, m, nu)
    s = np.arange(J, dtype=np.uint64)
    N = 300
    r = np.array([oracle.richness(sc.simulate_culled(seed, s, 64.0)[0]) for seed in range(N)], dtype=np.float64)
    se = r.std(ddof=1) / math.sqrt(N)
    assert abs(r.mean() - expected) < 4 * se, (r.mean(), expected, se)


def test_validation_and_no_local_speciation():
    with pytest.raises(ValueError):
        oracle.Scenario.implicit(10, 10, 0.0, 0.1)  # a local lineage could never speciate
    with pytest.raises(ValueError):
        oracle.Scenario.implicit(10, 10, 0.5, 0.0)
    # m = 1: every local lineage leaves at its first event, so no two local samples coalesce in
    # the local community; species ids come from metacommunity events only
    sc = oracle.Scenario.implicit(5, 3, 1.0, 0.3)
    for seed in range(20):
        t, locs, _, _, done = sc.trace(seed, 2)
        assert done and locs[-1] >= 5  # speciated in the metacommunity (cell 1: loc >= C_max = 5)


def test_culled_equals_naive():
    sc = oracle.Scenario.implicit(200, 500, 0.2, 0.01)
    s = np.arange(200, dtype=np.uint64)
    for dW in (0.5, 16.0):
        assert np.array_equal(sc.simulate_naive(7, s)[0], sc.simulate_culled(7, s, dW)[0])
