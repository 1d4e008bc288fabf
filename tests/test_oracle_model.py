"""Model-level pins for the oracle: closed forms (Ewens / Vallade-Houchmandzadeh
non-spatial richness, its Poisson-binomial law, the Ewens sampling formula),
exact brute force on tiny landscapes, special cases, the event statistics the
paper tests (exponential inter-event and speciation times, uniform and normal
dispersal), stream correlation, and the invariants (culling, subsets,
permutations, duplicates) that make the GPU comparison meaningful."""
import math

import numpy as np
import pytest
from scipy import special, stats

import exact_chain as E
import oracle
from paper_2108_05815_amd import workloads as W


# --------------------------------------------------------------------------- #
# Non-spatial closed forms (appendix: analytical solutions, non-spatial)      #
# --------------------------------------------------------------------------- #

@pytest.fixture(scope="module")
def c1_richness():
    wl = W.config1(1000)
    sc = oracle.Scenario(wl.capacity, wl.weights, wl.nu)
    rich, singles = [], []
    for seed in wl.seeds:
        sp, _, _ = sc.simulate_naive(seed, wl.samples)
        rich.append(oracle.richness(sp))
        _, counts = np.unique(sp, return_counts=True)
        singles.append(int((counts == 1).sum()))
    return np.array(rich), np.array(singles)


def _theta(J, nu):
    # A lineage may pick its own slot (the deme index is uniform over all J
    # slots), so the footnote's "replacement allowed" form applies: J, not J-1.
    return J * nu / (1.0 - nu)


def test_ewens_mean_richness_config1(c1_richness):
    """Mean richness over 1000 seeds of J=1000, nu=0.1 equals theta (psi(theta+J) - psi(theta))."""
    J, nu = 1000, 0.1
    th = _theta(J, nu)
    expected = th * (special.digamma(th + J) - special.digamma(th))
    assert abs(expected - E.ewens_mean(J, nu)) < 1e-9
    rich, _ = c1_richness
    se = rich.std(ddof=1) / math.sqrt(len(rich))
    assert abs(rich.mean() - expected) < 4 * se, (rich.mean(), expected, se)


def test_richness_distribution_is_poisson_binomial(c1_richness):
    """The count-changing jump chain is the Hoppe urn, so S = sum_i Bernoulli(theta/(theta+i)):
    chi-square of the richness histogram against that exact law."""
    J, nu = 1000, 0.1
    th = _theta(J, nu)
    p = th / (th + np.arange(J))
    pmf = np.zeros(J + 1)
    pmf[0] = 1.0
    for pi in p:
        pmf[1:] = pmf[1:] * (1 - pi) + pmf[:-1] * pi
        pmf[0] *= 1 - pi
    rich, _ = c1_richness
    var = float((p * (1 - p)).sum())
    assert abs(rich.var(ddof=1) / var - 1.0) < 0.2
    edges = [0] + list(range(int(E.ewens_mean(J, nu) - 18), int(E.ewens_mean(J, nu) + 19), 4)) + [J + 1]
    obs = np.histogram(rich, bins=edges)[0]
    exp = np.array([pmf[a:b].sum() for a, b in zip(edges[:-1], edges[1:])]) * len(rich)
    chi2 = ((obs - exp) ** 2 / exp).sum()
    pval = stats.chi2.sf(chi2, len(obs) - 1)
    assert pval > 1e-3, (chi2, pval)


def test_ewens_sampling_formula_singletons(c1_richness):
    """Ewens sampling formula: E[#species with exactly one individual] = J theta / (theta + J - 1)."""
    J, nu = 1000, 0.1
    th = _theta(J, nu)
    _, singles = c1_richness
    se = singles.std(ddof=1) / math.sqrt(len(singles))
    assert abs(singles.mean() - J * th / (th + J - 1)) < 4 * se


def test_large_theta_limit_is_loose_sanity():
    """S ~ theta log(1/nu) for large theta (appendix, large-theta limit): same order of magnitude."""
    J, nu = 20000, 0.2
    wl = W.nonspatial(J, nu, [3])
    sc = oracle.Scenario(wl.capacity, wl.weights, nu)
    sp, _, _ = sc.simulate_naive(3, wl.samples)
    s = oracle.richness(sp)
    assert 0.5 < s / (_theta(J, nu) * math.log(1 / nu)) < 1.5
    assert abs(s - E.ewens_mean(J, nu)) < 5 * math.sqrt(E.ewens_mean(J, nu))


# --------------------------------------------------------------------------- #
# Exact brute force on tiny landscapes                                          #
# --------------------------------------------------------------------------- #

TINY = [
    ("3x3 cap1 R1 shared", np.ones((3, 3), np.uint32), W.gaussian_kernel(1.0, 1), 0, 0.2),
    ("3x4 cap1 R1 shared", np.ones((3, 4), np.uint32), W.gaussian_kernel(0.8, 1), 0, 0.3),
    ("3x3 mixed caps per-deme", np.array([[1, 2, 0], [0, 1, 3], [2, 0, 1]], np.uint32), W.gaussian_kernel(1.0, 1), 1,
     0.2),
    ("3x3 cap1 flat kernel", np.ones((3, 3), np.uint32), np.ones((3, 3)), 0, 0.1),
    ("nonspatial J=7", np.array([[7]], np.uint32), np.ones((1, 1)), 0, 0.25),
]


@pytest.mark.parametrize("name,cap,w,mode,nu", TINY, ids=[t[0] for t in TINY])
def test_tiny_landscape_matches_exact_chain(name, cap, w, mode, nu):
    """Monte Carlo mean richness of the oracle vs the exact expectation of the reverse-time chain."""
    sc = oracle.Scenario(cap, w, nu, mode=mode)
    n = sc.individuals
    samples = np.arange(n, dtype=np.uint64)
    exact = E.expected_richness(cap, w, mode, nu, range(n))
    N = 12000
    r = np.array([oracle.richness(sc.simulate_naive(seed, samples)[0]) for seed in range(N)], dtype=np.float64)
    se = r.std(ddof=1) / math.sqrt(N)
    assert abs(r.mean() - exact) < 4.5 * se, (name, r.mean(), exact, se)


def test_tiny_landscape_subset_sample():
    """Same, for a strict subset of slots sampled (survey-area semantics)."""
    cap = np.array([[1, 2, 0], [0, 1, 3], [2, 0, 1]], np.uint32)
    w = W.gaussian_kernel(1.2, 1)
    sc = oracle.Scenario(cap, w, 0.15, mode=1)
    pick = [0, 3, 4, 8]
    exact = E.expected_richness(cap, w, 1, 0.15, pick)
    N = 15000
    r = np.array([oracle.richness(sc.simulate_naive(seed, np.array(pick, np.uint64))[0]) for seed in range(N)])
    se = r.std(ddof=1) / math.sqrt(N)
    assert abs(r.mean() - exact) < 4.5 * se


# --------------------------------------------------------------------------- #
# Special cases                                                               #
# --------------------------------------------------------------------------- #

def test_nu_one_gives_one_species_per_distinct_sample():
    wl = W.spatial_torus(16, 2, 1.5, 3, 1.0, [9])
    sc = oracle.Scenario(wl.capacity, wl.weights, 1.0)
    samples = np.concatenate([wl.samples, wl.samples[:10]])
    sp, _, ev = sc.simulate_naive(9, samples)
    assert np.all(ev == 1)
    assert oracle.richness(sp) == len(wl.samples)
    assert np.array_equal(sp[-10:], sp[:10])


def test_single_sample_has_one_species():
    wl = W.config2()
    sc = oracle.Scenario(wl.capacity, wl.weights, 0.05)
    sp, _, _ = sc.simulate_naive(1, np.array([12345], np.uint64))
    assert oracle.richness(sp) == 1


def test_no_dispersal_no_coalescence_speciation_times_exponential():
    """Kernel concentrated on the own cell and one individual per cell: no lineage
    can meet another, so S = n, and speciation times are Exp(lambda nu) (the
    paper's speciation-time test with dispersal disabled)."""
    L, nu = 16, 0.05
    cap = np.ones((L, L), np.uint32)
    sc = oracle.Scenario(cap, np.ones((1, 1)), nu)
    times = []
    for seed in range(8):
        sp, ts, _ = sc.simulate_naive(seed, np.arange(L * L, dtype=np.uint64))
        assert oracle.richness(sp) == L * L
        times.extend(ts)
    assert stats.kstest(np.array(times) * nu, "expon").pvalue > 1e-3


def test_inter_event_times_along_a_lineage_are_exponential():
    """Inter-event times of a dispersing lineage are Exp(lambda) (paper: turnover test)."""
    wl = W.config2()
    sc = oracle.Scenario(wl.capacity, wl.weights, 1e-6)
    gaps = []
    for seed in range(4):
        t, *_ = sc.trace(seed, 777 + seed, max_events=5000)
        gaps.extend(np.diff(np.concatenate([[0.0], t])))
    assert stats.kstest(gaps, "expon").pvalue > 1e-3


def test_stationary_lineage_inter_event_times():
    """Stress case of a lineage that can never move (J = 1): gaps still Exp(lambda)."""
    sc = oracle.Scenario(np.array([[1]], np.uint32), np.ones((1, 1)), 1e-7)
    t, *_ = sc.trace(5, 0, max_events=8000)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert stats.kstest(gaps, "expon").pvalue > 1e-3


# --------------------------------------------------------------------------- #
# Dispersal law (paper: uniform and normal dispersal tests)                     #
# --------------------------------------------------------------------------- #

def _chi2_p(obs, probs, min_expected=5.0):
    exp = probs * obs.sum()
    keep = exp >= min_expected
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] == 0:
        o, e = o[:-1], e[:-1]
    chi2 = ((o - e) ** 2 / e).sum()
    return stats.chi2.sf(chi2, len(o) - 1)


def test_normal_dispersal_offsets_follow_kernel():
    """Realised (dx, dy) of dispersals on the config-2 kernel vs the exact kernel weights:
    joint chi-square and per-axis chi-square (the paper tests each axis)."""
    wl = W.config2()
    sc = oracle.Scenario(wl.capacity, wl.weights, 1e-7)
    R = 10
    joint = np.zeros((2 * R + 1, 2 * R + 1))
    for seed in range(6):
        _, _, dx, dy, _ = sc.trace(seed, 1000 * seed, max_events=20000)
        np.add.at(joint, (dy + R, dx + R), 1)
    p = wl.weights / wl.weights.sum()
    assert _chi2_p(joint.ravel(), p.ravel()) > 1e-3
    assert _chi2_p(joint.sum(0), p.sum(0)) > 1e-3
    assert _chi2_p(joint.sum(1), p.sum(1)) > 1e-3


def test_uniform_dispersal_visits_every_index_equally():
    """Non-spatial deme: every deme index is visited with equal probability."""
    J = 25
    sc = oracle.Scenario(np.array([[J]], np.uint32), np.ones((1, 1)), 1e-7)
    _, locs, _, _, _ = sc.trace(3, 0, max_events=50000)
    obs = np.bincount(locs, minlength=J).astype(float)
    assert _chi2_p(obs, np.full(J, 1.0 / J)) > 1e-3


def test_per_deme_dispersal_prefers_by_capacity():
    """Per-deme tables: the first parent cell from a fixed deme is drawn in proportion to kernel
    weight times target capacity, never onto uninhabitable cells, deme index uniform."""
    cap = W.fractal_capacity(16, 3, base_period=8)
    w = W.gaussian_kernel(1.5, 3)
    sc = oracle.Scenario(cap, w, 1e-9, mode=1)
    Wd = 16
    src = int(np.flatnonzero(cap.ravel() >= 4)[0])
    first = int(np.concatenate([[0], np.cumsum(cap.ravel())])[src])
    counts = {}
    cmax = sc.cmax
    for seed in range(12000):
        _, locs, dx, dy, _ = sc.trace(seed, first, max_events=2)
        cell = int(locs[1]) // cmax
        counts[cell] = counts.get(cell, 0) + 1
        assert cap.ravel()[cell] > 0
        assert int(locs[1]) % cmax < cap.ravel()[cell]
    x0, y0 = src % Wd, src // Wd
    mass = {}
    for dyy in range(-3, 4):
        for dxx in range(-3, 4):
            t = ((y0 + dyy) % 16) * 16 + (x0 + dxx) % 16
            m = w[dyy + 3, dxx + 3] * cap.ravel()[t]
            if m > 0:
                mass[t] = mass.get(t, 0.0) + m
    cells = sorted(mass)
    probs = np.array([mass[c] for c in cells])
    probs /= probs.sum()
    obs = np.array([counts.get(c, 0) for c in cells], float)
    assert sum(counts.values()) == obs.sum()
    assert _chi2_p(obs, probs) > 1e-3


# --------------------------------------------------------------------------- #
# Stream correlation (paper: Spearman test of adjacent start locations)         #
# --------------------------------------------------------------------------- #

def test_adjacent_location_streams_uncorrelated():
    """100-draw event-time streams of four lineages at adjacent cells, over 300 seeds: Spearman
    correlations between the cells' waiting times are not significant overall."""
    sc = oracle.Scenario(np.ones((8, 8), np.uint32), W.gaussian_kernel(1.0, 1), 0.01)
    pvals = []
    for seed in range(300):
        streams = []
        for loc in (0, 1, 8, 9):
            t, out = 0.0, []
            for _ in range(100):
                n = sc.next_event_time(seed, loc, t)
                out.append(n - t)
                t = n
            streams.append(out)
        for a in range(4):
            for b in range(a + 1, 4):
                pvals.append(stats.spearmanr(streams[a], streams[b]).pvalue)
    # p-values of independent tests are uniform: Fisher's method, and a KS check of uniformity
    fisher = stats.combine_pvalues(pvals, method="fisher").pvalue
    assert 1e-3 < fisher < 1 - 1e-3
    assert stats.kstest(pvals, "uniform").pvalue > 1e-3


# --------------------------------------------------------------------------- #
# Invariants: culling, subsets, permutations, duplicates                       #
# --------------------------------------------------------------------------- #

SMALL = [
    W.nonspatial(300, 0.05, [4], name="nonspatial"),
    W.spatial_torus(24, 2, 1.5, 4, 0.02, [5], name="torus"),
    W.Workload("fractal", W.fractal_capacity(24, 11, base_period=8), W.gaussian_kernel(2.0, 5), 0.02, 1,
               np.zeros(0, np.uint64), [6]),
]


@pytest.mark.parametrize("wl", SMALL, ids=[w.name for w in SMALL])
@pytest.mark.parametrize("dW", [0.5, 3.0, 64.0])
def test_culled_equals_naive(wl, dW):
    """Any cull schedule gives bitwise the same species per sample as tracing each sample alone."""
    sc = oracle.Scenario(wl.capacity, wl.weights, wl.nu, mode=wl.mode)
    samples = np.arange(sc.individuals, dtype=np.uint64)
    a, _, ev_naive = sc.simulate_naive(wl.seeds[0], samples)
    b, ev_culled, rounds = sc.simulate_culled(wl.seeds[0], samples, dW)
    assert np.array_equal(a, b)
    assert ev_culled <= int(ev_naive.sum())
    assert rounds >= 1


def test_subset_and_permutation_invariance():
    """simulate(S) restricted to A equals simulate(A), in any order and with duplicates
    (isolated-individuals partitioning gives identical results)."""
    wl = SMALL[1]
    sc = oracle.Scenario(wl.capacity, wl.weights, wl.nu)
    n = sc.individuals
    full, _, _ = sc.simulate_culled(5, np.arange(n, dtype=np.uint64), 4.0)
    rng = np.random.default_rng(0)
    for _ in range(3):
        sub = rng.choice(n, size=97, replace=True).astype(np.uint64)
        part, _, _ = sc.simulate_culled(5, sub, 2.0)
        assert np.array_equal(part, full[sub.astype(np.int64)])
    perm = rng.permutation(n).astype(np.uint64)
    p2, _, _ = sc.simulate_naive(5, perm[:200])
    assert np.array_equal(p2, full[perm[:200].astype(np.int64)])


def test_seed_changes_result():
    wl = SMALL[1]
    sc = oracle.Scenario(wl.capacity, wl.weights, wl.nu)
    s = np.arange(100, dtype=np.uint64)
    assert not np.array_equal(sc.simulate_naive(1, s)[0], sc.simulate_naive(2, s)[0])


def test_species_ids_come_from_the_speciation_event():
    """Species id = species-domain hash of (location, time) of the speciation event."""
    wl = SMALL[1]
    sc = oracle.Scenario(wl.capacity, wl.weights, wl.nu)
    sp, ts, _ = sc.simulate_naive(8, np.arange(5, dtype=np.uint64))
    for k in range(5):
        t, locs, _, _, done = sc.trace(8, k, max_events=100000)
        assert done and t[-1] == ts[k]
        assert oracle.species_id(8, int(locs[-1]), float(t[-1])) == sp[k]


def test_rejects_out_of_range_samples():
    wl = SMALL[1]
    sc = oracle.Scenario(wl.capacity, wl.weights, wl.nu)
    with pytest.raises(ValueError):
        sc.simulate_naive(1, np.array([sc.individuals], np.uint64))
