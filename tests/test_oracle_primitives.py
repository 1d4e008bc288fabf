"""Pins for the oracle's primitives: the counter-based hash, the logarithm,
the alias tables and the next-event search.  Nothing here compares the oracle
with itself: each check is against published vectors, a library routine with a
known error bound, exact arithmetic, or a mathematical invariant."""
import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2108_05815_amd.workloads import gaussian_kernel

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if line:
                v = [int(x, 16) for x in line]
                rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expected", _kat())
def test_philox_known_answers(ctr, key, expected):
    """Philox4x32-10 block function equals the published known-answer vectors."""
    assert list(oracle.philox4x32_10(ctr, key)) == expected


def test_philox_strict_avalanche():
    """Strict avalanche criterion (background section on hash functions and the
    avalanche effect): flipping any one of the 192 input bits flips each of the
    128 output bits with probability 1/2."""
    rng = np.random.default_rng(1)
    trials = 96
    flips = np.zeros((192, 128))
    for _ in range(trials):
        ctr = rng.integers(0, 2**32, size=4, dtype=np.uint64).astype(np.uint32)
        key = rng.integers(0, 2**32, size=2, dtype=np.uint64).astype(np.uint32)
        base = oracle.philox4x32_10(ctr, key)
        for bit in range(192):
            c2, k2 = ctr.copy(), key.copy()
            if bit < 128:
                c2[bit // 32] ^= np.uint32(1 << (bit % 32))
            else:
                k2[(bit - 128) // 32] ^= np.uint32(1 << (bit % 32))
            out = oracle.philox4x32_10(c2, k2)
            diff = base ^ out
            flips[bit] += np.unpackbits(diff.view(np.uint8), bitorder="little")
    p = flips / trials
    sd = math.sqrt(0.25 / trials)
    assert np.abs(p - 0.5).max() < 5.5 * sd
    assert abs(p.mean() - 0.5) < 0.01


def test_log_special_values():
    assert oracle.log(1.0) == 0.0
    assert oracle.log(0.5) == -math.log(2.0)
    assert oracle.log(0.25) == -2.0 * math.log(2.0)
    assert oracle.log(2.0**-53) == float(-53 * mpmath.log(2))


def _ulp_error(x: float) -> float:
    mpmath.mp.prec = 160
    true = mpmath.log(mpmath.mpf(x))
    got = oracle.log(x)
    return float(abs(mpmath.mpf(got) - true) / mpmath.mpf(math.ulp(got) if got != 0 else 2.0**-1074))


def test_log_accuracy_against_arbitrary_precision():
    """Within 2 ulp of the exact logarithm on the 2^-53 grid the waiting-time
    sampler feeds it: random points, points near the sqrt(2) cut, near 1, tiny.
    (The worst case, about 1.9 ulp, is just below the cut, where e*ln2 and
    log(m) cancel to half their size.)"""
    rng = np.random.default_rng(2)
    q = rng.integers(1, 2**53, size=1500, dtype=np.int64)
    xs = [float(int(v)) * 2.0**-53 for v in q]
    cut = float.fromhex("0x1.6a09e667f3bcdp-1")
    xs += [math.nextafter(cut, 0), cut, math.nextafter(cut, 1), 1.0 - 2.0**-53, 1.0 - 2**-40,
           2.0**-53, 3 * 2.0**-53, 0.5 + 2**-53, 0.9999, 1e-3, 0.75]
    worst = max(_ulp_error(x) for x in xs)
    assert worst <= 2.0, worst


def test_log_matches_libm_closely():
    """Against the C library's log (itself within 1 ulp): at most 2 ulp apart on 20000 grid points."""
    rng = np.random.default_rng(3)
    q = rng.integers(1, 2**53, size=20000, dtype=np.int64)
    worst = 0.0
    for v in q:
        x = float(int(v)) * 2.0**-53
        a, b = oracle.log(x), math.log(x)
        worst = max(worst, abs(a - b) / math.ulp(b))
    assert worst <= 2.0


@pytest.mark.parametrize("weights", [
    [1.0],
    [1.0, 1.0, 1.0],
    [0.1, 0.2, 0.3, 0.4],
    [5.0, 0.0, 1.0, 0.0, 2.0],
    list(gaussian_kernel(2.0, 10).ravel()),
    list(gaussian_kernel(4.0, 15).ravel()),
    list(np.random.default_rng(4).random(97) ** 3),
])
def test_alias_table_reconstructs_weights(weights):
    """Each outcome's mass in the Vose table (own column probability plus the
    remainders of the columns aliased to it) equals w_i / sum(w), checked in
    exact rational arithmetic.  The table's own f64 rounding accumulates over at
    most n updates of one column, so each outcome may be off by n * 2^-52 in
    absolute probability; a wrong alias or a dropped remainder is off by ~1/n."""
    w = np.asarray(weights, dtype=np.float64)
    prob, alias = oracle.alias_build(w)
    n = len(w)
    assert np.all((prob >= 0.0) & (prob <= 1.0))
    assert np.all(alias < n)
    mass = [Fraction(0)] * n
    for j in range(n):
        pj = Fraction(float(prob[j]))
        mass[j] += pj
        if alias[j] != j:
            mass[int(alias[j])] += 1 - pj
        else:
            mass[j] += 1 - pj
    total = sum(Fraction(float(x)) for x in w)
    for i in range(n):
        want = Fraction(float(w[i])) / total
        got = mass[i] / n
        assert abs(got - want) <= n * Fraction(1, 2**52), (i, float(got), float(want))
        if w[i] == 0.0:
            assert got == 0


def test_alias_rejects_bad_weights():
    for bad in ([0.0, 0.0], [-1.0, 2.0], [float("nan")], [float("inf"), 1.0]):
        with pytest.raises(ValueError):
            oracle.alias_build(bad)


def _scenario(L=8, cap=1, sigma=1.5, R=2, nu=0.01):
    return oracle.Scenario(np.full((L, L), cap, np.uint32), gaussian_kernel(sigma, R), nu)


def test_next_event_time_is_the_next_point_of_a_fixed_point_set():
    """Aligning the RNGs of colliding individuals: the event times at one slot form one fixed set
    of points, and the next event after any t is the smallest point strictly beyond t.  A lineage
    arriving anywhere in (t_prev, t_next) finds exactly t_next (bitwise)."""
    sc = _scenario()
    rng = np.random.default_rng(5)
    for loc in (0, 7, 33, 63):
        for seed in (1, 2**63 + 5):
            pts = []
            t = 0.0
            while t < 40.0:
                t = sc.next_event_time(seed, loc, t)
                pts.append(t)
            pts = np.array(pts)
            assert np.all(np.diff(pts) > 0)
            probes = list(rng.uniform(0, 38.0, size=200)) + [float(k) for k in range(38)] + list(pts[:-1])
            probes += [math.nextafter(p, 0) for p in pts[:-1]] + [math.nextafter(p, 100) for p in pts[:-2]]
            for tq in probes:
                want = pts[np.searchsorted(pts, tq, side="right")]
                assert sc.next_event_time(seed, loc, tq) == want


def test_inter_event_times_are_exponential_at_a_fixed_slot():
    """Memoryless sums of exponentials: the gaps between consecutive points at one slot are
    Exp(lambda), also across interval boundaries (KS test), for lambda = 1 and lambda = 4."""
    for lam, dt in ((1.0, 1.0), (4.0, 0.5), (0.5, 2.0)):
        sc = oracle.Scenario(np.full((4, 4), 1, np.uint32), gaussian_kernel(1.0, 1), 0.01, lam=lam, dt=dt)
        gaps = []
        for loc in range(4):
            t, prev = 0.0, 0.0
            for _ in range(1500):
                t = sc.next_event_time(11, loc, t)
                gaps.append(t - prev)
                prev = t
        p = stats.kstest(np.array(gaps) * lam, "expon").pvalue
        assert p > 1e-3, (lam, dt, p)


def test_scenario_validation():
    cap = np.ones((8, 8), np.uint32)
    w = gaussian_kernel(1.0, 1)
    for kwargs in (dict(nu=0.0), dict(nu=1.5), dict(nu=float("nan"))):
        with pytest.raises(ValueError):
            oracle.Scenario(cap, w, **kwargs)
    with pytest.raises(ValueError):
        oracle.Scenario(cap, w, 0.1, dt=3.0)  # dt must be a power of two
    with pytest.raises(ValueError):
        oracle.Scenario(cap, gaussian_kernel(1.0, 4), 0.1)  # 2R+1 > W
    with pytest.raises(ValueError):
        oracle.Scenario(np.zeros((4, 4), np.uint32), gaussian_kernel(1.0, 1), 0.1, mode=1)
    z = cap.copy()
    z[0, 0] = 0
    with pytest.raises(ValueError):
        oracle.Scenario(z, w, 0.1, mode=0)  # shared table needs every deme habitable
    oracle.Scenario(z, w, 0.1, mode=1)
