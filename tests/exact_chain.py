"""Exact expected species richness of the reverse-time neutral model on tiny
landscapes, by solving the jump chain over sets of occupied slots.

This is a pin for the oracle that shares nothing with it: it works from the
model's definition (background sections on the neutral model and its
reverse-time coalescence simulation; "Coalescence a la Gillespie"), not from
the Independent algorithm's RNG construction.

Model.  A slot is an indexed location (cell, deme index).  Every occupied slot
carries an event stream of rate lambda; the rates are equal, so the next
event belongs to a uniformly chosen lineage.  At an event of the lineage at
slot a: with probability nu it speciates (one new species; a leaves the set);
otherwise its parent slot b is drawn from the dispersal law D(a, .) -- target
cell by kernel weight (times target capacity in per-deme mode), deme index
uniform over the target's capacity.  If b holds another lineage the two
coalesce (a leaves); if b == a nothing changes; otherwise a moves to b.

S(A) = expected number of species found from the occupied set A satisfies

  S(A) = 1/|A| sum_{a in A} [ nu (1 + S(A - a))
                              + (1-nu) sum_b D(a,b) S(next(A, a, b)) ]

which is solved level by level in |A| (a linear system per level, because a
move or a no-op keeps |A|).
"""
from __future__ import annotations

from itertools import combinations

import numpy as np


def slots_of(capacity: np.ndarray):
    H, W = capacity.shape
    out = []
    for c in range(H * W):
        for i in range(int(capacity.flat[c])):
            out.append((c, i))
    return out


def dispersal_law(capacity: np.ndarray, weights: np.ndarray, mode: int) -> np.ndarray:
    """D[a, b] over slots, from the exact kernel weights (no alias table)."""
    H, W = capacity.shape
    R = weights.shape[0] // 2
    slots = slots_of(capacity)
    index = {s: k for k, s in enumerate(slots)}
    n = len(slots)
    D = np.zeros((n, n), dtype=np.float64)
    for a, (c, _) in enumerate(slots):
        x, y = c % W, c // W
        cell_mass = {}
        for dy in range(-R, R + 1):
            for dx in range(-R, R + 1):
                w = weights[dy + R, dx + R]
                tx, ty = (x + dx) % W, (y + dy) % H
                t = ty * W + tx
                if mode == 1:
                    w = w * capacity[ty, tx]
                if w > 0:
                    cell_mass[t] = cell_mass.get(t, 0.0) + w
        total = sum(cell_mass.values())
        for t, m in cell_mass.items():
            cap_t = int(capacity.flat[t])
            for i in range(cap_t):
                D[a, index[(t, i)]] += (m / total) / cap_t
    return D


def expected_richness(capacity: np.ndarray, weights: np.ndarray, mode: int, nu: float, start_slots) -> float:
    """E[S] for the set of initially occupied slots (indices into slots_of(capacity))."""
    D = dispersal_law(capacity, weights, mode)
    return expected_richness_law(D, np.full(D.shape[0], nu), start_slots)


def implicit_law(J: int, J_meta: int, m: float) -> tuple[np.ndarray, list]:
    """Slot-level law of the spatially implicit model (background section "Spatially Implicit"):
    slots 0..J-1 are the local community, J..J+J_meta-1 the metacommunity.  A local lineage's
    parent is a uniform metacommunity slot with probability m, else a uniform local slot; a
    metacommunity lineage's parent is a uniform metacommunity slot."""
    n = J + J_meta
    D = np.zeros((n, n))
    D[:J, :J] = (1.0 - m) / J
    D[:J, J:] = m / J_meta
    D[J:, J:] = 1.0 / J_meta
    return D, list(range(J))


def richness_table(D: np.ndarray, nu_slot: np.ndarray, m_max: int) -> dict:
    """E[S] for every occupied set of at most m_max slots, under a slot-level dispersal law D and a
    per-slot speciation probability."""
    n = D.shape[0]
    S = {frozenset(): 0.0}
    for m in range(1, m_max + 1):
        level = [frozenset(c) for c in combinations(range(n), m)]
        pos = {A: k for k, A in enumerate(level)}
        M = np.eye(len(level))
        rhs = np.zeros(len(level))
        for A, row in pos.items():
            for a in A:
                rest = A - {a}
                nu = nu_slot[a]
                rhs[row] += nu * (1.0 + S[rest]) / m
                for b in range(n):
                    p = D[a, b]
                    if p == 0.0:
                        continue
                    coef = (1.0 - nu) * p / m
                    if b in rest:
                        rhs[row] += coef * S[rest]
                    elif b == a:
                        M[row, row] -= coef
                    else:
                        M[row, pos[rest | {b}]] -= coef
        sol = np.linalg.solve(M, rhs)
        for A, k in pos.items():
            S[A] = float(sol[k])
    return S


def expected_richness_law(D: np.ndarray, nu_slot: np.ndarray, start_slots) -> float:
    """E[S] for a slot-level dispersal law D and a per-slot speciation probability."""
    start = frozenset(start_slots)
    return richness_table(D, nu_slot, len(start))[start]


def protracted_expected_richness_law(D: np.ndarray, nu_slot: np.ndarray, tau: float, start_slots) -> float:
    """E[S] under protracted speciation (appendix "Protracted Speciation"): for the first tau
    generations back from the present no speciation counts, so the occupied set evolves by
    dispersal and coalescence alone, each lineage moving once per generation on average (a
    continuous-time chain over occupied sets, solved with a matrix exponential); from tau on,
    the point-speciation chain above takes over from whichever set is occupied then (the events
    are memoryless, so the two phases join at tau)."""
    from scipy.linalg import expm

    n = D.shape[0]
    start = frozenset(start_slots)
    sets = [frozenset(c) for m in range(1, len(start) + 1) for c in combinations(range(n), m)]
    pos = {A: k for k, A in enumerate(sets)}
    Q = np.zeros((len(sets), len(sets)))
    for A, row in pos.items():
        for a in A:
            rest = A - {a}
            for b in range(n):
                p = D[a, b]
                if p == 0.0 or b == a:
                    continue
                to = rest if b in rest else rest | {b}
                Q[row, pos[to]] += p
                Q[row, row] -= p
    P = expm(Q * tau)[pos[start]]
    S = richness_table(D, nu_slot, len(start))
    return float(sum(P[k] * S[A] for A, k in pos.items()))


def ewens_mean(J: int, nu: float) -> float:
    """Closed form for the non-spatial deme when a lineage may pick its own slot: theta = J nu / (1 - nu),
    E[S] = sum_{i<J} theta / (theta + i)."""
    theta = J * nu / (1.0 - nu)
    return float(sum(theta / (theta + i) for i in range(J)))
