"""Seeded synthetic inputs for the Independent-algorithm workloads.

This module holds input generation only -- landscapes, dispersal-kernel
weights, sample sets, seeds, scenario mixes and request streams -- and none of
the method's arithmetic (no RNG priming, no alias tables, no event sampling).
Both the HIP path and the CPU oracle consume what it produces.  All randomness
comes from numpy's PCG64 with fixed seeds, so every input is reproducible.

Workloads (they stand in for the paper's scenarios and the Madingley maps,
which are not available):

* ``nonspatial``: one well-mixed deme of J individuals on a 1x1 torus with a
  1x1 kernel (the paper's non-spatial scenario, closed community).
* ``spatial_torus``: an L x L torus with constant deme capacity and a point-
  evaluated Gaussian kernel exp(-(dx^2+dy^2)/(2 sigma^2)) over |dx|,|dy| <= R
  (the paper's spatially explicit scenario with normal dispersal).
* ``fractal_habitat``: a heterogeneous capacity map from periodic fractal
  value noise, with a rank threshold that makes a fixed fraction of cells
  uninhabitable and splits the rest into equal-size capacity classes (stands in
  for a habitat map with per-cell dispersal).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    """One scenario plus the samples and seed(s) to simulate it with."""
    name: str
    capacity: np.ndarray          # (H, W) uint32
    weights: np.ndarray           # (2R+1, 2R+1) float64
    nu: float
    mode: int                     # 0: one shared kernel table, 1: per-deme tables over habitable targets
    samples: np.ndarray           # uint64 dense individual ids
    seeds: list = field(default_factory=list)
    lam: float = 1.0
    dt: float = 1.0
    meta: dict = field(default_factory=dict)
    sampler: int = 0              # 0: exponential sums, 1: Poisson count per interval
    tau: float = 0.0              # protracted speciation (generations); 0: point speciation

    @property
    def individuals(self) -> int:
        return int(self.capacity.astype(np.uint64).sum())


def gaussian_kernel(sigma: float, radius: int) -> np.ndarray:
    """Point-evaluated Gaussian weights on the (2R+1)^2 grid; row = dy + R, column = dx + R."""
    d = np.arange(-radius, radius + 1, dtype=np.float64)
    dy, dx = np.meshgrid(d, d, indexing="ij")
    return np.exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma))


def all_samples(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.uint64)


def sample_fraction(n: int, frac: float, seed: int) -> np.ndarray:
    """round(frac * n) distinct dense ids drawn without replacement, sorted."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = int(round(frac * n))
    return np.sort(rng.choice(n, size=m, replace=False)).astype(np.uint64)


def nonspatial(J: int, nu: float, seeds, name: str = "nonspatial") -> Workload:
    cap = np.array([[J]], dtype=np.uint32)
    w = np.ones((1, 1), dtype=np.float64)
    return Workload(name, cap, w, nu, 0, all_samples(J), list(seeds), meta={"J": J})


def spatial_torus(L: int, cap: int, sigma: float, radius: int, nu: float, seeds, samples=None,
                  name: str = "spatial") -> Workload:
    capacity = np.full((L, L), cap, dtype=np.uint32)
    n = L * L * cap
    return Workload(name, capacity, gaussian_kernel(sigma, radius), nu, 0,
                    all_samples(n) if samples is None else samples, list(seeds),
                    meta={"L": L, "cap": cap, "sigma": sigma, "R": radius})


def _smoothstep(x: np.ndarray) -> np.ndarray:
    return x * x * (3.0 - 2.0 * x)


def fractal_value_noise(L: int, seed: int, octaves: int = 6, base_period: int = 256,
                        gain: float = 0.5) -> np.ndarray:
    """Periodic fractal value noise on an L x L grid: octave o has a random
    lattice of period base_period / 2^o (uniform [0,1) values, wrapped), bilinear
    interpolation with smoothstep weights, amplitude gain^o."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.zeros((L, L), dtype=np.float64)
    amp = 1.0
    period = base_period
    for _ in range(octaves):
        period = max(1, period)
        cells = max(1, L // period)
        lattice = rng.random((cells, cells))
        coord = np.arange(L, dtype=np.float64) / period
        i0 = np.floor(coord).astype(np.int64) % cells
        i1 = (i0 + 1) % cells
        f = _smoothstep(coord - np.floor(coord))
        # rows (y) then columns (x)
        top = lattice[i0][:, i0] * (1 - f)[None, :] + lattice[i0][:, i1] * f[None, :]
        bot = lattice[i1][:, i0] * (1 - f)[None, :] + lattice[i1][:, i1] * f[None, :]
        out += amp * (top * (1 - f)[:, None] + bot * f[:, None])
        amp *= gain
        period //= 2
    return out


def fractal_capacity(L: int, seed: int, zero_frac: float = 0.3, max_cap: int = 8, octaves: int = 6,
                     base_period: int = 256) -> np.ndarray:
    """Rank-threshold fractal noise: exactly floor(zero_frac * L^2) lowest cells get capacity 0, the
    rest are split by rank into max_cap equal bins with capacities 1..max_cap."""
    noise = fractal_value_noise(L, seed, octaves=octaves, base_period=base_period)
    order = np.argsort(noise, axis=None, kind="stable")
    n = L * L
    n_zero = int(math.floor(zero_frac * n))
    cap = np.zeros(n, dtype=np.uint32)
    rest = order[n_zero:]
    bins = (np.arange(len(rest)) * max_cap) // len(rest) + 1
    cap[rest] = bins.astype(np.uint32)
    return cap.reshape(L, L)


# ---------------------------------------------------------------------------
# The five workload configurations (and scaled-down variants for parity tests)
# ---------------------------------------------------------------------------

def config1(n_seeds: int = 1000) -> Workload:
    """Non-spatial deme of J = 1000, all sampled, nu = 0.1, seeds 0..n_seeds-1."""
    return nonspatial(1000, 0.1, range(n_seeds), name="C1 nonspatial J=1000 nu=0.1")


def config2(seeds=(42,)) -> Workload:
    """256 x 256 torus, one individual per cell, Gaussian sigma = 2 on a 21 x 21 kernel, nu = 1e-3."""
    return spatial_torus(256, 1, 2.0, 10, 1e-3, seeds, name="C2 torus 256x256 sigma=2 R=10 nu=1e-3")


def config3(L: int = 1024, seeds=(42,), noise_seed: int = 7, sample_seed: int = 8, frac: float = 0.1) -> Workload:
    """L x L fractal habitat (30% empty, capacities 1..8), per-deme tables over a 31 x 31 Gaussian
    kernel with sigma = 4, nu = 1e-5, a 10% uniform sample of individuals."""
    base = min(256, L // 4) if L < 1024 else 256
    cap = fractal_capacity(L, noise_seed, base_period=base)
    n = int(cap.astype(np.uint64).sum())
    return Workload(f"C3 fractal habitat {L}x{L} sigma=4 R=15 nu=1e-5 10% sample", cap, gaussian_kernel(4.0, 15),
                    1e-5, 1, sample_fraction(n, frac, sample_seed), list(seeds),
                    meta={"L": L, "sigma": 4.0, "R": 15, "frac": frac})


def config4(master_seed: int = 2108, n: int = 256, side_range=(64, 512), nu_range=(1e-6, 1e-2),
            sigma_range=(1.0, 6.0), cap_range=(1, 4)) -> list:
    """Scenario mix: side log-uniform in side_range, constant capacity per scenario uniform in
    cap_range, sigma uniform in sigma_range with R = ceil(5 sigma), nu log-uniform in nu_range, one
    distinct 64-bit seed per scenario, all individuals sampled."""
    rng = np.random.Generator(np.random.PCG64(master_seed))
    out = []
    seeds = set()
    for k in range(n):
        L = int(round(math.exp(rng.uniform(math.log(side_range[0]), math.log(side_range[1])))))
        cap = int(rng.integers(cap_range[0], cap_range[1] + 1))
        sigma = float(rng.uniform(*sigma_range))
        R = int(math.ceil(5.0 * sigma))
        R = min(R, (L - 1) // 2)
        nu = float(math.exp(rng.uniform(math.log(nu_range[0]), math.log(nu_range[1]))))
        seed = int(rng.integers(0, 2**63 - 1, dtype=np.int64)) * 2 + int(rng.integers(0, 2))
        while seed in seeds:
            seed += 1
        seeds.add(seed)
        w = spatial_torus(L, cap, sigma, R, nu, [seed], name=f"C4[{k}] L={L} cap={cap} sigma={sigma:.2f} nu={nu:.2e}")
        out.append(w)
    return out


def config5_requests(rate: float = 200.0, duration: float = 60.0, seed: int = 5, master_seed: int = 2109,
                     spatial_side=(64, 512), J_range=(1e3, 1e6), nu_range=(1e-6, 1e-2)):
    """Poisson request stream: arrival times (s) and one request spec per arrival, half config-4-like
    spatial scenarios, half non-spatial demes with J log-uniform in J_range; materialize() turns a spec
    into its Workload (done on arrival, so the stream itself stays small)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rng.poisson(rate * duration))
    arrivals = np.sort(rng.uniform(0.0, duration, size=n))
    mix = np.random.Generator(np.random.PCG64(master_seed))
    specs = []
    for k in range(n):
        nu = float(math.exp(mix.uniform(math.log(nu_range[0]), math.log(nu_range[1]))))
        seed_k = int(mix.integers(0, 2**62))
        if mix.random() < 0.5:
            L = int(round(math.exp(mix.uniform(math.log(spatial_side[0]), math.log(spatial_side[1])))))
            cap = int(mix.integers(1, 5))
            sigma = float(mix.uniform(1.0, 6.0))
            R = min(int(math.ceil(5.0 * sigma)), (L - 1) // 2)
            specs.append({"kind": "spatial", "L": L, "cap": cap, "sigma": sigma, "R": R, "nu": nu, "seed": seed_k,
                          "name": f"req{k} spatial L={L}"})
        else:
            J = int(round(math.exp(mix.uniform(math.log(J_range[0]), math.log(J_range[1])))))
            specs.append({"kind": "nonspatial", "J": J, "nu": nu, "seed": seed_k, "name": f"req{k} nonspatial J={J}"})
    return arrivals, specs


def materialize(spec: dict) -> Workload:
    if spec["kind"] == "spatial":
        return spatial_torus(spec["L"], spec["cap"], spec["sigma"], spec["R"], spec["nu"], [spec["seed"]],
                             name=spec["name"])
    return nonspatial(spec["J"], spec["nu"], [spec["seed"]], name=spec["name"])


def spec_individuals(spec: dict) -> int:
    return spec["L"] * spec["L"] * spec["cap"] if spec["kind"] == "spatial" else spec["J"]
