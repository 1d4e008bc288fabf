"""CPU oracle for the Independent algorithm (arXiv 2108.05815).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``, never by the product package.
It wraps ``oracle.c`` (plain single-threaded C, no FMA contraction) through
ctypes.  The shared library is built with gcc into ``oracle/_build`` on first
use, or whenever the source is newer than the built file.

Every function cites the section of the paper it follows; see ``oracle.c`` for
the step-by-step definitions.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_OUT_DIR, "liboracle.so")
_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-fvisibility=hidden", "-Wall", "-Wextra", "-Wno-unused-parameter"]

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into oracle/_build/liboracle.so and return its path."""
    os.makedirs(_OUT_DIR, exist_ok=True)
    stale = (not os.path.exists(_LIB_PATH)) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    if force or stale:
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.run(["gcc", *_FLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        lib = C.CDLL(build())
        u32p, u64p, f64p, i32p = (C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
                                  C.POINTER(C.c_double), C.POINTER(C.c_int32))
        lib.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        lib.or_philox4x32_10.restype = None
        lib.or_log.argtypes = [C.c_double]
        lib.or_log.restype = C.c_double
        lib.or_alias_build.argtypes = [f64p, C.c_uint32, f64p, u32p]
        lib.or_alias_build.restype = C.c_int
        lib.or_scenario_create.argtypes = [C.c_uint32, C.c_uint32, u32p, C.c_uint32, f64p, C.c_uint32,
                                           C.c_double, C.c_double, C.c_double, C.POINTER(C.c_void_p)]
        lib.or_scenario_create.restype = C.c_int
        lib.or_scenario_destroy.argtypes = [C.c_void_p]
        lib.or_scenario_destroy.restype = None
        lib.or_scenario_individuals.argtypes = [C.c_void_p]
        lib.or_scenario_individuals.restype = C.c_uint64
        lib.or_scenario_cmax.argtypes = [C.c_void_p]
        lib.or_scenario_cmax.restype = C.c_uint32
        lib.or_scenario_table.argtypes = [C.c_void_p, C.c_uint32, f64p, u32p, u32p, C.c_uint32]
        lib.or_scenario_table.restype = C.c_uint32
        lib.or_sample_location.argtypes = [C.c_void_p, C.c_uint64]
        lib.or_sample_location.restype = C.c_uint32
        lib.or_event_outcome.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_double]
        lib.or_event_outcome.restype = C.c_uint32
        lib.or_philox_array.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.c_uint64,
                                        C.POINTER(C.c_uint32)]
        lib.or_philox_array.restype = None
        lib.or_log_u53o_array.argtypes = [C.POINTER(C.c_uint64), C.c_uint64, C.POINTER(C.c_double)]
        lib.or_log_u53o_array.restype = None
        lib.or_next_event_time_array.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_uint32),
                                                 C.POINTER(C.c_double), C.c_uint64, C.POINTER(C.c_double)]
        lib.or_next_event_time_array.restype = None
        lib.or_event_outcome_array.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_uint32), C.POINTER(C.c_double),
                                               C.c_uint64, C.POINTER(C.c_uint32)]
        lib.or_event_outcome_array.restype = None
        lib.or_scenario_create_implicit.argtypes = [C.c_uint32, C.c_uint32, C.c_double, C.c_double, C.c_double,
                                                    C.c_double, C.POINTER(C.c_void_p)]
        lib.or_scenario_create_implicit.restype = C.c_int
        lib.or_scenario_set_sampler.argtypes = [C.c_void_p, C.c_uint32]
        lib.or_scenario_set_sampler.restype = C.c_int
        lib.or_scenario_set_protracted.argtypes = [C.c_void_p, C.c_double]
        lib.or_scenario_set_protracted.restype = C.c_int
        lib.or_event_stream.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_uint64), C.c_uint64, C.c_uint64,
                                        C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_uint32), C.c_uint64, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
                                        C.POINTER(C.c_uint64)]
        lib.or_event_stream.restype = C.c_int
        lib.or_next_event_time.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_double]
        lib.or_next_event_time.restype = C.c_double
        lib.or_simulate_naive.argtypes = [C.c_void_p, C.c_uint64, u64p, C.c_uint64, u64p, f64p, u64p]
        lib.or_simulate_naive.restype = C.c_int
        lib.or_simulate_culled.argtypes = [C.c_void_p, C.c_uint64, u64p, C.c_uint64, C.c_double, u64p,
                                           u64p, u64p]
        lib.or_simulate_culled.restype = C.c_int
        lib.or_trace.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint64, f64p, u32p, i32p, i32p,
                                 C.POINTER(C.c_int)]
        lib.or_trace.restype = C.c_uint64
        lib.or_richness.argtypes = [u64p, C.c_uint64]
        lib.or_richness.restype = C.c_uint64
        lib.or_species_id.argtypes = [C.c_uint64, C.c_uint32, C.c_double]
        lib.or_species_id.restype = C.c_uint64
        _lib = lib
        return lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block function (Salmon et al. 2011, cited in the paper's
    related work on counter-based PRNGs)."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.or_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def philox_array(ctr, key) -> np.ndarray:
    """Philox4x32-10 of every counter row (n x 4 u32) under one key (2 u32)."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros_like(c)
    lib.or_philox_array(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), len(c), _ptr(out, C.c_uint32))
    return out


def log_u53o_array(r) -> np.ndarray:
    """log(((r >> 11) + 1) 2^-53) for every u64 draw r, as the event-time search takes it."""
    lib = _load()
    x = np.ascontiguousarray(r, dtype=np.uint64)
    out = np.zeros(len(x), dtype=np.float64)
    lib.or_log_u53o_array(_ptr(x, C.c_uint64), len(x), _ptr(out, C.c_double))
    return out


def log(x: float) -> float:
    """The reproducible natural logarithm used for Exp(lambda) waiting times."""
    return _load().or_log(float(x))


def alias_build(weights) -> tuple[np.ndarray, np.ndarray]:
    """Vose alias table (prob, alias) of a weight vector."""
    lib = _load()
    w = np.ascontiguousarray(weights, dtype=np.float64)
    prob = np.zeros(len(w), dtype=np.float64)
    alias = np.zeros(len(w), dtype=np.uint32)
    rc = lib.or_alias_build(_ptr(w, C.c_double), len(w), _ptr(prob, C.c_double), _ptr(alias, C.c_uint32))
    if rc != 0:
        raise ValueError(f"alias build failed ({rc})")
    return prob, alias


EVENT_SPECIATION = 0xFFFFFFFF


def richness(species) -> int:
    """Number of distinct species identities (sort + count runs)."""
    s = np.ascontiguousarray(species, dtype=np.uint64)
    return int(_load().or_richness(_ptr(s, C.c_uint64), len(s)))


def species_id(seed: int, loc: int, t: float) -> int:
    return int(_load().or_species_id(seed, loc, t))


class Scenario:
    """A landscape (W x H torus of deme capacities), a (2R+1)^2 dispersal kernel
    of weights, speciation probability nu, turnover rate lambda and repriming
    interval dt.  mode 0 shares one alias table over the kernel between all
    demes; mode 1 builds one table per habitable deme over weight x target
    capacity (zero-capacity targets dropped)."""

    def __init__(self, capacity, weights, nu: float, *, mode: int = 0, lam: float = 1.0, dt: float = 1.0,
                 sampler: int = 0, tau: float = 0.0):
        lib = _load()
        cap = np.ascontiguousarray(capacity, dtype=np.uint32)
        if cap.ndim != 2:
            raise ValueError("capacity must be a 2-D (H, W) array")
        w = np.ascontiguousarray(weights, dtype=np.float64)
        side = w.shape[0]
        if w.ndim != 2 or w.shape[1] != side or side % 2 != 1:
            raise ValueError("weights must be a square (2R+1, 2R+1) array")
        self.H, self.W = cap.shape
        self.R = side // 2
        self.nu, self.mode, self.lam, self.dt = nu, mode, lam, dt
        self._cap, self._w = cap, w
        h = C.c_void_p()
        rc = lib.or_scenario_create(self.W, self.H, _ptr(cap, C.c_uint32), self.R, _ptr(w, C.c_double), mode,
                                    nu, lam, dt, C.byref(h))
        if rc != 0:
            raise ValueError(f"invalid scenario ({rc})")
        self._h = h
        self._lib = lib
        self.sampler = sampler
        if sampler and lib.or_scenario_set_sampler(h, sampler) != 0:
            raise ValueError("invalid event-time sampler")
        self._set_tau(tau)

    def _set_tau(self, tau: float):
        """Protracted speciation (appendix "Protracted Speciation"): speciation draws at events
        fewer than tau generations (lambda * t < tau) before the present are ignored."""
        self.tau = tau
        if tau and self._lib.or_scenario_set_protracted(self._h, tau) != 0:
            raise ValueError("invalid protracted speciation tau")

    @classmethod
    def implicit(cls, J: int, J_meta: int, m: float, nu_meta: float, *, lam: float = 1.0, dt: float = 1.0,
                 sampler: int = 0, tau: float = 0.0):
        """The spatially implicit scenario: local community J (sample ids 0..J-1) with migration
        probability m per event into a dynamic metacommunity of J_meta with speciation nu_meta."""
        self = cls.__new__(cls)
        lib = _load()
        h = C.c_void_p()
        if lib.or_scenario_create_implicit(J, J_meta, m, nu_meta, lam, dt, C.byref(h)) != 0:
            raise ValueError("invalid spatially implicit scenario")
        self._h, self._lib = h, lib
        self.H, self.W, self.R = 1, 2, 0
        self.nu, self.mode, self.lam, self.dt, self.sampler = nu_meta, 2, lam, dt, sampler
        self._cap, self._w = np.array([[J, J_meta]], np.uint32), np.ones((1, 1))
        if sampler and lib.or_scenario_set_sampler(h, sampler) != 0:
            raise ValueError("invalid event-time sampler")
        self._set_tau(tau)
        return self

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.or_scenario_destroy(h)
            self._h = None

    @property
    def individuals(self) -> int:
        return int(self._lib.or_scenario_individuals(self._h))

    @property
    def cmax(self) -> int:
        return int(self._lib.or_scenario_cmax(self._h))

    def sample_location(self, sample: int) -> int:
        return int(self._lib.or_sample_location(self._h, sample))

    def table(self, cell: int = 0):
        """(prob, alias, kernel index) of the alias table deme `cell` samples from."""
        side = 2 * self.R + 1
        cap = side * side
        prob = np.zeros(cap, np.float64)
        alias = np.zeros(cap, np.uint32)
        kidx = np.zeros(cap, np.uint32)
        n = self._lib.or_scenario_table(self._h, cell, _ptr(prob, C.c_double), _ptr(alias, C.c_uint32),
                                        _ptr(kidx, C.c_uint32), cap)
        return prob[:n], alias[:n], kidx[:n]

    def next_event_time(self, seed: int, loc: int, t_last: float) -> float:
        return float(self._lib.or_next_event_time(self._h, seed, loc, t_last))

    def _samples(self, samples):
        s = np.ascontiguousarray(samples, dtype=np.uint64)
        return s

    def simulate_naive(self, seed: int, samples):
        """Plain definition: every sample traced alone until it speciates.
        Returns (species u64[n], speciation time f64[n], events u64[n])."""
        s = self._samples(samples)
        n = len(s)
        sp = np.zeros(n, np.uint64)
        ts = np.zeros(n, np.float64)
        ev = np.zeros(n, np.uint64)
        rc = self._lib.or_simulate_naive(self._h, seed, _ptr(s, C.c_uint64), n, _ptr(sp, C.c_uint64),
                                         _ptr(ts, C.c_double), _ptr(ev, C.c_uint64))
        if rc != 0:
            raise ValueError(f"simulate_naive failed ({rc})")
        return sp, ts, ev

    def simulate_culled(self, seed: int, samples, dW: float = 16.0):
        """Horizon rounds with (location, next-event time) deduplication.
        Returns (species u64[n], committed events, rounds)."""
        s = self._samples(samples)
        n = len(s)
        sp = np.zeros(n, np.uint64)
        ev = C.c_uint64()
        rounds = C.c_uint64()
        rc = self._lib.or_simulate_culled(self._h, seed, _ptr(s, C.c_uint64), n, dW, _ptr(sp, C.c_uint64),
                                          C.byref(ev), C.byref(rounds))
        if rc != 0:
            raise ValueError(f"simulate_culled failed ({rc})")
        return sp, int(ev.value), int(rounds.value)

    def next_event_time_array(self, seed: int, loc, t) -> np.ndarray:
        l = np.ascontiguousarray(loc, dtype=np.uint32)
        x = np.ascontiguousarray(t, dtype=np.float64)
        out = np.zeros(len(l), dtype=np.float64)
        self._lib.or_next_event_time_array(self._h, seed, _ptr(l, C.c_uint32), _ptr(x, C.c_double), len(l),
                                           _ptr(out, C.c_double))
        return out

    def event_outcome_array(self, seed: int, loc, t) -> np.ndarray:
        l = np.ascontiguousarray(loc, dtype=np.uint32)
        x = np.ascontiguousarray(t, dtype=np.float64)
        out = np.zeros(len(l), dtype=np.uint32)
        self._lib.or_event_outcome_array(self._h, seed, _ptr(l, C.c_uint32), _ptr(x, C.c_double), len(l),
                                         _ptr(out, C.c_uint32))
        return out

    def event_outcome(self, seed: int, loc: int, t: float) -> int:
        """Outcome of the event at (loc, t): the new location, or EVENT_SPECIATION."""
        return int(self._lib.or_event_outcome(self._h, seed, loc, t))

    def event_stream(self, seed: int, samples):
        """The reduced event stream (sections on sorting events and reporting coalescence): every
        event of the samples' lineages once, sorted by (t, origin), as arrays t, prior (the smallest
        prior event time of its copies), origin and outcome (EVENT_SPECIATION for a speciation);
        and the coalescences as arrays t, parent (the first lineage's arrival) and location, sorted
        by (t, location, parent)."""
        s = self._samples(samples)
        n = len(s)
        ne, nc = C.c_uint64(), C.c_uint64()
        ev_cap, co_cap = 0, 0
        while True:
            et, ep = np.zeros(max(ev_cap, 1)), np.zeros(max(ev_cap, 1))
            ef, eo = np.zeros(max(ev_cap, 1), np.uint32), np.zeros(max(ev_cap, 1), np.uint32)
            ct, cp, cl = np.zeros(max(co_cap, 1)), np.zeros(max(co_cap, 1)), np.zeros(max(co_cap, 1), np.uint32)
            rc = self._lib.or_event_stream(self._h, seed, _ptr(s, C.c_uint64), n, ev_cap, _ptr(et, C.c_double),
                                           _ptr(ep, C.c_double), _ptr(ef, C.c_uint32), _ptr(eo, C.c_uint32), co_cap,
                                           _ptr(ct, C.c_double), _ptr(cp, C.c_double), _ptr(cl, C.c_uint32),
                                           C.byref(ne), C.byref(nc))
            if rc != 0:
                raise ValueError(f"event_stream failed ({rc})")
            if ne.value <= ev_cap and nc.value <= co_cap:
                break
            ev_cap, co_cap = ne.value, nc.value
        k, m = ne.value, nc.value
        return (dict(t=et[:k], prior=ep[:k], origin=ef[:k], outcome=eo[:k]),
                dict(t=ct[:m], parent=cp[:m], loc=cl[:m]))

    def trace(self, seed: int, sample: int, max_events: int = 1 << 16):
        """Event trace of one sample: (times, locations, dx, dy, speciated)."""
        times = np.zeros(max_events, np.float64)
        locs = np.zeros(max_events, np.uint32)
        dxs = np.zeros(max_events, np.int32)
        dys = np.zeros(max_events, np.int32)
        done = C.c_int()
        n = self._lib.or_trace(self._h, seed, sample, max_events, _ptr(times, C.c_double), _ptr(locs, C.c_uint32),
                               _ptr(dxs, C.c_int32), _ptr(dys, C.c_int32), C.byref(done))
        return times[:n], locs[:n], dxs[:n], dys[:n], bool(done.value)
