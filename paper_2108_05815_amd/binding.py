"""Thin ctypes binding of libnecsim_hip (include/necsim_hip.h).

Argument marshalling only: every step of the method runs in the HIP library.
Functions keep the C names (nh_scenario_create, nh_batch_run, ...); the
``Scenario`` class and ``simulate`` / ``batch_run`` helpers wrap them for numpy
arrays and PyTorch device tensors (PyTorch provides device memory and streams).

Importing this module loads ``libnecsim_hip.so`` from the package directory
and raises ``ImportError`` if it has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnecsim_hip.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2108_05815_amd/build.py (or __graft_entry__.build())")

_lib = C.CDLL(LIB_PATH)

NH_OK, NH_EINVAL, NH_ENOMEM, NH_EDEVICE, NH_ETIMEOUT = 0, -1, -2, -3, -4
NH_SUSPENDED = 1
NH_DISPERSAL_SHARED, NH_DISPERSAL_PER_DEME = 0, 1


class nh_habitat(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("h_capacity", C.POINTER(C.c_uint32))]


class nh_dispersal(C.Structure):
    _fields_ = [("radius", C.c_uint32), ("h_weights", C.POINTER(C.c_double)), ("mode", C.c_uint32)]


class nh_params(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("delta_t", C.c_double), ("sampler", C.c_uint32),
                ("reserved", C.c_uint32), ("tau", C.c_double)]


class nh_config(C.Structure):
    _fields_ = [("horizon0", C.c_double), ("horizon_growth", C.c_double), ("horizon_step_max", C.c_double),
                ("block_size", C.c_uint32), ("blocks_per_cu", C.c_uint32), ("rounds_per_graph", C.c_uint32),
                ("event_timing", C.c_uint32), ("coop_max", C.c_uint32), ("table_placement", C.c_uint32),
                ("timeout_s", C.c_double), ("solo_max", C.c_uint32), ("launch", C.c_uint32),
                ("solo_step", C.c_double), ("max_rounds", C.c_uint32), ("barrier_wait_ms", C.c_uint32),
                ("endgame", C.c_uint32)]


class nh_stats(C.Structure):
    _fields_ = [("events", C.c_uint64), ("lineages", C.c_uint64), ("speciated", C.c_uint64),
                ("merged", C.c_uint64), ("rounds", C.c_uint64), ("richness", C.c_uint64),
                ("device_ms", C.c_double), ("philox_calls", C.c_uint64), ("exp_draws", C.c_uint64),
                ("round_kernels", C.c_uint64), ("round_kernel_ms", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class nh_job(C.Structure):
    _fields_ = [("scenario", C.c_void_p), ("seed", C.c_uint64), ("d_sample_ids", C.c_void_p), ("n", C.c_uint64),
                ("d_species_out", C.c_void_p), ("d_richness_out", C.c_void_p), ("d_spec_loc_out", C.c_void_p),
                ("d_spec_time_out", C.c_void_p), ("d_abundance_ids_out", C.c_void_p),
                ("d_abundance_counts_out", C.c_void_p)]


class nh_stream_out(C.Structure):
    _fields_ = [("d_events", C.c_void_p), ("events_cap", C.c_uint64), ("d_coalescences", C.c_void_p),
                ("n_events", C.c_uint64), ("n_coalescences", C.c_uint64)]


# nh_event and nh_coalescence records as numpy dtypes (24 bytes each)
EVENT_DTYPE = np.dtype([("t", "<f8"), ("t_prior", "<f8"), ("origin", "<u4"), ("outcome", "<u4")])
COALESCENCE_DTYPE = np.dtype([("t", "<f8"), ("t_parent", "<f8"), ("loc", "<u4"), ("reserved", "<u4")])
NH_EVENT_SPECIATION = 0xFFFFFFFF
NH_LAUNCH_PERSISTENT, NH_LAUNCH_GRAPHS = 0, 1


class nh_primitive_io(C.Structure):
    _fields_ = [("d_ctr", C.c_void_p), ("d_philox_out", C.c_void_p), ("d_r", C.c_void_p), ("d_log_out", C.c_void_p),
                ("d_loc", C.c_void_p), ("d_t", C.c_void_p), ("d_next_out", C.c_void_p),
                ("d_next_group_out", C.c_void_p), ("d_outcome_out", C.c_void_p), ("d_step_loc_out", C.c_void_p),
                ("d_step_t_out", C.c_void_p)]


class nh_server_config(C.Structure):
    _fields_ = [("lineage_capacity", C.c_uint64), ("max_jobs", C.c_uint32), ("lookahead", C.c_uint32),
                ("cfg", nh_config), ("tail_blocks", C.c_uint32)]


class nh_completion(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("status", C.c_int), ("rounds", C.c_uint32), ("richness", C.c_uint64),
                ("events", C.c_uint64), ("lineages", C.c_uint64), ("speciated", C.c_uint64), ("merged", C.c_uint64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib.nh_scenario_create.argtypes = [C.POINTER(nh_habitat), C.POINTER(nh_dispersal), C.c_double,
                                    C.POINTER(nh_params), C.POINTER(C.c_void_p)]
_lib.nh_scenario_create.restype = C.c_int
_lib.nh_scenario_create_implicit.argtypes = [C.c_uint32, C.c_uint32, C.c_double, C.c_double, C.POINTER(nh_params),
                                             C.POINTER(C.c_void_p)]
_lib.nh_scenario_create_implicit.restype = C.c_int
_lib.nh_scenario_destroy.argtypes = [C.c_void_p]
_lib.nh_scenario_destroy.restype = None
_lib.nh_scenario_individuals.argtypes = [C.c_void_p]
_lib.nh_scenario_individuals.restype = C.c_uint64
_lib.nh_scenario_table_bytes.argtypes = [C.c_void_p]
_lib.nh_scenario_table_bytes.restype = C.c_uint64
_lib.nh_workspace_bytes.argtypes = [C.c_uint64, C.c_uint32]
_lib.nh_workspace_bytes.restype = C.c_uint64
_lib.nh_scenario_footprint_bytes.argtypes = [C.c_void_p, C.c_uint64]
_lib.nh_scenario_footprint_bytes.restype = C.c_uint64
_lib.nh_batch_run.argtypes = [C.POINTER(nh_job), C.c_uint32, C.c_void_p, C.c_uint64, C.POINTER(nh_config),
                              C.POINTER(nh_stats), C.c_void_p]
_lib.nh_batch_run.restype = C.c_int
_lib.nh_batch_resume.argtypes = _lib.nh_batch_run.argtypes
_lib.nh_batch_resume.restype = C.c_int
_lib.nh_event_stream.argtypes = [C.POINTER(nh_job), C.c_uint32, C.c_void_p, C.c_uint64, C.POINTER(nh_stream_out),
                                 C.c_void_p]
_lib.nh_event_stream.restype = C.c_int
_lib.nh_struct_bytes.argtypes = [C.c_char_p]
_lib.nh_struct_bytes.restype = C.c_uint64
_lib.nh_measure_event_latency.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.POINTER(C.c_double), C.c_void_p]
_lib.nh_measure_event_latency.restype = C.c_int
_lib.nh_eval_primitives.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.POINTER(nh_primitive_io), C.c_uint32,
                                    C.c_void_p]
_lib.nh_eval_primitives.restype = C.c_int
_lib.nh_simulate_device.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p,
                                    C.POINTER(nh_config), C.POINTER(nh_stats), C.c_void_p]
_lib.nh_simulate_device.restype = C.c_int
_lib.nh_simulate_async.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p,
                                   C.POINTER(nh_config), C.c_void_p]
_lib.nh_simulate_async.restype = C.c_int
_lib.nh_simulate_noalloc.argtypes = _lib.nh_simulate_async.argtypes
_lib.nh_simulate_noalloc.restype = C.c_int
_lib.nh_simulate.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_uint64), C.c_uint64, C.POINTER(C.c_uint64),
                             C.POINTER(C.c_uint64), C.POINTER(nh_stats)]
_lib.nh_simulate.restype = C.c_int
_lib.nh_server_bytes.argtypes = [C.c_uint64, C.c_uint32]
_lib.nh_server_bytes.restype = C.c_uint64
_lib.nh_server_create.argtypes = [C.POINTER(nh_server_config), C.c_void_p, C.POINTER(C.c_void_p)]
_lib.nh_server_create.restype = C.c_int
_lib.nh_server_submit.argtypes = [C.c_void_p, C.POINTER(nh_job), C.c_uint64]
_lib.nh_server_submit.restype = C.c_int
_lib.nh_server_progress.argtypes = [C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
_lib.nh_server_progress.restype = C.c_int
_lib.nh_server_poll.argtypes = [C.c_void_p, C.POINTER(nh_completion), C.c_uint32, C.POINTER(C.c_uint32)]
_lib.nh_server_poll.restype = C.c_int
_lib.nh_server_drain.argtypes = [C.c_void_p, C.c_double]
_lib.nh_server_drain.restype = C.c_int
_lib.nh_server_destroy.argtypes = [C.c_void_p]
_lib.nh_server_destroy.restype = None
_lib.nh_last_error.argtypes = []
_lib.nh_last_error.restype = C.c_char_p
_lib.nh_version.argtypes = []
_lib.nh_version.restype = C.c_char_p
_lib.nh_measure_mix_peak.argtypes = [C.POINTER(C.c_double), C.c_void_p]
_lib.nh_measure_mix_peak.restype = C.c_int
_lib.nh_measure_gather.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_double), C.c_void_p]
_lib.nh_measure_gather.restype = C.c_int

# The C names, for callers that want the raw ABI.
nh_scenario_create = _lib.nh_scenario_create
nh_scenario_destroy = _lib.nh_scenario_destroy
nh_scenario_create_implicit = _lib.nh_scenario_create_implicit
nh_scenario_individuals = _lib.nh_scenario_individuals
nh_scenario_table_bytes = _lib.nh_scenario_table_bytes
nh_workspace_bytes = _lib.nh_workspace_bytes
nh_scenario_footprint_bytes = _lib.nh_scenario_footprint_bytes
nh_batch_run = _lib.nh_batch_run
nh_batch_resume = _lib.nh_batch_resume
nh_event_stream = _lib.nh_event_stream
nh_simulate_device = _lib.nh_simulate_device
nh_simulate = _lib.nh_simulate
nh_simulate_async = _lib.nh_simulate_async
nh_simulate_noalloc = _lib.nh_simulate_noalloc
nh_last_error = _lib.nh_last_error
nh_version = _lib.nh_version
nh_measure_mix_peak = _lib.nh_measure_mix_peak
nh_measure_gather = _lib.nh_measure_gather
nh_measure_event_latency = _lib.nh_measure_event_latency
nh_eval_primitives = _lib.nh_eval_primitives
nh_server_bytes = _lib.nh_server_bytes
nh_server_create = _lib.nh_server_create
nh_server_submit = _lib.nh_server_submit
nh_server_progress = _lib.nh_server_progress
nh_server_poll = _lib.nh_server_poll
nh_server_drain = _lib.nh_server_drain
nh_server_destroy = _lib.nh_server_destroy

EXPORTED = ["nh_scenario_create", "nh_scenario_create_implicit", "nh_scenario_destroy", "nh_scenario_individuals", "nh_scenario_table_bytes",
            "nh_workspace_bytes", "nh_scenario_footprint_bytes", "nh_batch_run", "nh_batch_resume", "nh_event_stream",
            "nh_simulate_device", "nh_simulate_async", "nh_simulate_noalloc",
            "nh_simulate", "nh_last_error", "nh_version", "nh_server_bytes", "nh_server_create",
            "nh_server_submit", "nh_server_progress", "nh_server_poll", "nh_server_drain", "nh_server_destroy",
            "nh_measure_mix_peak", "nh_measure_gather", "nh_measure_event_latency", "nh_eval_primitives",
            "nh_struct_bytes"]


class NecsimError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where} failed ({code}): {_lib.nh_last_error().decode()}")


def _check(code: int, where: str):
    if code != NH_OK:
        raise NecsimError(code, where)


def make_config(**kw) -> nh_config:
    c = nh_config()
    for k, v in kw.items():
        if v is not None:
            setattr(c, k, v)
    return c


class Scenario:
    """Device-resident scenario tables (nh_scenario_create)."""

    def __init__(self, capacity, weights, nu: float, *, mode: int = NH_DISPERSAL_SHARED, lam: float = 1.0,
                 dt: float = 1.0, sampler: int = 0, tau: float = 0.0):
        """tau > 0: protracted speciation (speciation draws at events fewer than tau generations,
        lambda * t < tau, before the present are ignored and those events disperse)."""
        cap = np.ascontiguousarray(capacity, dtype=np.uint32)
        if cap.ndim != 2:
            raise ValueError("capacity must be a 2-D (H, W) array")
        w = np.ascontiguousarray(weights, dtype=np.float64)
        if w.ndim != 2 or w.shape[0] != w.shape[1] or w.shape[0] % 2 != 1:
            raise ValueError("weights must be a square (2R+1, 2R+1) array")
        hab = nh_habitat(cap.shape[1], cap.shape[0], cap.ctypes.data_as(C.POINTER(C.c_uint32)))
        disp = nh_dispersal(w.shape[0] // 2, w.ctypes.data_as(C.POINTER(C.c_double)), mode)
        par = nh_params(lam, dt, sampler, 0, tau)
        h = C.c_void_p()
        _check(_lib.nh_scenario_create(C.byref(hab), C.byref(disp), nu, C.byref(par), C.byref(h)),
               "nh_scenario_create")
        self._h = h
        self.nu, self.mode, self.lam, self.dt, self.sampler, self.tau = nu, mode, lam, dt, sampler, tau
        self.shape = cap.shape

    @classmethod
    def implicit(cls, J: int, J_meta: int, m: float, nu_meta: float, *, lam: float = 1.0, dt: float = 1.0,
                 sampler: int = 0, tau: float = 0.0):
        """nh_scenario_create_implicit: local community J (sample ids 0..J-1) with migration
        probability m into a dynamic metacommunity of J_meta with speciation nu_meta."""
        self = cls.__new__(cls)
        h = C.c_void_p()
        par = nh_params(lam, dt, sampler, 0, tau)
        _check(_lib.nh_scenario_create_implicit(J, J_meta, m, nu_meta, C.byref(par), C.byref(h)),
               "nh_scenario_create_implicit")
        self._h = h
        self.nu, self.mode, self.lam, self.dt, self.sampler, self.tau = nu_meta, 2, lam, dt, sampler, tau
        self.shape = (1, 2)
        return self

    @classmethod
    def from_workload(cls, wl):
        return cls(wl.capacity, wl.weights, wl.nu, mode=wl.mode, lam=wl.lam, dt=wl.dt,
                   sampler=getattr(wl, "sampler", 0), tau=getattr(wl, "tau", 0.0))

    @property
    def handle(self):
        return self._h

    @property
    def individuals(self) -> int:
        return int(_lib.nh_scenario_individuals(self._h))

    @property
    def table_bytes(self) -> int:
        return int(_lib.nh_scenario_table_bytes(self._h))

    def footprint_bytes(self, n_samples: int) -> int:
        return int(_lib.nh_scenario_footprint_bytes(self._h, n_samples))

    def close(self):
        if getattr(self, "_h", None):
            _lib.nh_scenario_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def simulate(scenario: Scenario, seed: int, samples) -> tuple[np.ndarray, int, dict]:
    """Host-buffer simulate (nh_simulate): returns (species u64[n], richness, stats)."""
    s = np.ascontiguousarray(samples, dtype=np.uint64)
    out = np.zeros(len(s), dtype=np.uint64)
    rich = C.c_uint64()
    st = nh_stats()
    _check(_lib.nh_simulate(scenario.handle, seed, s.ctypes.data_as(C.POINTER(C.c_uint64)), len(s),
                            out.ctypes.data_as(C.POINTER(C.c_uint64)), C.byref(rich), C.byref(st)), "nh_simulate")
    return out, int(rich.value), st.as_dict()


def simulate_async(scenario: Scenario, seed: int, samples, out, rich=None, config: nh_config | None = None,
                   stream=None) -> None:
    """nh_simulate_async: enqueue one whole run on `stream` (torch.cuda.Stream or None for the current
    one) and return at once.  samples: u64/int64 device tensor; out: int64 device tensor of the same
    length; rich: one-element int64 device tensor or None (it reads -1, i.e. ~0, if the run failed
    on the device).  Synchronise the stream before reading them."""
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    n = samples.numel()
    _check(_lib.nh_simulate_async(scenario.handle, int(seed) & (2**64 - 1), samples.data_ptr() if n else None, n,
                                  out.data_ptr() if out.numel() else None,
                                  rich.data_ptr() if rich is not None else None,
                                  C.byref(config) if config is not None else None, C.c_void_p(s.cuda_stream)),
           "nh_simulate_async")


def simulate_noalloc(scenario: Scenario, seed: int, samples, out, rich=None, config: nh_config | None = None,
                     stream=None) -> None:
    """nh_simulate_noalloc: as simulate_async, with the library's fixed device scratch as the
    workspace (no allocation; at most about 480,000 samples)."""
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    n = samples.numel()
    _check(_lib.nh_simulate_noalloc(scenario.handle, int(seed) & (2**64 - 1), samples.data_ptr() if n else None, n,
                                    out.data_ptr() if out.numel() else None,
                                    rich.data_ptr() if rich is not None else None,
                                    C.byref(config) if config is not None else None, C.c_void_p(s.cuda_stream)),
           "nh_simulate_noalloc")


def workspace_bytes(n_total: int, n_jobs: int) -> int:
    return int(_lib.nh_workspace_bytes(n_total, n_jobs))


def _job(scn, seed, samples, out, rich, reporters=None) -> nh_job:
    """reporters (optional dict of device tensors with one slot per sample): spec_loc (int32),
    spec_time (float64): the speciation event behind each sample's species; abundance_ids (int64),
    abundance_counts (int32): one (species, samples) pair per species, richness of them written."""
    j = nh_job()
    j.scenario = scn.handle
    j.seed = int(seed) & (2**64 - 1)
    j.d_sample_ids = samples.data_ptr() if samples.numel() else None
    j.n = samples.numel()
    j.d_species_out = out.data_ptr() if out.numel() else None
    j.d_richness_out = rich.data_ptr() if rich is not None else None
    r = reporters or {}
    for field, key in (("d_spec_loc_out", "spec_loc"), ("d_spec_time_out", "spec_time"),
                       ("d_abundance_ids_out", "abundance_ids"), ("d_abundance_counts_out", "abundance_counts")):
        t = r.get(key)
        if t is not None:
            if t.numel() < samples.numel():
                raise ValueError(f"reporter {key} needs {samples.numel()} slots")
            setattr(j, field, t.data_ptr() if t.numel() else None)
    return j


def server_bytes(lineage_capacity: int, max_jobs: int) -> int:
    return int(_lib.nh_server_bytes(lineage_capacity, max_jobs))


class Server:
    """Continuous-batching engine (nh_server_*): a resident lineage pool in HBM that admits jobs
    while others run.  Keeps each job's tensors and scenario alive until its completion is polled."""

    def __init__(self, lineage_capacity: int, max_jobs: int = 1024, lookahead: int = 16,
                 config: nh_config | None = None, stream=None, tail_blocks: int = 0):
        cfg = nh_server_config()
        cfg.lineage_capacity = lineage_capacity
        cfg.max_jobs = max_jobs
        cfg.lookahead = lookahead
        cfg.tail_blocks = tail_blocks
        if config is not None:
            cfg.cfg = config
        h = C.c_void_p()
        st = C.c_void_p(stream.cuda_stream) if stream is not None else None
        _check(_lib.nh_server_create(C.byref(cfg), st, C.byref(h)), "nh_server_create")
        self._h = h
        self._held = {}
        self._buf = (nh_completion * 512)()

    def submit(self, tag: int, scenario: Scenario, seed: int, samples, out, rich=None, keep=None, reporters=None):
        j = _job(scenario, seed, samples, out, rich, reporters)
        _check(_lib.nh_server_submit(self._h, C.byref(j), tag), "nh_server_submit")
        self._held[tag] = (scenario, samples, out, rich, keep, reporters)

    def progress(self) -> tuple[int, int]:
        a, p = C.c_uint32(), C.c_uint32()
        _check(_lib.nh_server_progress(self._h, C.byref(a), C.byref(p)), "nh_server_progress")
        return a.value, p.value

    def poll(self) -> list:
        out = []
        while True:
            n = C.c_uint32()
            _check(_lib.nh_server_poll(self._h, self._buf, len(self._buf), C.byref(n)), "nh_server_poll")
            for k in range(n.value):
                d = self._buf[k].as_dict()
                d["held"] = self._held.pop(d["tag"], None)
                out.append(d)
            if n.value < len(self._buf):
                return out

    def drain(self, timeout_s: float = 600.0):
        _check(_lib.nh_server_drain(self._h, timeout_s), "nh_server_drain")

    def close(self):
        if getattr(self, "_h", None):
            _lib.nh_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _batch(fn, name, jobs, workspace, config, stream):
    import torch

    arr = (nh_job * len(jobs))()
    for k, job in enumerate(jobs):
        arr[k] = _job(*job)
    st = (nh_stats * len(jobs))()
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = fn(arr, len(jobs), workspace.data_ptr(), workspace.numel(), C.byref(config) if config is not None else None,
            st, C.c_void_p(s.cuda_stream))
    if rc != NH_SUSPENDED:
        _check(rc, name)
    return [dict(x.as_dict(), suspended=rc == NH_SUSPENDED) for x in st]


def batch_run(jobs, workspace, config: nh_config | None = None, stream=None):
    """nh_batch_run over device buffers.

    jobs: list of (Scenario, seed, samples_tensor u64/int64 on the device, species_out tensor,
    richness_out tensor or None[, reporters dict as for _job]).  workspace: a uint8 device tensor of at least
    workspace_bytes(sum n, len(jobs)) bytes.  stream: a torch.cuda.Stream or None (current stream).
    Returns the list of per-job stats dicts; each has suspended=True if config.max_rounds stopped
    the run (continue it with batch_resume)."""
    return _batch(_lib.nh_batch_run, "nh_batch_run", jobs, workspace, config, stream)


def batch_resume(jobs, workspace, config: nh_config | None = None, stream=None):
    """nh_batch_resume: continue a suspended run from the state in `workspace` (the same jobs)."""
    return _batch(_lib.nh_batch_resume, "nh_batch_resume", jobs, workspace, config, stream)


def event_stream_device(jobs, workspace, events, coalescences, stream=None):
    """nh_event_stream into device buffers: events[k] and coalescences[k] are uint8 device tensors
    (or None for events, to count only) of whole EVENT_DTYPE / COALESCENCE_DTYPE records, the
    latter with room for job k's samples.  Returns [(n_events, n_coalescences)] per job."""
    import torch

    arr = (nh_job * len(jobs))()
    for k, job in enumerate(jobs):
        arr[k] = _job(*job)
    outs = (nh_stream_out * len(jobs))()
    for k in range(len(jobs)):
        ev = events[k]
        cap = 0 if ev is None else ev.numel() // EVENT_DTYPE.itemsize
        outs[k] = nh_stream_out(None if ev is None else ev.data_ptr(), cap, coalescences[k].data_ptr(), 0, 0)
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(_lib.nh_event_stream(arr, len(jobs), workspace.data_ptr(), workspace.numel(), outs,
                                C.c_void_p(s.cuda_stream)), "nh_event_stream")
    return [(int(o.n_events), int(o.n_coalescences)) for o in outs]


def event_stream(jobs, workspace, events_cap=None, stream=None):
    """nh_event_stream for the jobs of the batch run that just finished in `workspace` (the same job
    tuples as given to batch_run).  events_cap: records of room per job (a list, or one int for all);
    None counts first and then makes room for every event.  Returns per job a dict with the events
    and coalescences as numpy arrays of EVENT_DTYPE and COALESCENCE_DTYPE and the total counts
    (n_events may exceed the room given)."""
    import torch

    dev = workspace.device
    co = [torch.empty(max(int(job[2].numel()), 1) * COALESCENCE_DTYPE.itemsize, dtype=torch.uint8, device=dev)
          for job in jobs]
    if events_cap is None:
        counts = event_stream_device(jobs, workspace, [None] * len(jobs), co, stream)
        events_cap = [c[0] for c in counts]
    if isinstance(events_cap, int):
        events_cap = [events_cap] * len(jobs)
    ev = [torch.empty(max(cap, 1) * EVENT_DTYPE.itemsize, dtype=torch.uint8, device=dev)[:cap * EVENT_DTYPE.itemsize]
          for cap in events_cap]
    counts = event_stream_device(jobs, workspace, ev, co, stream)
    res = []
    for k, (ne, nc) in enumerate(counts):
        e = ev[k].cpu().numpy().view(EVENT_DTYPE)[:min(ne, events_cap[k])]
        c = co[k].cpu().numpy().view(COALESCENCE_DTYPE)[:nc]
        res.append(dict(events=e, coalescences=c, n_events=ne, n_coalescences=nc))
    return res


def measure_mix_peak(stream=None) -> float:
    """Algorithmic lane-ops/s the chip sustains for the event path's Philox + log mix."""
    import torch
    x = C.c_double()
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(_lib.nh_measure_mix_peak(C.byref(x), C.c_void_p(s.cuda_stream)), "nh_measure_mix_peak")
    return x.value


def measure_event_latency(scn, seed: int = 1, steps: int = 20000, stream=None) -> float:
    """Nanoseconds per event of one lineage walking alone (nh_measure_event_latency)."""
    import torch
    x = C.c_double()
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(_lib.nh_measure_event_latency(scn.handle, seed, steps, C.byref(x), C.c_void_p(s.cuda_stream)),
           "nh_measure_event_latency")
    return x.value


def eval_primitives(scn, seed: int, ctr=None, r=None, loc=None, t=None, use_lds: bool = True, stream=None) -> dict:
    """nh_eval_primitives on host arrays (copied to the device and back): Philox blocks of ctr
    (n x 4 u32), logarithms of the draws r (u64), and for the (loc, t) pairs the one-lane and group
    next event times, the event outcomes and one group step each."""
    import torch
    dev = torch.device("cuda:0")
    s = stream if stream is not None else torch.cuda.current_stream()
    io = nh_primitive_io()
    keep, out = [], {}

    def put(a, dtype):
        x = torch.from_numpy(np.ascontiguousarray(a).view(dtype)).to(dev)
        keep.append(x)
        return x.data_ptr()

    def make(name, count, dtype):
        x = torch.empty(max(count, 1), dtype=dtype, device=dev)
        out[name] = x
        return x.data_ptr()

    n = 0
    if ctr is not None:
        c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
        n = max(n, len(c))
        io.d_ctr, io.d_philox_out = put(c.reshape(-1).view(np.int32), np.int32), make("philox", 4 * len(c), torch.int32)
    if r is not None:
        rr = np.ascontiguousarray(r, dtype=np.uint64)
        n = max(n, len(rr))
        io.d_r, io.d_log_out = put(rr.view(np.int64), np.int64), make("log", len(rr), torch.float64)
    if loc is not None:
        l = np.ascontiguousarray(loc, dtype=np.uint32)
        n = max(n, len(l))
        io.d_loc, io.d_t = put(l.view(np.int32), np.int32), put(np.ascontiguousarray(t, dtype=np.float64), np.float64)
        io.d_next_out = make("next", len(l), torch.float64)
        io.d_next_group_out = make("next_group", len(l), torch.float64)
        io.d_outcome_out = make("outcome", len(l), torch.int32)
        io.d_step_loc_out = make("step_loc", len(l), torch.int32)
        io.d_step_t_out = make("step_t", len(l), torch.float64)
    lens = [len(x) for x in (ctr if ctr is None else np.asarray(ctr).reshape(-1, 4), r, loc) if x is not None]
    if len(set(lens)) > 1:
        raise ValueError("ctr, r and loc must have the same number of items")
    _check(_lib.nh_eval_primitives(scn.handle, seed, n, C.byref(io), int(use_lds), C.c_void_p(s.cuda_stream)),
           "nh_eval_primitives")
    res = {}
    for name, x in out.items():
        a = x.cpu().numpy()
        if name in ("philox", "outcome", "step_loc"):
            a = a.view(np.uint32)
        res[name] = a.reshape(-1, 4)[:n] if name == "philox" else a[:n]
    return res


def measure_gather(table, stream=None) -> float:
    """Useful bytes/s of random 16-byte gathers from a device tensor `table`."""
    import torch
    x = C.c_double()
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(_lib.nh_measure_gather(table.data_ptr(), table.numel() * table.element_size(), C.byref(x),
                                  C.c_void_p(s.cuda_stream)), "nh_measure_gather")
    return x.value
