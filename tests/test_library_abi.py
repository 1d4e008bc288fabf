"""Host-only checks of the C-ABI library: it loads, exports every symbol the
header declares, and rejects invalid scenarios before touching the GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "necsim_hip.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nh_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def B():
    from paper_2108_05815_amd import binding
    return binding


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("nh_scenario_create", "nh_scenario_destroy", "nh_batch_run", "nh_simulate",
                     "nh_simulate_device", "nh_last_error", "nh_workspace_bytes", "nh_scenario_footprint_bytes"):
        assert required in names


def test_library_exports_every_declared_symbol(B):
    lib = C.CDLL(B.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(B.EXPORTED)
    assert b"gfx950" in B.nh_version()


def test_binding_struct_layouts_match_the_library(B):
    """Every ctypes copy of a public struct has the library's size (a field added on one side only
    shows here, on the CPU), and the event record dtypes are the C records."""
    for cls in (B.nh_habitat, B.nh_dispersal, B.nh_params, B.nh_config, B.nh_stats, B.nh_job, B.nh_stream_out,
                B.nh_server_config, B.nh_completion, B.nh_primitive_io):
        assert B._lib.nh_struct_bytes(cls.__name__.encode()) == C.sizeof(cls), cls.__name__
    assert B._lib.nh_struct_bytes(b"nh_event") == B.EVENT_DTYPE.itemsize
    assert B._lib.nh_struct_bytes(b"nh_coalescence") == B.COALESCENCE_DTYPE.itemsize
    assert B._lib.nh_struct_bytes(b"no_such_struct") == 0


def test_workspace_sizes_grow_with_the_batch(B):
    a = B.workspace_bytes(1000, 1)
    b = B.workspace_bytes(2000, 1)
    c = B.workspace_bytes(2000, 64)
    assert 0 < a < b < c
    assert B.workspace_bytes(0, 1) > 0


@pytest.mark.parametrize("kwargs,msg", [
    (dict(nu=0.0), "nu"),
    (dict(nu=1.5), "nu"),
    (dict(nu=float("nan")), "nu"),
    (dict(dt=3.0), "delta_t"),
    (dict(dt=-1.0), "delta_t"),
    (dict(lam=0.0), "lambda"),
    (dict(lam=float("inf")), "lambda"),
    (dict(lam=4096.0, dt=512.0), "2^20"),
    (dict(tau=-1.0), "tau"),
    (dict(tau=float("nan")), "tau"),
    (dict(tau=float("inf")), "tau"),
    (dict(tau=2.0 ** 58, lam=0.125), "tau"),
])
def test_scenario_parameter_validation(B, kwargs, msg):
    nu = kwargs.pop("nu", 0.1)
    with pytest.raises(B.NecsimError) as e:
        B.Scenario(np.ones((8, 8), np.uint32), np.ones((3, 3)), nu, **kwargs)
    assert e.value.code == B.NH_EINVAL
    assert msg in str(e.value)


def test_scenario_shape_validation(B):
    with pytest.raises(B.NecsimError):
        B.Scenario(np.ones((4, 4), np.uint32), np.ones((5, 5)), 0.1)  # 2R+1 > W
    with pytest.raises(B.NecsimError):
        B.Scenario(np.zeros((4, 4), np.uint32), np.ones((3, 3)), 0.1, mode=1)  # nothing habitable
    cap = np.ones((4, 4), np.uint32)
    cap[1, 2] = 0
    with pytest.raises(B.NecsimError):
        B.Scenario(cap, np.ones((3, 3)), 0.1, mode=0)  # shared table with an empty deme
    w = np.ones((3, 3))
    w[0, 0] = -1.0
    with pytest.raises(B.NecsimError):
        B.Scenario(np.ones((4, 4), np.uint32), w, 0.1)
    with pytest.raises(B.NecsimError):
        B.Scenario(np.ones((4, 4), np.uint32), np.zeros((3, 3)), 0.1)
    big = np.full((1 << 10, 1 << 10), 1 << 12, np.uint32)
    with pytest.raises(B.NecsimError) as e:
        B.Scenario(big, np.ones((1, 1)), 0.1)
    assert "2^32" in str(e.value)


def test_isolated_deme_in_per_deme_mode_is_rejected(B):
    cap = np.zeros((9, 9), np.uint32)
    cap[4, 4] = 3
    w = np.ones((3, 3))
    w[1, 1] = 0.0  # no self-dispersal and no habitable neighbour
    with pytest.raises(B.NecsimError) as e:
        B.Scenario(cap, w, 0.1, mode=1)
    assert "habitable mass" in str(e.value)


def test_resume_rejects_bad_calls_before_touching_the_gpu(B):
    assert B.nh_batch_resume(None, 0, None, 0, None, None, None) == B.NH_EINVAL
    assert B.nh_batch_resume(None, 1, None, 0, None, None, None) == B.NH_EINVAL


def test_event_stream_rejects_bad_calls_before_touching_the_gpu(B):
    from paper_2108_05815_amd import binding as bd
    assert B.nh_event_stream(None, 0, None, 0, None, None) == B.NH_EINVAL
    stand_in = C.create_string_buffer(64)  # a non-NULL scenario handle these checks never read
    jobs = (bd.nh_job * 1)()
    jobs[0].scenario = C.addressof(stand_in)
    jobs[0].seed, jobs[0].n, jobs[0].d_sample_ids, jobs[0].d_species_out = 1, 4, 256, 256
    outs = (bd.nh_stream_out * 1)()
    assert B.nh_event_stream(jobs, 1, None, 0, None, None) == B.NH_EINVAL           # no outputs
    outs[0].events_cap = 8                                                        # room but no buffer
    outs[0].d_coalescences = 256
    assert B.nh_event_stream(jobs, 1, None, 0, outs, None) == B.NH_EINVAL
    outs[0].events_cap, outs[0].d_coalescences = 0, None                          # no coalescence buffer
    assert B.nh_event_stream(jobs, 1, None, 0, outs, None) == B.NH_EINVAL
    outs[0].d_coalescences = 256                                                  # workspace too small
    assert B.nh_event_stream(jobs, 1, None, 0, outs, None) == B.NH_ENOMEM
    assert "workspace" in bd.nh_last_error().decode()


@pytest.mark.parametrize("J,Jm,m,nu", [(0, 10, 0.5, 0.1), (10, 0, 0.5, 0.1), (10, 10, 0.0, 0.1), (10, 10, 1.5, 0.1),
                                       (10, 10, 0.5, 0.0), (10, 10, float("nan"), 0.1)])
def test_implicit_scenario_validation(B, J, Jm, m, nu):
    h = C.c_void_p()
    assert B.nh_scenario_create_implicit(J, Jm, m, nu, None, C.byref(h)) == B.NH_EINVAL


def test_measurement_and_primitive_entry_points_reject_bad_calls_before_touching_the_gpu(B):
    from paper_2108_05815_amd import binding as bd
    x = C.c_double()
    assert B.nh_measure_event_latency(None, 1, 100, C.byref(x), None) == B.NH_EINVAL
    stand_in = C.create_string_buffer(64)  # a non-NULL scenario handle these checks never read
    assert B.nh_measure_event_latency(C.addressof(stand_in), 1, 0, C.byref(x), None) == B.NH_EINVAL
    assert B.nh_eval_primitives(None, 1, 1, None, 0, None) == B.NH_EINVAL
    io = bd.nh_primitive_io()
    io.d_ctr = 256  # an input without its output
    assert B.nh_eval_primitives(C.addressof(stand_in), 1, 1, C.byref(io), 0, None) == B.NH_EINVAL
    io = bd.nh_primitive_io()
    io.d_next_out = 256  # an event output without locations and times
    assert B.nh_eval_primitives(C.addressof(stand_in), 1, 1, C.byref(io), 0, None) == B.NH_EINVAL
    assert "d_loc" in bd.nh_last_error().decode()
