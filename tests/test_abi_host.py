"""C ABI on the host: the library loads, exports every declared symbol, validates
its arguments and derives shapes / baselines without a device."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_0909_0001_amd as omni
import skysim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "omniscope.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(omni_\w+)\s*\(", src, re.M)))


def test_header_declarations_match_binding_list():
    assert declared_symbols() == sorted(omni.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(omni.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_strerror_covers_codes():
    for code, name in omni.STATUS.items():
        assert omni.strerror(code) and omni.strerror(code) != "unknown status"
    assert omni.strerror(-99) == "unknown status"


def test_host_only_shapes():
    p = omni.Plan([[8, 8], [8, 8]], None, 64, "ci8", host_only=True)
    assert p.vis_shape() == (64, 15, 15, 15, 15)
    assert p.accumulator_bytes() == 64 * 16**4 * 8
    p = omni.Plan([[5, 1], [1, 3]], None, 2, host_only=True)
    assert p.vis_shape() == (2, 9, 1, 1, 5)


def test_host_only_baselines_match_oracle():
    w = skysim.WORKLOADS["hier8x8"]
    level_dims = [[3, 4], [2, 5]]
    p = omni.Plan(level_dims, w.A, 1, host_only=True)
    assert np.allclose(p.baselines(), oracle.baselines(level_dims, w.A), atol=1e-12)


def test_describe_is_json():
    import json

    p = omni.Plan([[16, 16]], None, 1, host_only=True)
    d = json.loads(p.describe())
    assert d["arrays"][0]["M"] == 1024


@pytest.mark.parametrize(
    "kwargs, code",
    [
        (dict(level_dims=np.zeros((0, 2)), nchan=1), "OMNI_E_SHAPE"),
        (dict(level_dims=[[0, 4]], nchan=1), "OMNI_E_SHAPE"),
        (dict(level_dims=[[4, 4]], nchan=0), "OMNI_E_INVAL"),
        (dict(level_dims=[[2, 2]] * 5, nchan=1), "OMNI_E_SHAPE"),
        (dict(level_dims=[[2048, 4096]], nchan=1), "OMNI_E_SHAPE"),
        (dict(level_dims=[[4, 4]], A=[[np.nan, 0], [0, 1]], nchan=1), "OMNI_E_GEOM"),
        # a_1 = 2 a_2 with i_2 in 0..2 makes grid points collide (Sec. II.D uniqueness)
        (dict(level_dims=[[2, 1], [3, 1]], A=[[[2, 0], [0, 1]], [[1, 0], [0, 1]]], nchan=1), "OMNI_E_GEOM"),
        (dict(level_dims=[[4, 4]], nchan=1, time_block=-1), "OMNI_E_INVAL"),
    ],
)
def test_plan_validation(kwargs, code):
    with pytest.raises(omni.OmniError) as ei:
        omni.Plan(host_only=True, **kwargs)
    assert omni.STATUS[ei.value.code] == code


def test_interleaved_grid_is_accepted():
    # a_1 = (5,0), a_2 = (7,0), i in 0..3: no collisions (Sec. II.D example)
    p = omni.Plan([[4, 1], [4, 1]], [[[7, 0], [0, 1]], [[5, 0], [0, 1]]], 1, host_only=True)
    assert p.vis_shape() == (1, 7, 1, 7, 1)


def test_host_only_plan_refuses_device_calls():
    p = omni.Plan([[4, 4]], None, 1, host_only=True)
    with pytest.raises(omni.OmniError) as ei:
        p.correlate_into(0, 0, 0, stream=0)
    assert omni.STATUS[ei.value.code] == "OMNI_E_STATE"


def test_null_arguments():
    assert omni.lib.omni_plan(None, 1, None, None, 1, None) == -1
    assert omni.lib.omni_destroy(None) == 0
    assert omni.lib.omni_correlate(None, None, 0, None, None, 0) == -1


def test_no_device_is_reported():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(omni.OmniError) as ei:
        omni.Plan([[4, 4]], None, 1)
    assert omni.STATUS[ei.value.code] == "OMNI_E_NODEV"


def test_unsupported_shapes_are_refused_not_crashed():
    # an odd axis length above 32 cannot be split into short DFTs of length <= 32
    with pytest.raises(omni.OmniError) as ei:
        omni.Plan([[33, 2]], None, 1, host_only=True)
    assert omni.STATUS[ei.value.code] == "OMNI_E_SHAPE"


def test_plan_flags_are_validated():
    """Unknown plan flags are refused; the graph flag is accepted on a host-only plan."""
    opts = omni._Opts(omni.DTYPES["ci8"], omni.FORMS["fp32"], 0, omni.PLAN_HOST_ONLY | 0x20)
    h = ctypes.c_void_p()
    dims = np.array([[4, 4]], dtype=np.int32)
    rc = omni.lib.omni_plan(ctypes.byref(h), 1, dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), None, 1,
                            ctypes.byref(opts))
    assert omni.STATUS[rc] == "OMNI_E_INVAL"
    p = omni.Plan([[4, 4]], None, 1, "ci8", host_only=True, graph=True)
    assert p.vis_shape() == (1, 7, 7)


def test_stage_times_need_a_timing_plan():
    p = omni.Plan([[4, 4]], None, 1, host_only=True)
    with pytest.raises(omni.OmniError) as ei:
        p.stage_times("call")
    assert omni.STATUS[ei.value.code] == "OMNI_E_STATE"


def test_tune_and_chunk_options_are_validated():
    """An unknown tune mode or a negative chunk cap is refused by the C ABI."""
    dims = np.array([[4, 4]], dtype=np.int32)
    h = ctypes.c_void_p()
    for tune, chunk in ((3, 0), (-1, 0), (0, -5)):
        opts = omni._Opts(omni.DTYPES["ci8"], omni.FORMS["fp32"], 0, omni.PLAN_HOST_ONLY, tune, None, chunk)
        rc = omni.lib.omni_plan(ctypes.byref(h), 1, dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), None, 1,
                                ctypes.byref(opts))
        assert omni.STATUS[rc] == "OMNI_E_INVAL", (tune, chunk)
    with pytest.raises(ValueError):
        omni.Plan([[4, 4]], None, 1, "ci8", host_only=True, tune="sometimes")


@pytest.mark.parametrize("form", ["fp32", "mixed"])
def test_chunk_cap_sets_front_chunk(form):
    """The chunk_T option caps the front passes' time chunk (a grid that needs front passes)."""
    import json

    ld = [[2, 16], [16, 16]]
    free = json.loads(omni.Plan(ld, None, 2, "ci4", form, host_only=True).describe())["arrays"][0]
    assert free["mode"] == "front" and free["chunk_T"] == 256
    capped = json.loads(omni.Plan(ld, None, 2, "ci4", form, host_only=True, chunk_T=7).describe())["arrays"][0]
    assert capped["chunk_T"] == 7


def _host_plan(dtype, level_dims=((4, 4),), F=3, batch=None):
    if batch is not None:
        return omni.Plan(batch=batch, dtype=dtype, host_only=True)
    return omni.Plan([list(ld) for ld in level_dims], None, F, dtype, host_only=True)


@pytest.mark.parametrize(
    "dtype, make, match",
    [
        ("ci8", lambda: np.zeros((2, 3, 16, 2), np.int8), "torch tensor"),
        ("ci8", lambda: __import__("torch").zeros((2, 3, 16, 2), dtype=__import__("torch").int16), "int8"),
        ("ci8", lambda: __import__("torch").zeros((2, 3, 16), dtype=__import__("torch").int8), "shape"),
        ("ci8", lambda: __import__("torch").zeros((2, 3, 15, 2), dtype=__import__("torch").int8), "shape"),
        ("ci8", lambda: __import__("torch").zeros((2, 2, 16, 2), dtype=__import__("torch").int8), "shape"),
        ("ci4", lambda: __import__("torch").zeros((2, 3, 16, 2), dtype=__import__("torch").uint8), "shape"),
        ("ci4", lambda: __import__("torch").zeros((2, 3, 16), dtype=__import__("torch").float32), "uint8"),
        ("cf32", lambda: __import__("torch").zeros((2, 3, 16), dtype=__import__("torch").float32), "shape"),
        ("cf32", lambda: __import__("torch").zeros((2, 3, 16, 2), dtype=__import__("torch").float64), "float32"),
        ("ci8", lambda: __import__("torch").zeros((2, 3, 2, 16), dtype=__import__("torch").int8).transpose(2, 3),
         "contiguous"),
        ("ci8", lambda: __import__("torch").zeros((2, 3, 16, 2), dtype=__import__("torch").int8), "on the GPU"),
    ],
)
def test_binding_rejects_bad_voltages_before_any_device_call(dtype, make, match):
    """A mis-typed, mis-shaped, strided or host-resident voltage tensor raises ValueError in the binding; the
    library is never reached (a host-only plan would answer OMNI_E_STATE)."""
    p = _host_plan(dtype)
    with pytest.raises(ValueError, match=match):
        p.correlate(make())
    if dtype != "cf32":
        with pytest.raises(ValueError, match=match):
            p.direct_correlate(make())


def test_binding_rejects_bad_outputs_and_batches():
    import torch

    p = _host_plan("ci8")
    good_shape = p.vis_shape()
    volt = torch.zeros((2, 3, 16, 2), dtype=torch.int8)
    for bad, match in (
        (torch.zeros(good_shape, dtype=torch.complex128), "complex64"),
        (torch.zeros((3, 7, 8), dtype=torch.complex64), "shape"),
        (torch.zeros(good_shape[::-1], dtype=torch.complex64).permute(2, 1, 0), "contiguous"),
        (torch.zeros(good_shape, dtype=torch.complex64), "on the GPU"),
    ):
        with pytest.raises(ValueError, match=match):
            p._check_out(bad, 0, None)
    with pytest.raises(ValueError, match="batch plan"):
        _host_plan("ci8", batch=[([[4, 4]], None, 3), ([[2, 2]], None, 1)]).correlate(volt)
    bp = _host_plan("ci8", batch=[([[4, 4]], None, 3), ([[2, 2]], None, 1)])
    with pytest.raises(ValueError, match="expected 2 voltage tensors"):
        bp.correlate_batch([volt])
    with pytest.raises(ValueError, match="same number of samples"):
        bp.correlate_batch([volt, torch.zeros((5, 1, 4, 2), dtype=torch.int8)])
    with pytest.raises(ValueError, match="shape"):
        bp.correlate_batch([volt, torch.zeros((2, 3, 16, 2), dtype=torch.int8)])
    with pytest.raises(ValueError, match="accumulator buffer"):
        p.accumulator_get(np.zeros(3))


def test_fold_plan_validates_before_any_device_call():
    """The fold entry points refuse bad arguments, planless or A-less plans and host-only plans
    without touching a device."""
    ld, A = skysim.PAPER_LAYOUTS["Blocks"]
    p = omni.Plan(ld, A, 1, "ci8", host_only=True)
    h = ctypes.c_void_p()

    def plan_fold(plan, opts):
        return omni.lib.omni_fold_plan(ctypes.byref(h), plan, 0, ctypes.byref(opts) if opts is not None else None)

    good = omni._FoldOpts(1.0, 1.0, 1.0, 1.0, 5, 1)
    assert omni.STATUS[plan_fold(p._h, good)] == "OMNI_E_STATE"  # host-only plan
    for bad in (omni._FoldOpts(0.0, 1.0, 1.0, 1.0, 1, 0), omni._FoldOpts(1.0, -1.0, 1.0, 1.0, 1, 0),
                omni._FoldOpts(1.0, 1.0, float("nan"), 1.0, 1, 0), omni._FoldOpts(1.0, 1.0, 1.0, 0.0, 1, 0),
                omni._FoldOpts(1.0, 1.0, 1.0, 1.0, 4, 0), omni._FoldOpts(1.0, 1.0, 1.0, 1.0, 0, 0)):
        assert omni.STATUS[plan_fold(p._h, bad)] == "OMNI_E_INVAL"
    assert omni.STATUS[omni.lib.omni_fold_plan(ctypes.byref(h), p._h, 3, None)] == "OMNI_E_INVAL"
    assert omni.STATUS[omni.lib.omni_fold_plan(None, p._h, 0, None)] == "OMNI_E_INVAL"
    no_a = omni.Plan(ld, None, 1, "ci8", host_only=True)
    assert omni.STATUS[plan_fold(no_a._h, good)] == "OMNI_E_STATE"
    assert omni.lib.omni_fold(None, None, 1, None, None) == -1
    assert omni.lib.omni_baseline_profile(None, None, 1, None, None, None, None) == -1
    assert omni.lib.omni_fold_destroy(None) == 0


def test_fengine_validates_before_any_device_call():
    f = omni.lib.omni_fengine
    st = omni.STATUS
    assert st[f(16, 0, 4, 64, 16, 2, 16, None)] == "OMNI_E_INVAL"  # N < 1
    assert st[f(16, 8, -1, 64, 16, 2, 16, None)] == "OMNI_E_INVAL"  # T < 0
    assert st[f(16, 8, 4, 48, 16, 2, 16, None)] == "OMNI_E_SHAPE"  # F not 16 / 32 / 64
    assert st[f(16, 8, 4, 64, 16, 0, 16, None)] == "OMNI_E_INVAL"  # cf32 output
    assert f(None, 8, 0, 64, None, 2, None, None) == 0  # T == 0: nothing to do
    assert st[f(None, 8, 4, 64, 16, 2, 16, None)] == "OMNI_E_INVAL"  # NULL raw
    assert st[f(24, 8, 4, 64, 16, 2, 16, None)] == "OMNI_E_INVAL"  # raw not 16-byte aligned
    assert st[f(16, 8, 4, 64, 12, 2, 16, None)] == "OMNI_E_INVAL"  # gains not 8-byte aligned
    assert st[f(16, 8, 4, 64, 16, 1, 17, None)] == "OMNI_E_INVAL"  # ci8 output not 2-byte aligned


def test_beam_space_plans_on_the_host():
    """Beam-space plans: pointings last in the visibility shape, unpadded transforms on the lowest level's axes,
    the general kernel; refusals for one level, one block, and for the baseline metadata."""
    import json

    p = omni.Plan([[4, 4], [8, 8]], np.stack([np.eye(2) * 8, np.eye(2)]), 2, "ci8", host_only=True, beams=True)
    assert p.vis_shape() == (2, 7, 7, 8, 8)
    a = json.loads(p.describe())["arrays"][0]
    assert [(x["n"], x["m"]) for x in a["axes"]] == [(4, 8), (4, 8), (8, 8), (8, 8)]
    assert a["kernel"] == "fused_fp32" and a["M"] == 8 * 8 * 8 * 8
    with pytest.raises(omni.OmniError) as ei:
        p.baselines()
    assert omni.STATUS[ei.value.code] == "OMNI_E_STATE"
    q = omni.Plan([[4, 1], [1, 8]], None, 1, "ci4", host_only=True, beams=True)
    assert q.vis_shape() == (1, 7, 1, 1, 8)
    for ld in ([[8, 8]], [[1, 1], [8, 8]]):
        with pytest.raises(omni.OmniError) as ei:
            omni.Plan(ld, None, 1, "ci8", host_only=True, beams=True)
        assert omni.STATUS[ei.value.code] == "OMNI_E_SHAPE"
    assert a["beams"] == "unpadded"
    # where the ordinary plan has a fixed-shape kernel, the beam-space plan runs it and keeps the even cells
    r = omni.Plan([[8, 8], [8, 8]], None, 4, "ci8", "mixed", host_only=True, beams=True)
    b = json.loads(r.describe())["arrays"][0]
    assert (b["kernel"], b["beams"]) == ("fused8x4_mixed", "subset") and r.vis_shape() == (4, 15, 15, 8, 8)
    c = omni.Plan([[1, 64], [64, 1]], None, 2, "ci4", "mixed", host_only=True, beams=True)
    assert json.loads(c.describe())["arrays"][0]["beams"] == "subset" and c.vis_shape() == (2, 1, 127, 64, 1)


def test_hybrid_plan_validates_before_any_device_call():
    h = ctypes.c_void_p()
    f = omni.lib.omni_hybrid_plan
    st = omni.STATUS
    assert st[f(None, 4, 8, 8, 1, 2, None, None)] == "OMNI_E_INVAL"
    assert st[f(ctypes.byref(h), 3, 8, 8, 1, 2, None, None)] == "OMNI_E_SHAPE"  # P not a power of two
    assert st[f(ctypes.byref(h), 4, 12, 8, 1, 2, None, None)] == "OMNI_E_SHAPE"  # side 12
    assert st[f(ctypes.byref(h), 4, 8, 64, 1, 2, None, None)] == "OMNI_E_SHAPE"  # side 64 (m = 128)
    assert st[f(ctypes.byref(h), 4, 8, 8, 0, 2, None, None)] == "OMNI_E_INVAL"
    assert st[f(ctypes.byref(h), 4, 8, 8, 1, 7, None, None)] == "OMNI_E_INVAL"
    assert omni.lib.omni_hybrid_correlate(None, None, 0, None, None, 0) == -1
    assert omni.lib.omni_hybrid_destroy(None) == 0
    # a valid geometry goes as far as the device check
    rc = f(ctypes.byref(h), 4, 8, 8, 1, 2, None, None)
    assert st[rc] in ("OMNI_E_NODEV", "OMNI_OK")
    if rc == 0:
        omni.lib.omni_hybrid_destroy(h)


def _run_with_log_level(level, code):
    import subprocess
    import sys

    env = dict(os.environ)
    if level is None:
        env.pop("OMNI_LOG_LEVEL", None)
    else:
        env["OMNI_LOG_LEVEL"] = str(level)
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=120)


_LOG_PROBE = """
import paper_0909_0001_amd as omni
try:
    omni.Plan([[0, 4]], None, 1, host_only=True)
except omni.OmniError:
    pass
omni.Plan([[4, 4]], None, 1, host_only=True)
print("done")
"""


def test_log_level_controls_stderr():
    """OMNI_LOG_LEVEL: unset or 0 silent; 1 reports the returned error; 2 also the plan's description."""
    quiet = _run_with_log_level(None, _LOG_PROBE)
    assert quiet.returncode == 0 and "done" in quiet.stdout
    assert "omniscope:" not in quiet.stderr
    errors = _run_with_log_level(1, _LOG_PROBE)
    assert errors.returncode == 0
    lines = [ln for ln in errors.stderr.splitlines() if ln.startswith("omniscope:")]
    assert len(lines) == 1 and "error" in lines[0]
    verbose = _run_with_log_level(2, _LOG_PROBE)
    plans = [ln for ln in verbose.stderr.splitlines() if ln.startswith("omniscope: plan {")]
    assert len(plans) == 1 and '"arrays"' in plans[0]
