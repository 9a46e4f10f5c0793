"""Python binding of libomniscope (the MI355X hierarchical-grid correlator).

Thin ctypes marshalling over the C ABI in include/omniscope.h: every step of
the correlation runs in the library's HIP kernels.  torch is used only to own
device memory and to name the current HIP stream.  Importing this package
fails loudly if the library has not been built (``python
paper_0909_0001_amd/build.py``); there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libomniscope.so")

OMNI_OK = 0
STATUS = {
    0: "OMNI_OK",
    -1: "OMNI_E_INVAL",
    -2: "OMNI_E_SHAPE",
    -3: "OMNI_E_GEOM",
    -4: "OMNI_E_NODEV",
    -5: "OMNI_E_NOMEM",
    -6: "OMNI_E_HIP",
    -7: "OMNI_E_STATE",
}
DTYPES = {"cf32": 0, "ci8": 1, "ci4": 2}
FORMS = {"fp32": 0, "mixed": 1}
PLAN_HOST_ONLY = 0x1
PLAN_TIMING = 0x2
PLAN_GRAPH = 0x8
PLAN_BEAMS = 0x10
TUNE = {False: 0, None: 0, "off": 0, "cache": 1, True: 2, "search": 2}
STAGES = {"forward": 0, "reduce": 1, "inverse": 2, "call": 3, "kernel": 4}
NO_RESET = 0x1
NO_FINALIZE = 0x2

#: Every symbol include/omniscope.h declares.
EXPORTS = [
    "omni_plan",
    "omni_plan_batch",
    "omni_correlate",
    "omni_correlate_batch",
    "omni_direct_correlate",
    "omni_direct_correlate_noalloc",
    "omni_n_arrays",
    "omni_vis_shape",
    "omni_baselines",
    "omni_accumulator_bytes",
    "omni_accumulator_get",
    "omni_accumulator_set",
    "omni_plan_describe",
    "omni_stage_times",
    "omni_destroy",
    "omni_strerror",
    "omni_last_error",
    "omni_fold_plan",
    "omni_fold_shape",
    "omni_fold",
    "omni_baseline_profile",
    "omni_fold_destroy",
    "omni_fengine",
    "omni_hybrid_plan",
    "omni_hybrid_correlate",
    "omni_hybrid_baselines",
    "omni_hybrid_destroy",
]


class OmniError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class _Opts(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int),
        ("form", ctypes.c_int),
        ("time_block", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("tune", ctypes.c_int32),
        ("tune_cache", ctypes.c_char_p),
        ("chunk_T", ctypes.c_int32),
    ]


class _FoldOpts(ctypes.Structure):
    _fields_ = [
        ("du", ctypes.c_double),
        ("dv", ctypes.c_double),
        ("dr", ctypes.c_double),
        ("radius_scale", ctypes.c_double),
        ("boxcar", ctypes.c_int32),
        ("zero_origin", ctypes.c_int32),
    ]


class _ArrayDesc(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32),
        ("dims", ctypes.POINTER(ctypes.c_int32)),
        ("A", ctypes.POINTER(ctypes.c_double)),
        ("nchan", ctypes.c_int32),
    ]


def _load():
    # torch owns the device memory and streams this library works on, so its HIP
    # runtime must be the one in the process: import it before the library pulls
    # in libamdhip64.so.7 by soname (the system copy would otherwise be loaded
    # first and torch would start a second, device-less runtime).
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python paper_0909_0001_amd/build.py` (no CPU fallback exists)"
        )
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sig = {
        "omni_plan": (ctypes.c_int, [ctypes.POINTER(P), i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double), i32,
                                     ctypes.POINTER(_Opts)]),
        "omni_plan_batch": (ctypes.c_int, [ctypes.POINTER(P), i32, ctypes.POINTER(_ArrayDesc), ctypes.POINTER(_Opts)]),
        "omni_correlate": (ctypes.c_int, [P, P, i64, P, P, u32]),
        "omni_correlate_batch": (ctypes.c_int, [P, ctypes.POINTER(P), i64, ctypes.POINTER(P), P, u32]),
        "omni_direct_correlate": (ctypes.c_int, [P, P, i64, P, P]),
        "omni_direct_correlate_noalloc": (ctypes.c_int, [P, P, i64, P, P]),
        "omni_n_arrays": (ctypes.c_int, [P, ctypes.POINTER(i32)]),
        "omni_vis_shape": (ctypes.c_int, [P, i32, ctypes.POINTER(i32), ctypes.POINTER(i64)]),
        "omni_baselines": (ctypes.c_int, [P, i32, ctypes.POINTER(ctypes.c_double)]),
        "omni_accumulator_bytes": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_size_t)]),
        "omni_accumulator_get": (ctypes.c_int, [P, P, ctypes.c_size_t, P]),
        "omni_accumulator_set": (ctypes.c_int, [P, P, ctypes.c_size_t, P]),
        "omni_plan_describe": (ctypes.c_int, [P, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
        "omni_stage_times": (ctypes.c_int, [P, i32, i32, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(i32)]),
        "omni_destroy": (ctypes.c_int, [P]),
        "omni_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "omni_last_error": (ctypes.c_char_p, []),
        "omni_fold_plan": (ctypes.c_int, [ctypes.POINTER(P), P, i32, ctypes.POINTER(_FoldOpts)]),
        "omni_fold_shape": (ctypes.c_int, [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "omni_fold": (ctypes.c_int, [P, P, i32, P, P]),
        "omni_baseline_profile": (ctypes.c_int, [P, P, i32, P, P, P, P]),
        "omni_fold_destroy": (ctypes.c_int, [P]),
        "omni_fengine": (ctypes.c_int, [P, i64, i64, i32, P, i32, P, P]),
        "omni_hybrid_plan": (ctypes.c_int, [ctypes.POINTER(P), i32, i32, i32, i32, i32,
                                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
        "omni_hybrid_correlate": (ctypes.c_int, [P, P, i64, P, P, u32]),
        "omni_hybrid_baselines": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_double)]),
        "omni_hybrid_destroy": (ctypes.c_int, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(code: int) -> None:
    if code != OMNI_OK:
        raise OmniError(code, lib.omni_last_error().decode())


def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


class Plan:
    """A correlation plan for one array (or a batch of arrays) of a hierarchical grid.

    ``level_dims``: [[n_x, n_y], ...] per level (outer first);  ``A``: [levels, 2, 2]
    lattice matrices (columns = lattice vectors), or None.  ``tune``: False / "off",
    "cache" (stored schedule, else search) or True / "search"; ``tune_cache``: file of
    tuned schedules; ``chunk_T``: cap on the time samples per front-pass chunk (0: the
    planner's choice); ``beams``: beam-space variant (the lowest level's blocks are
    transformed into pointings, which are correlated over the outer levels; visibilities
    [F, 2n_1-1, ..., n_x, n_y]).

    Every device call checks its tensors against the plan before the library is
    called (dtype for the plan's sample format, shape [T, F, N(, 2)], contiguity,
    device; the output's shape and dtype): the C ABI receives raw pointers and
    cannot.  A mismatch raises ValueError.
    """

    def __init__(
        self,
        level_dims=None,
        A=None,
        nchan: int = 1,
        dtype: str = "cf32",
        form: str = "fp32",
        time_block: int = 0,
        host_only: bool = False,
        batch: Sequence[tuple] | None = None,
        timing: bool = False,
        tune=False,
        graph: bool = False,
        tune_cache: str | None = None,
        chunk_T: int = 0,
        beams: bool = False,
    ):
        self._h = ctypes.c_void_p()
        if dtype not in DTYPES:
            raise ValueError(f"unknown sample format {dtype!r} (cf32, ci8, ci4)")
        if form not in FORMS:
            raise ValueError(f"unknown form {form!r} (fp32, mixed)")
        if tune not in TUNE:
            raise ValueError(f"unknown tune mode {tune!r} (off, cache, search)")
        flags = (PLAN_HOST_ONLY if host_only else 0) | (PLAN_TIMING if timing else 0) | (PLAN_GRAPH if graph else 0)
        flags |= PLAN_BEAMS if beams else 0
        self._cache_path = tune_cache.encode() if tune_cache else None
        opts = _Opts(DTYPES[dtype], FORMS[form], time_block, flags, TUNE[tune], self._cache_path, chunk_T)
        self.dtype, self.form, self.graph = dtype, form, graph
        self._keep = []
        self._graph_outs = None
        if batch is None:
            dims = np.ascontiguousarray(np.asarray(level_dims, dtype=np.int32).reshape(-1, 2))
            levels = dims.shape[0]
            Ap = None
            if A is not None:
                Aa = np.ascontiguousarray(np.asarray(A, dtype=np.float64).reshape(levels, 2, 2))
                self._keep.append(Aa)
                Ap = Aa.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            _check(lib.omni_plan(ctypes.byref(self._h), levels, dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 Ap, nchan, ctypes.byref(opts)))
        else:
            descs = (_ArrayDesc * len(batch))()
            for i, (ld, Ab, nc) in enumerate(batch):
                dims = np.ascontiguousarray(np.asarray(ld, dtype=np.int32).reshape(-1, 2))
                self._keep.append(dims)
                descs[i].levels = dims.shape[0]
                descs[i].dims = dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
                if Ab is not None:
                    Aa = np.ascontiguousarray(np.asarray(Ab, dtype=np.float64).reshape(dims.shape[0], 2, 2))
                    self._keep.append(Aa)
                    descs[i].A = Aa.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                descs[i].nchan = nc
            _check(lib.omni_plan_batch(ctypes.byref(self._h), len(batch), descs, ctypes.byref(opts)))
        n = ctypes.c_int32()
        _check(lib.omni_n_arrays(self._h, ctypes.byref(n)))
        self.n_arrays = n.value
        # per array: (F, N) from the visibility shape [F, 2n_1 - 1, ...]
        # per array: (F, N)
        level_sets = [level_dims] if batch is None else [ld for ld, _, _ in batch]
        self._fn = []
        for i in range(self.n_arrays):
            N = int(np.prod(np.asarray(level_sets[i], dtype=np.int64)))
            self._fn.append((int(self.vis_shape(i)[0]), N))

    # -- metadata ---------------------------------------------------------
    def vis_shape(self, array: int = 0) -> tuple:
        nd = ctypes.c_int32()
        shape = (ctypes.c_int64 * 9)()
        _check(lib.omni_vis_shape(self._h, array, ctypes.byref(nd), shape))
        return tuple(shape[i] for i in range(nd.value))

    def baselines(self, array: int = 0) -> np.ndarray:
        shp = self.vis_shape(array)[1:]
        uv = np.zeros(int(np.prod(shp)) * 2, dtype=np.float64)
        _check(lib.omni_baselines(self._h, array, uv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return uv.reshape(tuple(shp) + (2,))

    def describe(self) -> str:
        need = ctypes.c_size_t()
        _check(lib.omni_plan_describe(self._h, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        _check(lib.omni_plan_describe(self._h, buf, need.value, ctypes.byref(need)))
        return buf.value.decode()

    def stage_times(self, stage: str = "forward", max_calls: int = 256) -> list:
        """Per-call durations (ms) of a stage over the most recent calls (plans made with timing=True)."""
        buf = (ctypes.c_float * max_calls)()
        n = ctypes.c_int32()
        _check(lib.omni_stage_times(self._h, STAGES[stage], max_calls, buf, ctypes.byref(n)))
        return [buf[i] for i in range(n.value)]

    def accumulator_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(lib.omni_accumulator_bytes(self._h, ctypes.byref(b)))
        return b.value

    # -- argument checks (the C ABI sees raw pointers only) ---------------
    def _check_volt(self, volt, array: int = 0) -> int:
        """Validate one array's voltages [T, F, N(, 2)] against the plan (dtype, shape, contiguity); returns T."""
        import torch

        F, N = self._fn[array]
        if not isinstance(volt, torch.Tensor):
            raise ValueError(f"array {array}: voltages must be a torch tensor, got {type(volt).__name__}")
        want = {
            "cf32": {torch.float32: (F, N, 2), torch.complex64: (F, N)},
            "ci8": {torch.int8: (F, N, 2)},
            "ci4": {torch.uint8: (F, N), torch.int8: (F, N)},
        }[self.dtype]
        if volt.dtype not in want:
            raise ValueError(f"array {array}: {self.dtype} samples must be "
                             + " or ".join(str(d).replace("torch.", "") for d in want) + f", got {volt.dtype}")
        shp = want[volt.dtype]
        if volt.dim() != 1 + len(shp) or tuple(volt.shape[1:]) != shp:
            raise ValueError(f"array {array}: voltages must have shape [T, {', '.join(map(str, shp))}] for this plan "
                             f"({self.dtype}, F={F}, N={N}), got {list(volt.shape)}")
        if not volt.is_contiguous():
            raise ValueError(f"array {array}: voltages must be contiguous")
        return int(volt.shape[0])

    def _check_volt_device(self, volt, array: int = 0) -> None:
        import torch

        if volt.device.type != "cuda":
            raise ValueError(f"array {array}: voltages must be on the GPU, got device {volt.device}")
        if volt.device.index != torch.cuda.current_device():
            raise ValueError(f"array {array}: voltages are on {volt.device}, the current device is "
                             f"cuda:{torch.cuda.current_device()}")
        if volt.shape[0] > 0 and volt.data_ptr() % 4:
            raise ValueError(f"array {array}: voltage pointer must be 4-byte aligned")

    def _check_out(self, out, array: int, like) -> None:
        import torch

        if not isinstance(out, torch.Tensor):
            raise ValueError(f"array {array}: out must be a torch tensor, got {type(out).__name__}")
        if out.dtype != torch.complex64:
            raise ValueError(f"array {array}: out must be complex64, got {out.dtype}")
        if tuple(out.shape) != self.vis_shape(array):
            raise ValueError(f"array {array}: out must have shape {list(self.vis_shape(array))}, got {list(out.shape)}")
        if not out.is_contiguous():
            raise ValueError(f"array {array}: out must be contiguous")
        if out.device.type != "cuda":
            raise ValueError(f"array {array}: out must be on the GPU, got device {out.device}")
        if like is not None and out.device != like.device:
            raise ValueError(f"array {array}: out is on {out.device}, voltages on {like.device}")

    # -- device calls -----------------------------------------------------
    def correlate_into(self, volt, T: int, vis, stream=None, flags: int = 0) -> None:
        """Raw call with device pointers (int).  Tensors are checked as in ``correlate``; plain integer pointers
        cannot be checked and are the caller's responsibility."""
        if hasattr(volt, "data_ptr"):
            if self._check_volt(volt) != T:
                raise ValueError(f"T={T} does not match the voltages' {volt.shape[0]} samples")
            self._check_volt_device(volt)
        if hasattr(vis, "data_ptr"):
            self._check_out(vis, 0, volt if hasattr(volt, "data_ptr") else None)
        vp = volt.data_ptr() if hasattr(volt, "data_ptr") else volt
        op = vis.data_ptr() if hasattr(vis, "data_ptr") else vis
        _check(lib.omni_correlate(self._h, vp, T, op, _stream_handle(stream), flags))

    def correlate(self, volt, flags: int = 0, out=None, stream=None):
        """Correlate device voltages [T, F, N(, 2)] -> complex64 visibilities [F, 2n_1-1, ...]."""
        if self.n_arrays != 1:
            raise ValueError("batch plan: use correlate_batch")
        outs = self.correlate_batch([volt], flags=flags, outs=None if out is None else [out], stream=stream)
        return outs[0] if outs else None

    def direct_correlate(self, volt, out=None, stream=None):
        """Direct N^2 correlator (comparison baseline, integer samples): device [T, F, N(, 2)] -> complex64
        visibilities [F, 2n_1-1, ...], exact up to the final rounding to float32."""
        import torch

        if self.n_arrays != 1:
            raise ValueError("the direct correlator takes single-array plans")
        T = self._check_volt(volt)
        self._check_volt_device(volt)
        if out is None:
            out = torch.empty(self.vis_shape(0), dtype=torch.complex64, device=volt.device)
        self._check_out(out, 0, volt)
        _check(lib.omni_direct_correlate(self._h, volt.data_ptr(), T, out.data_ptr(), _stream_handle(stream)))
        return out

    def direct_correlate_noalloc(self, volt, out, stream=None):
        """``direct_correlate`` through the entry point that allocates nothing (the library's fixed device
        scratch): ``out`` must be given; the binding allocates nothing either."""
        if self.n_arrays != 1:
            raise ValueError("the direct correlator takes single-array plans")
        T = self._check_volt(volt)
        self._check_volt_device(volt)
        self._check_out(out, 0, volt)
        _check(lib.omni_direct_correlate_noalloc(self._h, volt.data_ptr(), T, out.data_ptr(), _stream_handle(stream)))
        return out

    def correlate_batch(self, volts, flags: int = 0, outs=None, stream=None):
        """Correlate every array of the plan: ``volts[i]`` is array i's [T, F_i, N_i(, 2)] (a common T).
        Returns the list of visibility tensors (``outs`` if given).  A graph plan without ``outs`` reuses one set
        of output tensors for every call (its captured graph writes fixed addresses)."""
        import torch

        if len(volts) != self.n_arrays:
            raise ValueError(f"expected {self.n_arrays} voltage tensors, got {len(volts)}")
        Ts = [self._check_volt(v, i) for i, v in enumerate(volts)]
        if len(set(Ts)) != 1:
            raise ValueError(f"every array of a batch takes the same number of samples, got T = {Ts}")
        for i, v in enumerate(volts):
            self._check_volt_device(v, i)
        T = Ts[0]
        if outs is None and not (flags & NO_FINALIZE):
            if self.graph:
                if self._graph_outs is None:
                    self._graph_outs = [torch.empty(self.vis_shape(i), dtype=torch.complex64, device=volts[0].device)
                                        for i in range(self.n_arrays)]
                outs = self._graph_outs
            else:
                outs = [torch.empty(self.vis_shape(i), dtype=torch.complex64, device=volts[0].device)
                        for i in range(self.n_arrays)]
        if outs is not None:
            if len(outs) != self.n_arrays:
                raise ValueError(f"expected {self.n_arrays} output tensors, got {len(outs)}")
            for i, o in enumerate(outs):
                self._check_out(o, i, volts[i])
        vp = (ctypes.c_void_p * self.n_arrays)(*[v.data_ptr() if T > 0 else 0 for v in volts])
        op = (ctypes.c_void_p * self.n_arrays)(*([o.data_ptr() for o in outs] if outs else [0] * self.n_arrays))
        _check(lib.omni_correlate_batch(self._h, vp, T, op, _stream_handle(stream), flags))
        return outs

    def accumulator_get(self, buf, stream=None) -> None:
        self._check_acc(buf)
        ptr = buf.data_ptr() if hasattr(buf, "data_ptr") else buf.ctypes.data
        _check(lib.omni_accumulator_get(self._h, ptr, self.accumulator_bytes(), _stream_handle(stream)))

    def accumulator_set(self, buf, stream=None) -> None:
        self._check_acc(buf)
        ptr = buf.data_ptr() if hasattr(buf, "data_ptr") else buf.ctypes.data
        _check(lib.omni_accumulator_set(self._h, ptr, self.accumulator_bytes(), _stream_handle(stream)))

    def _check_acc(self, buf) -> None:
        nb = buf.numel() * buf.element_size() if hasattr(buf, "data_ptr") else buf.nbytes
        contiguous = buf.is_contiguous() if hasattr(buf, "data_ptr") else buf.flags["C_CONTIGUOUS"]
        if nb != self.accumulator_bytes() or not contiguous:
            raise ValueError(f"accumulator buffer must be contiguous and hold {self.accumulator_bytes()} bytes, "
                             f"got {nb}")

    def close(self) -> None:
        if self._h:
            lib.omni_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def fengine(raw, F: int, gains, dtype: str = "ci4", out=None, stream=None):
    """F-engine (Appendix A steps 2-3): raw int8 samples [N, 2 F T] (antenna-major, 16-byte aligned GPU tensor)
    and complex64 gains [N, F] -> the correlator's voltages [T, F, N] (ci4, uint8) or [T, F, N, 2] (ci8, int8)."""
    import torch

    if dtype not in ("ci4", "ci8"):
        raise ValueError("the F-engine writes ci4 or ci8 samples")
    if raw.dtype != torch.int8 or raw.dim() != 2 or not raw.is_contiguous() or raw.device.type != "cuda":
        raise ValueError("raw must be a contiguous int8 GPU tensor [N, 2 F T]")
    N, S = raw.shape
    if F not in (16, 32, 64) or S % (2 * F):
        raise ValueError(f"F must be 16, 32 or 64 and divide the {S} samples per antenna into 2F-sample blocks")
    T = S // (2 * F)
    if gains.dtype != torch.complex64 or tuple(gains.shape) != (N, F) or not gains.is_contiguous() \
            or gains.device != raw.device:
        raise ValueError(f"gains must be a contiguous complex64 tensor [{N}, {F}] on the raw samples' device")
    shape = (T, F, N) if dtype == "ci4" else (T, F, N, 2)
    tdt = torch.uint8 if dtype == "ci4" else torch.int8
    if out is None:
        out = torch.empty(shape, dtype=tdt, device=raw.device)
    if out.dtype != tdt or tuple(out.shape) != shape or not out.is_contiguous() or out.device != raw.device:
        raise ValueError(f"out must be a contiguous {tdt} tensor of shape {shape} on the raw samples' device")
    _check(lib.omni_fengine(raw.data_ptr(), N, T, F, gains.data_ptr(), DTYPES[dtype], out.data_ptr(),
                            _stream_handle(stream)))
    return out


class Hybrid:
    """Hybrid tiles (Sec. III): P tiles of nx x ny antennas at arbitrary offsets; ``correlate`` gives every ordered
    pair's cross-correlation over index differences, complex64 [F, P, P, 2nx-1, 2ny-1].  ``offsets`` [P, 2] and
    ``A`` [2, 2] (columns = a tile's lattice vectors) are metadata for ``baselines``."""

    def __init__(self, P: int, nx: int, ny: int, nchan: int = 1, dtype: str = "cf32", offsets=None, A=None):
        if dtype not in DTYPES:
            raise ValueError(f"unknown sample format {dtype!r} (cf32, ci8, ci4)")
        self._h = ctypes.c_void_p()
        self.P, self.nx, self.ny, self.F, self.dtype = P, nx, ny, nchan, dtype
        self.N = P * nx * ny
        op = Ap = None
        self._keep = []
        if offsets is not None:
            o = np.ascontiguousarray(np.asarray(offsets, dtype=np.float64).reshape(P, 2))
            self._keep.append(o)
            op = o.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if A is not None:
            a = np.ascontiguousarray(np.asarray(A, dtype=np.float64).reshape(2, 2))
            self._keep.append(a)
            Ap = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        _check(lib.omni_hybrid_plan(ctypes.byref(self._h), P, nx, ny, nchan, DTYPES[dtype], op, Ap))

    def vis_shape(self) -> tuple:
        return (self.F, self.P, self.P, 2 * self.nx - 1, 2 * self.ny - 1)

    def correlate(self, volt, flags: int = 0, out=None, stream=None):
        import torch

        want = {"cf32": torch.float32, "ci8": torch.int8, "ci4": torch.uint8}[self.dtype]
        tail = (self.F, self.N, 2) if self.dtype != "ci4" else (self.F, self.N)
        if volt.dtype != want or tuple(volt.shape[1:]) != tail or not volt.is_contiguous() or volt.device.type != "cuda":
            raise ValueError(f"voltages must be a contiguous {want} GPU tensor [T, {', '.join(map(str, tail))}]")
        T = volt.shape[0]
        if out is None and not (flags & NO_FINALIZE):
            out = torch.empty(self.vis_shape(), dtype=torch.complex64, device=volt.device)
        if out is not None and (out.dtype != torch.complex64 or tuple(out.shape) != self.vis_shape()
                                or not out.is_contiguous() or out.device != volt.device):
            raise ValueError(f"out must be a contiguous complex64 tensor {self.vis_shape()} on the voltages' device")
        _check(lib.omni_hybrid_correlate(self._h, volt.data_ptr() if T > 0 else None, T,
                                         out.data_ptr() if out is not None else None, _stream_handle(stream), flags))
        return out

    def baselines(self) -> np.ndarray:
        uv = np.zeros(int(np.prod(self.vis_shape()[1:])) * 2, dtype=np.float64)
        _check(lib.omni_hybrid_baselines(self._h, uv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return uv.reshape(self.vis_shape()[1:] + (2,))

    def close(self) -> None:
        if self._h:
            lib.omni_hybrid_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Fold:
    """Physical-baseline fold of one array's visibilities onto a (u, v) pixel grid, and the
    baseline-distribution products (asinh map, radial distribution, boxcar) of Sec. III.

    ``plan`` must carry lattice matrices.  Pixel size ``du`` x ``dv`` (units of A), radial bins of
    width ``dr`` after multiplying |b| by ``radius_scale``, boxcar width ``boxcar`` (odd),
    ``zero_origin`` zeroes the zero-baseline pixel.  The cell -> pixel grouping is built on the
    device once, here.
    """

    def __init__(self, plan: Plan, array: int = 0, du: float = 1.0, dv: float = 1.0, dr: float = 1.0,
                 radius_scale: float = 1.0, boxcar: int = 1, zero_origin: bool = False):
        self._h = ctypes.c_void_p()
        self._plan = plan
        self.array = array
        o = _FoldOpts(du, dv, dr, radius_scale, boxcar, 1 if zero_origin else 0)
        _check(lib.omni_fold_plan(ctypes.byref(self._h), plan._h, array, ctypes.byref(o)))
        ny, nx, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.omni_fold_shape(self._h, ctypes.byref(ny), ctypes.byref(nx), ctypes.byref(nb)))
        self.shape = (ny.value, nx.value)
        self.nbins = nb.value
        self.F, _ = plan._fn[array]
        self._cells = int(np.prod(plan.vis_shape(array)[1:]))

    def fold(self, vis, out=None, stream=None):
        """complex64 visibilities [C, 2n_1-1, ...] (C <= F channels) -> complex128 image [C, ny, nx]."""
        import torch

        if vis.dtype != torch.complex64 or not vis.is_contiguous() or vis.device.type != "cuda":
            raise ValueError("vis must be a contiguous complex64 GPU tensor")
        C = vis.shape[0]
        if vis.numel() != C * self._cells or not 1 <= C <= self.F:
            raise ValueError(f"vis must be [C <= {self.F}, ...] with {self._cells} cells per channel")
        if out is None:
            out = torch.empty((C,) + self.shape, dtype=torch.complex128, device=vis.device)
        if out.dtype != torch.complex128 or tuple(out.shape) != (C,) + self.shape or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous complex128 tensor of shape {(C,) + self.shape}")
        if out.device != vis.device:
            raise ValueError("out and vis must be on one device")
        _check(lib.omni_fold(self._h, vis.data_ptr(), C, out.data_ptr(), _stream_handle(stream)))
        return out

    def profile(self, image, stream=None):
        """(asinh map [C, ny, nx], radial sums [C, nbins], boxcar-smoothed sums [C, nbins]) of Re image."""
        import torch

        if image.dtype != torch.complex128 or not image.is_contiguous() or image.device.type != "cuda":
            raise ValueError("image must be a contiguous complex128 GPU tensor")
        C = image.shape[0]
        if tuple(image.shape) != (C,) + self.shape or not 1 <= C <= self.F:
            raise ValueError(f"image must be [C <= {self.F}, {self.shape[0]}, {self.shape[1]}]")
        dev = image.device
        m = torch.empty((C,) + self.shape, dtype=torch.float64, device=dev)
        h = torch.empty((C, self.nbins), dtype=torch.float64, device=dev)
        sm = torch.empty((C, self.nbins), dtype=torch.float64, device=dev)
        _check(lib.omni_baseline_profile(self._h, image.data_ptr(), C, m.data_ptr(), h.data_ptr(), sm.data_ptr(),
                                         _stream_handle(stream)))
        return m, h, sm

    def close(self) -> None:
        if self._h:
            lib.omni_fold_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def strerror(code: int) -> str:
    return lib.omni_strerror(code).decode()
