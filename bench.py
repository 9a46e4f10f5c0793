#!/usr/bin/env python3
"""Throughput of the hierarchical-grid correlator on one MI355X.

One step = one batched correlate call over the whole workload: every time
sample of every channel of every array through the forward transform, |X|^2
and time integration, then the inverse transform to visibilities.  Inputs are
synthetic (seeded sky-plus-noise voltages, quantised) and already resident in
HBM.

Default (`--workload batch4`): the four arrays 32x32, 64x64, 128x128 and
16x16-of-16x16 (64 channels each, T = 2048, 4-bit samples) as one batched call
in the mixed form, captured as one HIP graph with one branch per array.
`value` is that call's antenna-samples/s; the float32 form on the same bytes
and the sequential (non-graph) batch are timed beside it.  `roofline` is the
main forward kernel of the dominant array (per-launch HIP events recorded by
the library around that kernel, array alone, same bytes), `roofline_call` the
whole call against the fixed work counts of all four arrays, `per_array` the
same kernel rooflines for every array.

`--workload NAME` times one workload of skysim.WORKLOADS in its own form, the
other form on the same bytes under `other_form`, and (integer samples, N <=
16384) the GPU direct N^2 correlator.

Prints ONE JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "antenna-samples/s correlated (N·T·F/s) vs FP32 FFT form, at stated rel. err"
# MI355X published peaks: fp32 vector 157.3 TFLOP/s (256 CUs x 4 SIMD x 16 lanes x 2 packed x 2 FMA x 2.4 GHz),
# dense fp16 MFMA 2.5 PFLOP/s, HBM 8 TB/s.
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_FP16_MFMA_TFLOPS = 2500.0
PEAK_INT8_MFMA_TOPS = 5000.0  # dense int8 matrix-core peak (no sparsity)
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fp32_form_flops_per_as(dims) -> float:
    """Fixed FP32 FFT-form work per antenna-sample: line-pruned FFT flops sum_p 2^p 10 log2 m_(p)
    over axes sorted by decreasing padded length, plus 4 * 2^d for |X|^2 and the time sum."""
    m = sorted((2 * n for n in dims if n > 1), reverse=True)
    d = len(m)
    return sum((2**p) * 10 * math.log2(mp) for p, mp in enumerate(m)) + 4 * 2**d


def mixed_form_flops_per_as(dims) -> float:
    """Fixed mixed-form MFMA work per antenna-sample: 2 (hi + lo twiddles) x 8 (flops of a real-embedded
    complex MAC) x sum_p 2^p c(m_(p)), axes by decreasing padded length; c(m) = m for m <= 32 (dense
    pruned DFT), else min over r1 r2 = m of r1 + 2 r2 + 2."""
    m = sorted((2 * n for n in dims if n > 1), reverse=True)

    def c(mm):
        if mm <= 32:
            return mm
        return min(r1 + 2 * (mm // r1) + 2 for r1 in range(2, mm) if mm % r1 == 0)

    return 16 * sum((2**p) * c(mp) for p, mp in enumerate(m))


def recorded_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary (its
    traffic_bytes_per_launch line), if the kernel's sources are unchanged since; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    # one or more sources (space-separated) with their hashes in the same order
    names, hashes = rec.get("source", "-").split(), rec.get("source_sha256", "").split()
    if len(names) != len(hashes):
        return None
    for name, want in zip(names, hashes):
        src = os.path.join(ROOT, "paper_0909_0001_amd", "csrc", name)
        if not os.path.isfile(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != want:
            return None
    v = rec.get("traffic_bytes_per_launch")
    return float(v) if v is not None else None


def copy_calibration() -> int:
    """Three plain 1 GiB device copies, for calibrating FETCH_SIZE / WRITE_SIZE against known bytes."""
    import torch

    n = 1 << 30
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copy calibration: 3 x 1 GiB device copies done")
    return 0


def front_axes(desc_array) -> int:
    return int(desc_array.get("n_front", 0))


def kernel_flops_per_as(dims, n_front: int, form: str) -> float:
    """Fixed work per antenna-sample of the main forward kernel alone: the form's count over the axes that
    kernel transforms (a front pass transforms the first n_front axes on the vector units and over HBM; its
    share is left out).  The front outputs are 2^n_front times the antennas, which the count carries."""
    dims = [n for n in dims if n > 1]
    front, rest = dims[:n_front], dims[n_front:]
    scale = 2 ** len(front)
    if form == "mixed":
        return scale * mixed_form_flops_per_as(rest)
    return scale * fp32_form_flops_per_as(rest)


def kernel_roofline(w, res, form):
    """Roofline entry of the main forward kernel of one plan, from the per-launch HIP events the library records
    around it (OMNI_STAGE_KERNEL) on the stream it runs on: algorithmic flops per launch / mean launch time."""
    arr = res["desc"]["arrays"][0]
    n_front = front_axes(arr)
    mixed_kernel = "mixed" in arr["kernel"]
    kform = "mixed" if mixed_kernel else "fp32"
    per_as = kernel_flops_per_as(w.dims, n_front, kform)
    launches = res["launches"]
    as_per_launch = w.antenna_samples() / launches
    launch_ms = res["stages"]["kernel"]
    achieved = per_as * as_per_launch / (launch_ms / 1e3) / 1e12
    peak, bound = (PEAK_FP16_MFMA_TFLOPS, "mfma") if mixed_kernel else (PEAK_FP32_VECTOR_TFLOPS, "alu")
    kname = arr["kernel"] + "_kernel"
    return {
        "bound": bound,
        "achieved": round(achieved, 3),
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4),
        "traffic": recorded_traffic(kname, w.name),
        "kernel": kname,
        "launch_ms": round(launch_ms, 4),
        "launches_per_call": launches,
        "algorithmic_flops_per_launch": per_as * as_per_launch,
        "algorithmic_flops_per_antenna_sample": per_as,
    }


def run_form(omni, w, raw, form, steps, warmup, tune="off", tune_cache=None, beams=False):
    """Plan (autotuned with tune="search"; beam-space with beams=True), warm up and time `steps` correlate calls;
    returns timings and the last visibilities."""
    import torch

    plan = omni.Plan(w.level_dims, w.A, w.nchan, w.dtype, form, timing=True, tune=tune, tune_cache=tune_cache,
                     beams=beams)
    desc = json.loads(plan.describe())
    log(f"bench[{w.name} {form}]: plan " + plan.describe())
    vis = torch.empty(plan.vis_shape(), dtype=torch.complex64, device=raw.device)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.correlate(raw, out=vis, stream=stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        plan.correlate(raw, out=vis, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e3
    ms = ev0.elapsed_time(ev1) / steps
    stages = {}
    for k in ("forward", "reduce", "inverse", "kernel"):
        v = plan.stage_times(k, steps)
        stages[k] = sum(v) / len(v)
    calls = sorted(plan.stage_times("call", steps))  # per-call events around each whole call
    stages["call_median"] = calls[len(calls) // 2] if len(calls) % 2 else 0.5 * (calls[len(calls) // 2 - 1] + calls[len(calls) // 2])
    stages["call_min"] = calls[0]
    arr = desc["arrays"][0]
    launches = -(-w.T // arr["chunk_T"]) if arr["n_front"] else 1
    log(f"bench[{w.name} {form}]: {ms:.3f} ms/step (wall {wall:.3f}); "
        + ", ".join(f"{k} {v:.3f} ms" for k, v in stages.items()) + f"; {launches} kernel launch(es) per call")
    return {"ms": ms, "stages": stages, "kernel": arr["kernel"] + "_kernel", "vis": vis, "plan": plan,
            "desc": desc, "launches": launches}


def roofline_of(w, res, work):
    """Roofline entry of a single-workload line: the main forward kernel (per-launch events)."""
    return kernel_roofline(w, res, res["desc"]["form"])


def run_direct(omni, w, raw, steps, warmup):
    """Time `steps` calls of the GPU direct N^2 correlator (the comparison baseline) on the same input."""
    import torch

    plan = omni.Plan(w.level_dims, w.A, w.nchan, w.dtype, "fp32")
    vis = torch.empty(plan.vis_shape(), dtype=torch.complex64, device=raw.device)
    stream = torch.cuda.current_stream()
    for _ in range(max(1, warmup)):
        plan.direct_correlate(raw, out=vis, stream=stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        plan.direct_correlate(raw, out=vis, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    log(f"bench[direct]: {ms:.3f} ms/step")
    return {"ms": ms, "vis": vis, "plan": plan}


BATCH4 = ["grid32", "grid64", "grid128", "hier16x16"]


def run_batch(omni, ws, raws, form, graph, steps, warmup, tune="off", tune_cache=None):
    """Plan the arrays as one batch (optionally as a graph plan; autotuned with tune="search"), warm up, time
    `steps` batched calls."""
    import torch

    plan = omni.Plan(batch=[(w.level_dims, w.A, w.nchan) for w in ws], dtype=ws[0].dtype, form=form,
                     timing=True, graph=graph, tune=tune, tune_cache=tune_cache)
    outs = [torch.empty(plan.vis_shape(i), dtype=torch.complex64, device=raws[0].device) for i in range(len(ws))]
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.correlate_batch(raws, outs=outs, stream=stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        plan.correlate_batch(raws, outs=outs, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    calls = sorted(plan.stage_times("call", steps))
    arrays = json.loads(plan.describe())["arrays"]
    kernels = [a["kernel"] for a in arrays]
    schedules = {w.name: {"wg_target": a["wg_target"], "block": a["block"], "tuned_ms": a["tuned_ms"]}
                 for w, a in zip(ws, arrays)}
    log(f"bench[batch4 {form} graph={graph} tune={tune}]: {ms:.3f} ms/call (call events: median "
        f"{calls[len(calls) // 2]:.3f}); kernels {kernels}; schedules {schedules}")
    return {"ms": ms, "call_ms": calls, "outs": outs, "kernels": kernels, "schedules": schedules}


def bench_fold(omni, torch, skysim, steps, warmup, vis128=None):
    """Sec. II.D fold and Sec. III baseline distributions on the GPU.

    * experiment: per example layout, one all-ones sample through the correlator (float32 form), the fold
      (origin zeroed) and the asinh map / radial sums / 5-bin boxcar, timed together per call;
    * throughput: the fold gather alone on the 128x128 array's 64-channel visibilities of the batched call
      (lattice 0.5, pixel 0.5: one cell per pixel), against HBM: algorithmic bytes = 8 B read per cell and
      16 B written per pixel, per channel.
    """
    import numpy as np

    out = {"experiment": {}}
    for name, (ld, A) in skysim.PAPER_LAYOUTS.items():
        N = int(np.prod([v for l in ld for v in l]))
        plan = omni.Plan(ld, A, 1, "ci8", "fp32")
        raw = torch.zeros((1, 1, N, 2), dtype=torch.int8, device="cuda")
        raw[..., 0] = 1
        fold = omni.Fold(plan, boxcar=5, zero_origin=True)
        vis = torch.empty(plan.vis_shape(), dtype=torch.complex64, device="cuda")
        img = torch.empty((1,) + fold.shape, dtype=torch.complex128, device="cuda")

        def step():
            plan.correlate(raw, out=vis)
            fold.fold(vis, out=img)
            return fold.profile(img)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        times = []
        for _ in range(steps):
            b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            b.record()
            step()
            e.record()
            e.synchronize()
            times.append(b.elapsed_time(e))
        times.sort()
        out["experiment"][name] = {"N": N, "image": list(fold.shape), "radial_bins": fold.nbins,
                                   "ms_median": round(times[len(times) // 2], 4)}
        del fold, plan
    if vis128 is not None:
        F = vis128.shape[0]
        plan = omni.Plan([[128, 128]], [skysim.lattice(0.5)], F, "ci4", "mixed", host_only=False)
        fold = omni.Fold(plan, du=0.5, dv=0.5)
        img = torch.empty((F,) + fold.shape, dtype=torch.complex128, device="cuda")
        for _ in range(warmup):
            fold.fold(vis128, out=img)
        torch.cuda.synchronize()
        b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        n = max(steps, 20)
        b.record()
        for _ in range(n):
            fold.fold(vis128, out=img)
        e.record()
        e.synchronize()
        ms = b.elapsed_time(e) / n
        cells = int(np.prod(vis128.shape[1:]))
        nbytes = F * (8 * cells + 16 * fold.shape[0] * fold.shape[1])
        gbs = nbytes / (ms / 1e3) / 1e9
        out["fold_grid128_64ch"] = {"ms_per_fold": round(ms, 5), "image": list(fold.shape),
                                    "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                                                 "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                                                 "algorithmic_bytes": nbytes}}
        del fold, plan
    return out


def beam_flops_per_as(dims, form) -> float:
    """Algorithmic work per antenna-sample of the beam-space variant: the counts of the two forms with the lowest
    level's two axes unpadded (m = n: a transform that adds no points).  Passes in decreasing m; the point count
    grows by m / n after each pass.  Mixed form: 16 flops (hi + lo, real-embedded complex MAC) x the growth so far
    x c(m) per pass (c(m) = m for m <= 32, as for the hot path); FP32 form: (m / n) 5 log2 m per point and pass,
    plus 4 flops per Fourier cell for |X|^2 and the time sum."""
    n = [v for v in dims]
    m = [2 * v for v in n[:-2]] + n[-2:]
    axes = sorted((k for k in range(len(n)) if n[k] > 1), key=lambda k: -m[k])
    total, growth = 0.0, 1.0
    for k in axes:
        if form == "mixed":
            c = m[k] if m[k] <= 32 else min(r1 + 2 * (m[k] // r1) + 2 for r1 in range(2, m[k]) if m[k] % r1 == 0)
            total += 16 * growth * c
        else:
            total += growth * (m[k] / n[k]) * 5 * math.log2(m[k])
        growth *= m[k] / n[k]
    return total if form == "mixed" else total + 4 * growth


def bench_beams(omni, torch, w, raw, steps, warmup, main_ms, form="mixed"):
    """Beam-space variant (Appendix A steps 4-5) on the same bytes as the array's hot-path call: every lowest-level
    16 x 16 block formed into 256 pointings, each correlated over the outer 16 x 16 level.  The plan runs the
    ordinary kernel of the grid and keeps the even Fourier cells of the block axes (the unpadded transform's
    cells), so the kernel does twice the variant's own work on the block axes; the roofline counts only the
    variant's algorithmic work, over the whole call."""
    res = run_form(omni, w, raw, form, steps, warmup, tune="search", beams=True)
    per_as = beam_flops_per_as(w.dims, form)
    achieved = per_as * w.antenna_samples() / (res["ms"] / 1e3) / 1e12
    peak, bound = (PEAK_FP16_MFMA_TFLOPS, "mfma") if form == "mixed" else (PEAK_FP32_VECTOR_TFLOPS, "alu")
    out = {"workload": f"{w.name} beam-space: {w.level_dims[-1][0] * w.level_dims[-1][1]} pointings a block, "
           f"{form} form", "kernel": res["kernel"], "route": res["desc"]["arrays"][0]["beams"],
           "ms_per_call": round(res["ms"], 4), "value": w.antenna_samples() / (res["ms"] / 1e3),
           "vs_hot_path_same_bytes": round(main_ms / res["ms"], 4) if main_ms == main_ms else None,
           "roofline": {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                        "frac": round(achieved / peak, 4), "algorithmic_flops_per_antenna_sample": per_as,
                        "note": "variant's own work over the whole call time"}}
    del res
    return out

def bench_hybrid(omni, torch, steps, warmup, P=16, nx=16, ny=16, F=64, T=2048):
    """Hybrid tiles (Sec. III): P tiles of nx x ny antennas (the 16x16-of-16x16 array's antennas, N = 4096 x P/16)
    at arbitrary offsets, 4-bit samples.  Work counted: the pair stage's P (P + 1) / 2 distinct tile pairs (the
    other half is their conjugate), one complex multiply-add (8 flops) each per Fourier cell (m = 2n per axis),
    channel and sample; it runs on the vector ALUs in float32."""
    gen = torch.Generator(device="cuda").manual_seed(20090840)
    N = P * nx * ny
    re = torch.randint(-7, 8, (T, F, N), generator=gen, device="cuda", dtype=torch.int16)
    im = torch.randint(-7, 8, (T, F, N), generator=gen, device="cuda", dtype=torch.int16)
    raw = ((re & 0xF) << 4 | (im & 0xF)).to(torch.uint8)
    del re, im
    h = omni.Hybrid(P, nx, ny, F, "ci4")
    out = torch.empty(h.vis_shape(), dtype=torch.complex64, device="cuda")
    for _ in range(max(1, warmup)):
        h.correlate(raw, out=out)
    torch.cuda.synchronize()
    b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.record()
    for _ in range(steps):
        h.correlate(raw, out=out)
    e.record()
    e.synchronize()
    ms = b.elapsed_time(e) / steps
    flops = 8.0 * (P * (P + 1) // 2) * (4 * nx * ny) * F * T
    tfs = flops / (ms / 1e3) / 1e12
    del raw, out, h
    return {"P": P, "tile": [nx, ny], "N": N, "F": F, "T": T, "ms_per_call": round(ms, 4),
            "value": N * T * F / (ms / 1e3), "unit": "antenna-samples/s",
            "roofline": {"bound": "alu", "achieved": round(tfs, 3), "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tfs / PEAK_FP32_VECTOR_TFLOPS, 4), "algorithmic_flops_per_call": flops,
                         "note": "pair-stage work over the whole call (tile transforms and the inverse included "
                                 "in the time)"}}


def bench_fengine(omni, torch, steps, warmup, N=16384, F=64, T=2048):
    """F-engine (Appendix A steps 2-3) on the 128x128 array's size: N antennas x T blocks of 2F int8 samples ->
    ci4 voltages [T][F][N].  Algorithmic HBM bytes: 2F in + F out per antenna and block (gains: 8 F per antenna);
    matrix-core work: the (2F outputs) x (2F samples) real product, 4 F^2 multiply-adds, run as three int8
    coefficient parts: 24 F^2 int8 operations per antenna and block, against the int8 matrix-core peak."""
    gen = torch.Generator(device="cuda").manual_seed(20090839)
    raw = torch.randint(-40, 41, (N, 2 * F * T), generator=gen, device="cuda", dtype=torch.int8)
    gains = torch.full((N, F), complex(2.5 / (23.0 * math.sqrt(F)), 0.0), dtype=torch.complex64, device="cuda")
    out = torch.empty((T, F, N), dtype=torch.uint8, device="cuda")
    for _ in range(max(1, warmup)):
        omni.fengine(raw, F, gains, "ci4", out=out)
    torch.cuda.synchronize()
    b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.record()
    for _ in range(steps):
        omni.fengine(raw, F, gains, "ci4", out=out)
    e.record()
    e.synchronize()
    ms = b.elapsed_time(e) / steps
    nbytes = N * T * (2 * F + F) + N * F * 8
    ops = 24.0 * F * F * N * T
    gbs = nbytes / (ms / 1e3) / 1e9
    tops = ops / (ms / 1e3) / 1e12
    hbm = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": round(gbs / PEAK_HBM_GBS, 4), "algorithmic_bytes": nbytes}
    mfma = {"bound": "mfma", "achieved": round(tops, 1), "peak": PEAK_INT8_MFMA_TOPS, "unit": "TOP/s",
            "frac": round(tops / PEAK_INT8_MFMA_TOPS, 4), "int8_ops": ops}
    del raw, out
    return {"N": N, "F": F, "T": T, "ms_per_call": round(ms, 4), "samples_per_s": N * T * 2 * F / (ms / 1e3),
            "roofline": hbm if hbm["frac"] >= mfma["frac"] else mfma, "roofline_hbm": hbm, "roofline_mfma": mfma}


def bench_aux(args) -> int:
    """Lines of their own for the steps around the correlator: the F-engine (`--workload fengine`) and the baseline
    fold with the Sec. III distributions (`--workload baselines`)."""
    import torch

    import paper_0909_0001_amd as omni
    import skysim

    torch.cuda.set_device(0)
    if args.workload == "fengine":
        r = bench_fengine(omni, torch, args.steps, args.warmup)
        line = {"metric": "raw samples/s channelised (F-engine)", "value": r["samples_per_s"], "unit": "samples/s",
                "ms_per_step": r["ms_per_call"], "config": {"workload": f"F-engine: N={r['N']} antennas, "
                f"T={r['T']} blocks of {2 * r['F']} int8 samples -> {r['F']} channels, ci4 [T][F][N]"},
                "roofline": r["roofline"], "detail": r}
    elif args.workload == "hybrid":
        r = bench_hybrid(omni, torch, args.steps, args.warmup)
        line = {"metric": "antenna-samples/s correlated (hybrid tiles, every tile pair)", "value": r["value"],
                "unit": "antenna-samples/s", "ms_per_step": r["ms_per_call"],
                "config": {"workload": f"hybrid tiles: {r['P']} tiles of {r['tile'][0]}x{r['tile'][1]}, "
                           f"F={r['F']}, T={r['T']}, ci4"}, "roofline": r["roofline"], "detail": r}
    elif args.workload == "beams":
        w = skysim.WORKLOADS["hier16x16"]
        raw = skysim.make_voltages(w, device=torch.device("cuda:0"))
        r = bench_beams(omni, torch, w, raw, args.steps, args.warmup, float("nan"))
        line = {"metric": "antenna-samples/s correlated (beam-space variant)", "value": r["value"],
                "unit": "antenna-samples/s", "ms_per_step": r["ms_per_call"], "config": {"workload": r["workload"]},
                "roofline": r["roofline"], "detail": r}
    else:
        r = bench_fold(omni, torch, skysim, args.steps, args.warmup)
        line = {"metric": "baseline distributions (Sec. III layouts)", "value": None, "unit": "ms",
                "config": {"workload": "all-ones sample through the correlator, fold, asinh map, radial sums, boxcar"},
                "detail": r}
    line.update({"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "data": "synthetic", "cpu_baseline": None,
                 "vs_baseline": None})
    print(json.dumps(line), flush=True)
    return 0


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_batch4(args) -> int:
    import numpy as np
    import torch

    import paper_0909_0001_amd as omni
    import skysim

    form = args.form or "mixed"
    other = "fp32" if form == "mixed" else "mixed"
    ws = [skysim.WORKLOADS[n] for n in BATCH4]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    raws = []
    for w in ws:
        log(f"bench: generating {w.name} N={w.N} F={w.nchan} T={w.T} {w.dtype}")
        raws.append(skysim.make_voltages(w, device=dev))
    torch.cuda.synchronize()
    # the timed line: one batched call of the four arrays as a HIP graph, `form` form
    # with autotuning, the graph plan searches and stores its schedules in a scratch cache file; the sequential
    # plan and the single-array runs take the same schedules from it (same launches, so the same bytes)
    import tempfile

    fd, cache = tempfile.mkstemp(prefix="omni_tune_", suffix=".txt")
    os.close(fd)
    again = "cache" if args.tune == "search" else "off"
    g = run_batch(omni, ws, raws, form, True, args.steps, args.warmup, args.tune, cache)
    seq = run_batch(omni, ws, raws, form, False, args.steps, args.warmup, again, cache)
    alt = (run_batch(omni, ws, raws, other, True, args.steps, args.warmup, args.tune, cache)
           if not args.no_other_form else None)
    same = all(torch.equal(a, b) for a, b in zip(g["outs"], seq["outs"]))
    work = sum(w.antenna_samples() for w in ws)
    ms = g["ms"]
    # each array alone (same bytes, same form): its main kernel's per-launch events give the rooflines; the
    # dominant array (the 16x16-of-16x16 one, most of the call) gives the line's `roofline`
    alone = {w.name: run_form(omni, w, r, form, args.steps, args.warmup, again, cache) for w, r in zip(ws, raws)}
    os.unlink(cache)
    per_array = {}
    for w in ws:
        res = alone[w.name]
        per_array[w.name] = {
            "N": w.N, "F": w.nchan, "T": w.T, "kernel": res["kernel"], "ms_alone": round(res["ms"], 4),
            "value_alone": w.antenna_samples() / (res["ms"] / 1e3),
            "roofline": kernel_roofline(w, res, form),
        }
    dom = max(ws, key=lambda w: alone[w.name]["ms"])
    # the whole call against the fixed work counts of every array in the form's own roof
    if form == "mixed":
        flops = sum(mixed_form_flops_per_as(w.dims) * w.antenna_samples() for w in ws)
        call_peak = PEAK_FP16_MFMA_TFLOPS
    else:
        flops = sum(fp32_form_flops_per_as(w.dims) * w.antenna_samples() for w in ws)
        call_peak = PEAK_FP32_VECTOR_TFLOPS
    call_achieved = flops / (ms / 1e3) / 1e12
    err = {"graph_equals_sequential_bytes": same}
    if alt is not None:
        # the two forms on the same bytes, per array, relative to the zero lag of each channel
        for w, a, b in zip(ws, g["outs"], alt["outs"]):
            av, bv = a.reshape(w.nchan, -1), b.reshape(w.nchan, -1)
            c = av.shape[1] // 2
            err[f"{w.name}_{form}_vs_{other}"] = float(((av - bv).abs().max(dim=1).values / bv[:, c].abs()).max())
    cpu = None
    if not args.no_cpu_baseline:
        # whole channels of the smallest arrays, smallest first, until about cpu_budget seconds of oracle work
        done_as, done_s, parts = 0, 0.0, []
        for i, w0 in enumerate(ws[:2]):
            if done_s >= args.cpu_budget:
                break
            rate, nch, secs, ref = cpu_oracle_baseline(raws[i].cpu(), w0, budget_s=args.cpu_budget - done_s)
            done_as += w0.N * w0.T * nch
            done_s += secs
            parts.append(f"{nch} of {w0.nchan} channels of {w0.name} (N={w0.N}) x all {w0.T} samples, {secs:.1f} s")
            got = g["outs"][i].cpu().numpy().reshape(w0.nchan, -1)
            c = got.shape[1] // 2
            err[f"{w0.name}_{form}_max_over_lags_vs_oracle_{nch}ch"] = max(
                float(np.max(np.abs(got[f] - ref[f])) / abs(ref[f][c])) for f in ref)
        cpu = {"value": done_as / done_s, "unit": "antenna-samples/s", "cores": len(os.sched_getaffinity(0)),
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": "; ".join(parts) + " (float64 pair products by BLAS matmul + histogram by index "
               "difference); the rate is over those arrays only, not extrapolated to the larger arrays, whose "
               "direct cost grows as N^2"}
    out = {
        "metric": METRIC,
        "value": work / (ms / 1e3),
        "unit": "antenna-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_call_median": g["call_ms"][len(g["call_ms"]) // 2],
        "ms_per_call_min": g["call_ms"][0],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16-mfma/f32-acc" if form == "mixed" else "f32",
        "data": "synthetic",
        "config": {
            "workload": "batch4: arrays 32x32, 64x64, 128x128 and 16x16-of-16x16 antennas, 64 channels each, "
            f"T=2048, 4-bit complex voltages (sky + noise), {form} form, one batched call as a HIP graph with one "
            "branch per array",
            "arrays": {w.name: {"N": w.N, "F": w.nchan, "T": w.T, "kernel": k} for w, k in zip(ws, g["kernels"])},
            "sample_format": "ci4",
            "form": form,
            "tune": args.tune,
            "schedules": g["schedules"],
        },
        "roofline": dict(per_array[dom.name]["roofline"],
                         note=f"main forward kernel of the dominant {dom.name} array, per-launch HIP events with the "
                         f"array alone ({per_array[dom.name]['ms_alone']:.3f} ms a call there)"),
        "roofline_call": {"bound": "mfma" if form == "mixed" else "alu", "achieved": round(call_achieved, 3),
                          "peak": call_peak, "unit": "TFLOP/s", "frac": round(call_achieved / call_peak, 4),
                          "algorithmic_flops_per_call": flops},
        "per_array": per_array,
        "cpu_baseline": cpu,
        "error_vs_oracle": err,
        "tolerance": {"fp32": 1e-5, "mixed": 2e-3},
        "sequential": {"ms_per_step": seq["ms"], "value": work / (seq["ms"] / 1e3),
                       "graph_speedup": seq["ms"] / ms},
    }
    if alt is not None:
        out[f"{other}_form"] = {"ms_per_step": alt["ms"], "value": work / (alt["ms"] / 1e3), "kernels": alt["kernels"]}
        out[f"speedup_vs_{other}_form"] = alt["ms"] / ms
    if not args.no_fold:
        log("bench: baseline fold and distributions")
        out["baseline_fold"] = bench_fold(omni, torch, skysim, args.steps, args.warmup,
                                          g["outs"][BATCH4.index("grid128")])
    if not args.no_fengine:
        log("bench: F-engine")
        out["fengine"] = bench_fengine(omni, torch, args.steps, args.warmup)
    if not args.no_hybrid:
        log("bench: hybrid tiles")
        out["hybrid_tiles"] = bench_hybrid(omni, torch, args.steps, args.warmup)
    if not args.no_beams:
        log("bench: beam-space variant")
        i16 = BATCH4.index("hier16x16")
        out["beam_space"] = bench_beams(omni, torch, ws[i16], raws[i16], args.steps, args.warmup,
                                        alone["hier16x16"]["ms"])
    print(json.dumps(out), flush=True)
    return 0


def cpu_oracle_baseline(raw_cpu, w, budget_s=10.0, max_channels=None):
    """Time the oracle (as it stands) on whole channels until ~budget_s of work."""
    max_channels = w.nchan if max_channels is None else max_channels
    import oracle

    T = raw_cpu.shape[0]
    done, t_used, results = 0, 0.0, {}
    while done < max_channels and (t_used < budget_s or done == 0):
        f = done
        sub = raw_cpu[:, f : f + 1].contiguous().numpy()
        t0 = time.perf_counter()
        x = oracle.decode(sub, w.dtype, T, 1, w.N)
        v = oracle.visibilities(x, w.dims)
        t_used += time.perf_counter() - t0
        results[f] = v.reshape(-1)
        done += 1
        log(f"cpu oracle: channel {f} done, {t_used:.1f} s so far")
    rate = w.N * T * done / t_used
    return rate, done, t_used, results


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch4",
                    help="batch4 (default), a workload name of skysim.WORKLOADS, fengine, baselines, hybrid or beams")
    ap.add_argument("--form", default=None, help="fp32 | mixed (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-other-form", action="store_true", help="time only the main form")
    ap.add_argument("--direct", action="store_true", help="also time the direct N^2 correlator at any N")
    ap.add_argument("--no-direct", action="store_true", help="never time the direct N^2 correlator")
    ap.add_argument("--tune", default="search", choices=["off", "search"],
                    help="plan-time autotuning of the schedules (default: search; planning is outside the timing)")
    ap.add_argument("--no-hybrid", action="store_true", help="skip the hybrid-tile measurement")
    ap.add_argument("--no-beams", action="store_true", help="skip the beam-space measurement")
    ap.add_argument("--no-fengine", action="store_true", help="skip the F-engine measurement")
    ap.add_argument("--no-fold", action="store_true", help="skip the baseline-fold measurements")
    ap.add_argument("--copy-calibration", action="store_true", help="only run 3 x 1 GiB device copies")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(
            "bench.py: the correlator runs on one GPU; a multi-GPU run (channels or time blocks sharded one per "
            f"GPU) is not implemented (asked for --gpus {args.gpus}, WORLD_SIZE {world})",
            file=sys.stderr,
        )
        return 2
    if args.copy_calibration:
        return copy_calibration()
    if args.workload == "batch4":
        return bench_batch4(args)
    if args.workload in ("fengine", "baselines", "hybrid", "beams"):
        return bench_aux(args)

    import numpy as np
    import torch

    import paper_0909_0001_amd as omni
    import skysim

    w = skysim.WORKLOADS[args.workload]
    form = args.form or w.form
    other = "mixed" if form == "fp32" else "fp32"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"bench: workload {w.name} N={w.N} F={w.nchan} T={w.T} {w.dtype} form={form}; generating voltages")
    raw = skysim.make_voltages(w, device=dev)
    torch.cuda.synchronize()

    main_res = run_form(omni, w, raw, form, args.steps, args.warmup, args.tune)
    alt = None
    if not args.no_other_form and not (other == "mixed" and w.dtype == "cf32"):
        alt = run_form(omni, w, raw, other, args.steps, args.warmup, args.tune)
    direct = None
    if w.dtype != "cf32" and not args.no_direct and (args.direct or w.N <= 16384):
        direct = run_direct(omni, w, raw, args.steps, args.warmup)
    work = w.antenna_samples()
    ms_per_step = main_res["ms"]
    value = work / (ms_per_step / 1e3)

    # Accuracy: zero lag of every channel against the exact total power; whole channels against the oracle.
    err = {}
    if w.dtype != "ci4":
        power = (raw.to(torch.float64) ** 2).sum(dim=(0, 2, 3))
        for tag, res in ((form, main_res), (other, alt), ("direct", direct)):
            if res is None:
                continue
            vh = res["vis"].reshape(w.nchan, -1)
            c = vh.shape[1] // 2
            err[f"{tag}_zero_lag_all_channels"] = float(((vh[:, c].real.double() - power).abs() / power).max())

    cpu = None
    if not args.no_cpu_baseline:
        raw_cpu = raw.cpu()
        rate, nch, secs, ref = cpu_oracle_baseline(raw_cpu, w, budget_s=args.cpu_budget)
        for tag, res in ((form, main_res), (other, alt), ("direct", direct)):
            if res is None:
                continue
            got = res["vis"].cpu().numpy().reshape(w.nchan, -1)
            c = got.shape[1] // 2
            e = max(float(np.max(np.abs(got[f] - ref[f])) / abs(ref[f][c])) for f in ref)
            err[f"{tag}_max_over_lags_vs_oracle_{nch}ch"] = e
        cpu = {
            "value": rate,
            "unit": "antenna-samples/s",
            "cores": len(os.sched_getaffinity(0)),
            "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{nch} of {w.nchan} channels x all {w.T} samples ({secs:.1f} s; float64 pair products "
            "by BLAS matmul + histogram by index difference)",
        }

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "antenna-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_call_median": main_res["stages"]["call_median"],
        "ms_per_call_min": main_res["stages"]["call_min"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if form == "fp32" else "f16-mfma/f32-acc",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: levels {w.level_dims}, N={w.N}, F={w.nchan}, T={w.T}, {w.dtype} voltages, "
            f"{form} form",
            "N": w.N,
            "F": w.nchan,
            "T": w.T,
            "sample_format": w.dtype,
            "form": form,
        },
        "roofline": roofline_of(w, main_res, work),
        "cpu_baseline": cpu,
        "error_vs_oracle": err,
        "tolerance": {"fp32": 1e-5, "mixed": 2e-3},
        "stage_ms": main_res["stages"],
    }
    if alt is not None:
        out["other_form"] = {
            "form": other,
            "config": f"{w.name}, same input bytes, {other} form",
            "value": work / (alt["ms"] / 1e3),
            "ms_per_step": alt["ms"],
            "stage_ms": alt["stages"],
            "roofline": roofline_of(w, alt, work),
            "speedup_vs_main_form": main_res["ms"] / alt["ms"],
        }
    if direct is not None:
        # int8 products of the pairs a <= b: 4 real products (2 ops each) per pair, sample and channel
        ops = 4.0 * w.N * (w.N + 1) * w.T * w.nchan
        tops = ops / (direct["ms"] / 1e3) / 1e12
        out["direct_n2"] = {
            "config": f"{w.name}, same input bytes, GPU direct N^2 correlator (int8 matrix cores, exact sums)",
            "value": work / (direct["ms"] / 1e3),
            "ms_per_step": direct["ms"],
            "int8_tops": round(tops, 2),
            "frac_of_int8_peak": round(tops / PEAK_INT8_MFMA_TOPS, 4),
            "speedup_of_main_form": direct["ms"] / main_res["ms"],
            "speedup_of_other_form": direct["ms"] / alt["ms"] if alt is not None else None,
        }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
