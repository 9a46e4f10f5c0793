#!/usr/bin/env python3
"""Throughput of the hierarchical-grid correlator on one MI355X.

One step = one omni_correlate call over the whole workload: every time sample
of every channel through the forward transform, |X|^2 and time integration,
then the inverse transform to visibilities.  Inputs are synthetic (seeded
sky-plus-noise voltages, quantised) and already resident in HBM.

Prints ONE JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "antenna-samples/s correlated (N·T·F/s) vs FP32 FFT form, at stated rel. err"
PEAK_FP32_VECTOR_TFLOPS = 157.3  # MI355X: 256 CUs x 4 SIMD x 16 lanes x 2 (packed) x 2 (FMA) x 2.4 GHz
PEAK_FP16_MFMA_TFLOPS = 2500.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fp32_form_flops_per_as(dims) -> float:
    """Fixed FP32 FFT-form work per antenna-sample: line-pruned FFT flops sum_p 2^p 10 log2 m_(p)
    over axes sorted by decreasing padded length, plus 4 * 2^d for |X|^2 and the time sum."""
    m = sorted((2 * n for n in dims if n > 1), reverse=True)
    d = len(m)
    return sum((2**p) * 10 * math.log2(mp) for p, mp in enumerate(m)) + 4 * 2**d


def cpu_oracle_baseline(raw_cpu, w, budget_s=10.0, max_channels=8):
    """Time the oracle (as it stands) on whole channels until ~budget_s of work."""
    import numpy as np

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
    ap.add_argument("--workload", default="hier8x8")
    ap.add_argument("--form", default=None, help="fp32 | mixed (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(
            "bench.py: the correlator runs on one GPU; a multi-GPU run (channels or time blocks sharded one per "
            f"GPU) is not part of this build (asked for --gpus {args.gpus}, WORLD_SIZE {world})",
            file=sys.stderr,
        )
        return 2

    import numpy as np
    import torch

    import paper_0909_0001_amd as omni
    import skysim

    w = skysim.WORKLOADS[args.workload]
    form = args.form or w.form
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"bench: workload {w.name} N={w.N} F={w.nchan} T={w.T} {w.dtype} form={form}; generating voltages")
    raw = skysim.make_voltages(w, device=dev)
    torch.cuda.synchronize()
    plan = omni.Plan(w.level_dims, w.A, w.nchan, w.dtype, form, timing=True)
    desc = json.loads(plan.describe())
    kernel_fwd = desc["arrays"][0]["kernel"] + "_kernel"
    log("bench: plan " + plan.describe())
    vis = torch.empty(plan.vis_shape(), dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream()

    for i in range(args.warmup):
        plan.correlate(raw, out=vis, stream=stream)
    torch.cuda.synchronize()
    log(f"bench: {args.warmup} warm-up steps done; timing {args.steps} steps")

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        plan.correlate(raw, out=vis, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    fwd = plan.stage_times("forward", args.steps)
    red = plan.stage_times("reduce", args.steps)
    inv = plan.stage_times("inverse", args.steps)
    fwd_ms = sum(fwd) / len(fwd)
    work = w.antenna_samples()
    value = work / (ms_per_step / 1e3)
    log(
        f"bench: {ms_per_step:.3f} ms/step (wall {wall / args.steps * 1e3:.3f}); forward kernel {fwd_ms:.3f} ms, "
        f"reduce {sum(red) / len(red):.3f} ms, inverse {sum(inv) / len(inv):.3f} ms"
    )

    flops_as = fp32_form_flops_per_as(w.dims)
    achieved = flops_as * work / (fwd_ms / 1e3) / 1e12
    roofline = {
        "bound": "alu",
        "achieved": round(achieved, 3),
        "peak": PEAK_FP32_VECTOR_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4),
        "traffic": None,
        "kernel": kernel_fwd,
        "kernel_ms": round(fwd_ms, 4),
        "algorithmic_flops_per_antenna_sample": flops_as,
    }

    # Accuracy: the zero lag of every channel against the exact total power.
    vh = vis.reshape(w.nchan, -1)
    c = vh.shape[1] // 2
    xf = raw.to(torch.float64)
    if w.dtype == "ci4":
        xf = None
    err = {}
    if xf is not None:
        power = (xf**2).sum(dim=(0, 2, 3))
        err["zero_lag_all_channels"] = float(((vh[:, c].real.double() - power).abs() / power).max())
        del xf

    cpu = None
    if not args.no_cpu_baseline:
        raw_cpu = raw.cpu()
        rate, nch, secs, ref = cpu_oracle_baseline(raw_cpu, w, budget_s=args.cpu_budget)
        got = vis.cpu().numpy().reshape(w.nchan, -1)
        e = max(float(np.max(np.abs(got[f] - ref[f])) / abs(ref[f][c])) for f in ref)
        err[f"max_abs_over_zero_lag_oracle_{nch}ch"] = e
        cpu = {
            "value": rate,
            "unit": "antenna-samples/s",
            "cores": len(os.sched_getaffinity(0)),
            "kind": "oracle",
            "sample": f"{nch} of {w.nchan} channels x all {w.T} samples ({secs:.1f} s, float64 pair products + binning)",
        }

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "antenna-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
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
        "roofline": roofline,
        "cpu_baseline": cpu,
        "error_vs_oracle": err,
        "stage_ms": {"forward": fwd_ms, "reduce": sum(red) / len(red), "inverse": sum(inv) / len(inv)},
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
