"""Parity of the HIP correlator with the CPU oracle, through the C ABI.

Tolerances: the float32 form must agree with the exact (float64) oracle to
1e-5 of the channel's zero-lag power, the mixed form to 2e-3 (per channel,
max over all lags):  err_f = max_Delta |V_gpu - V_oracle| / V_oracle_f[0].
"""

import math
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_0909_0001_amd as omni
import skysim
from tests.conftest import load_golden

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "mixed": 2e-3}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dims_of(level_dims):
    return [int(n) for ld in level_dims for n in ld]


def random_raw(dtype, T, F, N, gen, scale=1.0):
    if dtype == "cf32":
        return (torch.randn((T, F, N, 2), generator=gen) * scale).float()
    if dtype == "ci8":
        return torch.randint(-127, 128, (T, F, N, 2), generator=gen, dtype=torch.int16).to(torch.int8)
    re = torch.randint(-7, 8, (T, F, N), generator=gen, dtype=torch.int16)
    im = torch.randint(-7, 8, (T, F, N), generator=gen, dtype=torch.int16)
    return skysim.pack_ci4(re, im)


def oracle_vis(raw_cpu, dtype, level_dims):
    dims = dims_of(level_dims)
    T, F = raw_cpu.shape[0], raw_cpu.shape[1]
    x = oracle.decode(raw_cpu.numpy(), dtype, T, F, math.prod(dims))
    return oracle.visibilities(x, dims).reshape((F,) + tuple(2 * n - 1 for n in dims))


def rel_err(got, ref):
    F = ref.shape[0]
    g = got.reshape(F, -1)
    r = ref.reshape(F, -1)
    c = r.shape[1] // 2  # centre cell (Delta = 0) of an odd-sized row-major grid
    z = np.abs(r[:, c])
    z[z == 0] = 1.0
    return float(np.max(np.abs(g - r).max(axis=1) / z))


def gpu_vis(level_dims, raw_cpu, dtype, form="fp32", F=None, **kw):
    F = raw_cpu.shape[1] if F is None else F
    plan = omni.Plan(level_dims, None, F, dtype, form, **kw)
    vis = plan.correlate(raw_cpu.cuda())
    torch.cuda.synchronize()
    return vis.cpu().numpy(), plan


def chunk_count(plan, T, array=0):
    """Time chunks the plan's front passes take for T samples (1 for a grid without front passes)."""
    import json

    a = json.loads(plan.describe())["arrays"][array]
    return -(-T // a["chunk_T"]) if a["n_front"] else 1


# ---------------------------------------------------------------------------


def test_paper_example():
    """Sec. II.C worked example, run as a 1-level 2x3 plan and as a 9x1 plan with real voltages."""
    g = load_golden("paper_toy_example.txt")
    h = np.array(g["hypercube"], dtype=np.float32)
    raw = torch.zeros((1, 1, 6, 2), dtype=torch.float32)
    raw[0, 0, :, 0] = torch.from_numpy(h.ravel())
    say("paper example 2x3")
    vis, _ = gpu_vis([[2, 3]], raw, "cf32")
    want = np.array(g["vis_2d"])
    assert np.max(np.abs(vis[0] - want)) <= 1e-5 * 91
    v1 = np.array(g["voltages_1d"][0], dtype=np.float32)
    raw = torch.zeros((1, 1, 9, 2), dtype=torch.float32)
    raw[0, 0, :, 0] = torch.from_numpy(v1)
    say("paper example 9x1")
    vis, _ = gpu_vis([[9, 1]], raw, "cf32")
    assert np.max(np.abs(vis[0, :, 0] - np.array(g["vis_1d"][0]))) <= 1e-5 * 91


SHAPES = [
    [[4, 4]],
    [[3, 5]],
    [[7, 1]],
    [[1, 1]],
    [[2, 3], [4, 2]],
    [[8, 8]],
    [[6, 10]],
    [[16, 16]],
    [[32, 32]],
    [[5, 3], [3, 3]],
    [[2, 2], [2, 2], [2, 2]],
    [[4, 4], [4, 4]],
    [[8, 8], [8, 8]],
    [[3, 3], [3, 3], [5, 3]],
]


@pytest.mark.parametrize("dtype", ["cf32", "ci8", "ci4"])
@pytest.mark.parametrize("level_dims", SHAPES, ids=lambda s: "x".join(str(v) for ld in s for v in ld))
def test_random_shapes(level_dims, dtype):
    dims = dims_of(level_dims)
    N = math.prod(dims)
    gen = torch.Generator().manual_seed(N * 7 + len(dtype))
    T, F = 37, 3
    raw = random_raw(dtype, T, F, N, gen)
    say("shape", level_dims, dtype, "T", T, "F", F)
    vis, _ = gpu_vis(level_dims, raw, dtype)
    ref = oracle_vis(raw, dtype, level_dims)
    assert rel_err(vis, ref) <= TOL["fp32"]


def test_grid16_workload():
    """16x16 unit grid, 1 channel, T=1024 float voltages from 8 point sources + noise."""
    w = skysim.WORKLOADS["grid16"]
    raw = skysim.make_voltages(w)
    say("grid16 workload")
    vis, _ = gpu_vis(w.level_dims, raw, w.dtype)
    ref = oracle_vis(raw, w.dtype, w.level_dims)
    assert rel_err(vis, ref) <= TOL["fp32"]


def test_hier8x8_small_many_tiles():
    """The 8x8-of-8x8 geometry at full N with few samples and a ragged channel count."""
    w = skysim.WORKLOADS["hier8x8"]
    raw = skysim.make_voltages(w, T=75, nchan=5)
    say("hier8x8 T=75 F=5")
    vis, _ = gpu_vis(w.level_dims, raw, w.dtype)
    ref = oracle_vis(raw, w.dtype, w.level_dims)
    assert rel_err(vis, ref) <= TOL["fp32"]


def test_hier8x8_full_size():
    """Full 8x8-of-8x8 workload (F=64, T=4096, ci8): oracle on two channels, invariants on all 64."""
    w = skysim.WORKLOADS["hier8x8"]
    say("hier8x8 full size: generating")
    raw = skysim.make_voltages(w, device="cuda")
    plan = omni.Plan(w.level_dims, w.A, w.nchan, w.dtype, "fp32")
    say("hier8x8 full size: correlating")
    vis = plan.correlate(raw)
    torch.cuda.synchronize()
    vis_h = vis.cpu().numpy().reshape(w.nchan, -1)
    xf = raw.double()
    power = (xf**2).sum(dim=(0, 2, 3)).cpu().numpy()  # sum |x|^2 per channel
    s = xf.sum(dim=2)  # [T, F, 2] sum over antennas
    lagsum = (s**2).sum(dim=(0, 2)).cpu().numpy()  # sum_t |sum_a x|^2
    c = vis_h.shape[1] // 2
    assert np.max(np.abs(vis_h[:, c] - power) / power) <= TOL["fp32"]
    assert np.max(np.abs(vis_h.sum(axis=1) - lagsum) / power) <= TOL["fp32"] * 100
    for f in (0, 37):
        say("hier8x8 full size: oracle channel", f)
        sub = raw[:, f : f + 1].cpu()
        ref = oracle_vis(sub, w.dtype, w.level_dims)
        assert rel_err(vis_h[f : f + 1], ref) <= TOL["fp32"]


def test_empty_time_gives_zero():
    plan = omni.Plan([[4, 4]], None, 2, "ci8")
    out = torch.full(plan.vis_shape(), 7.0 + 1j, dtype=torch.complex64, device="cuda")
    plan.correlate_into(0, 0, out)
    torch.cuda.synchronize()
    assert not out.abs().max().item()


@pytest.mark.parametrize(
    "level_dims,T,split,form,chunk_T",
    [
        ([[4, 4], [2, 4]], 50, 20, "fp32", 0),  # general kernel
        ([[32, 32]], 50, 20, "fp32", 0),  # compile-time-shape kernel
        ([[2, 2], [8, 8], [4, 4]], 150, 70, "fp32", 32),  # front passes, 3 + 3 chunks, compile-time-shape kernel
        ([[4, 4], [4, 4], [4, 4]], 150, 70, "fp32", 32),  # front passes, 3 + 3 chunks, general kernel
        ([[8, 8], [8, 8]], 50, 21, "mixed", 0),  # 8x8x8x8 matrix-core kernel
        ([[2, 16], [16, 16]], 60, 25, "mixed", 8),  # front pass + (16,16,16) matrix-core kernel, 4 + 5 chunks
        ([[2, 2], [8, 8], [4, 4]], 60, 25, "mixed", 8),  # front passes + (8,8,4,4) matrix-core kernel
    ],
)
def test_split_integration_and_resume(level_dims, T, split, form, chunk_T):
    """T = T1 + T2 with OMNI_NO_RESET, and a checkpoint/resume of the accumulator, equal one call (front paths
    with several time chunks on both sides of the split)."""
    N = math.prod(dims_of(level_dims))
    gen = torch.Generator().manual_seed(5)
    raw = random_raw("ci8", T, 2, N, gen).cuda()
    say("split/resume", level_dims, form, T, split, "chunk_T", chunk_T)
    plan = omni.Plan(level_dims, None, 2, "ci8", form, chunk_T=chunk_T)
    if chunk_T:
        assert chunk_count(plan, split) >= 3 and chunk_count(plan, T - split) >= 3
    full = plan.correlate(raw).clone()
    plan.correlate(raw[:split].contiguous(), flags=omni.NO_FINALIZE)
    part = plan.correlate(raw[split:].contiguous(), flags=omni.NO_RESET)
    torch.cuda.synchronize()
    tol = 1e-6 if form == "fp32" else 1e-5  # the split changes the float32 blocks' rounding only
    assert torch.allclose(full, part, rtol=0, atol=tol * full.abs().max().item())
    # checkpoint after `split` samples, resume in a fresh plan
    plan.correlate(raw[:split].contiguous(), flags=omni.NO_FINALIZE)
    ck = np.zeros(plan.accumulator_bytes() // 8)
    plan.accumulator_get(ck)
    plan2 = omni.Plan(level_dims, None, 2, "ci8", form, chunk_T=chunk_T)
    plan2.accumulator_set(ck)
    resumed = plan2.correlate(raw[split:].contiguous(), flags=omni.NO_RESET)
    torch.cuda.synchronize()
    assert torch.allclose(full, resumed, rtol=0, atol=tol * full.abs().max().item())
    assert rel_err(resumed.cpu().numpy(), oracle_vis(raw.cpu(), "ci8", level_dims)) <= TOL[form]


def test_bitwise_deterministic():
    w = skysim.WORKLOADS["hier8x8"]
    raw = skysim.make_voltages(w, T=64, nchan=8).cuda()
    plan = omni.Plan(w.level_dims, None, 8, "ci8")
    a = plan.correlate(raw).clone()
    b = plan.correlate(raw).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_side_stream():
    gen = torch.Generator().manual_seed(9)
    raw = random_raw("cf32", 16, 2, 64, gen)
    ref = oracle_vis(raw, "cf32", [[8, 8]])
    plan = omni.Plan([[8, 8]], None, 2, "cf32")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        d = raw.cuda()
        out = plan.correlate(d, stream=s)
    s.synchronize()
    assert rel_err(out.cpu().numpy(), ref) <= TOL["fp32"]


def test_ci4_extremes():
    """All-extreme 4-bit samples (+-7, and -8 which the format can also hold)."""
    vals = torch.tensor([-8, -7, 7], dtype=torch.int16)
    gen = torch.Generator().manual_seed(11)
    T, F, N = 9, 2, 64
    re = vals[torch.randint(0, 3, (T, F, N), generator=gen)]
    im = vals[torch.randint(0, 3, (T, F, N), generator=gen)]
    raw = skysim.pack_ci4(re, im)
    vis, _ = gpu_vis([[8, 8]], raw, "ci4")
    assert rel_err(vis, oracle_vis(raw, "ci4", [[8, 8]])) <= TOL["fp32"]


# ---------------------------------------------------------------------------
# Mixed form (float16 MFMA stages with float32 accumulation).
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("dtype,time_block", [("ci8", 0), ("ci4", 0), ("ci8", 4)])
def test_mixed_hier8x8_small(dtype, time_block):
    """8x8-of-8x8 geometry, few samples, ragged channel count, both integer formats; a short float32 block
    makes the kernel add several blocks into its float64 partial sums."""
    w = skysim.WORKLOADS["hier8x8-mixed"]
    gen = torch.Generator().manual_seed(17)
    raw = random_raw(dtype, 75, 5, w.N, gen)
    say("mixed hier8x8 T=75 F=5", dtype, "time_block", time_block)
    vis, plan = gpu_vis(w.level_dims, raw, dtype, "mixed", time_block=time_block)
    assert '"fused8x4_mixed"' in plan.describe()
    ref = oracle_vis(raw, dtype, w.level_dims)
    err = rel_err(vis, ref)
    say("mixed error", err)
    assert err <= TOL["mixed"]


def test_mixed_sky_workload_full_size():
    """The full mixed-form workload (F=64, T=4096, ci8 sky + noise): oracle on two channels, zero lag on all."""
    w = skysim.WORKLOADS["hier8x8-mixed"]
    say("mixed full size: generating")
    raw = skysim.make_voltages(w, device="cuda")
    plan = omni.Plan(w.level_dims, w.A, w.nchan, w.dtype, "mixed")
    assert '"fused8x4_mixed"' in plan.describe()
    vis = plan.correlate(raw)
    torch.cuda.synchronize()
    vis_h = vis.cpu().numpy().reshape(w.nchan, -1)
    power = (raw.double() ** 2).sum(dim=(0, 2, 3)).cpu().numpy()
    c = vis_h.shape[1] // 2
    assert np.max(np.abs(vis_h[:, c] - power) / power) <= TOL["mixed"]
    for f in (3, 60):
        say("mixed full size: oracle channel", f)
        ref = oracle_vis(raw[:, f : f + 1].cpu(), w.dtype, w.level_dims)
        err = rel_err(vis_h[f : f + 1], ref)
        say("mixed full size error", f, err)
        assert err <= TOL["mixed"]


def test_mixed_other_shapes_fall_back_to_fp32_kernel():
    """Shapes (and sample formats) without a matrix-core kernel run the float32 kernels in a mixed plan."""
    gen = torch.Generator().manual_seed(23)
    raw = random_raw("ci8", 12, 2, 36, gen)
    vis, plan = gpu_vis([[6, 6]], raw, "ci8", "mixed")
    assert '"fused_fp32"' in plan.describe()
    assert rel_err(vis, oracle_vis(raw, "ci8", [[6, 6]])) <= TOL["fp32"]
    raw = random_raw("ci8", 12, 2, 1024, gen)
    vis, plan = gpu_vis([[32, 32]], raw, "ci8", "mixed")
    assert '"fused_ct_fp32"' in plan.describe()
    assert rel_err(vis, oracle_vis(raw, "ci8", [[32, 32]])) <= TOL["fp32"]


# ---------------------------------------------------------------------------
# Front mode (large per-channel grids) and the batched workload's shapes.
# ---------------------------------------------------------------------------


@pytest.mark.parametrize(
    "level_dims, dtype, T",
    [
        ([[4, 4], [4, 4], [4, 4]], "ci8", 150),
        ([[8, 8], [4, 4], [2, 2]], "cf32", 9),
        ([[4, 4], [4, 4], [4, 4]], "ci4", 7),
        ([[2, 2], [8, 8], [4, 4]], "ci8", 70),  # rest (8, 8, 4, 4): compile-time-shape kernel
    ],
)
def test_front_mode_full_oracle(level_dims, dtype, T):
    """Shapes whose grid needs front passes, at the planner's chunking (one chunk of up to 256 samples)."""
    N = math.prod(dims_of(level_dims))
    gen = torch.Generator().manual_seed(N + T)
    raw = random_raw(dtype, T, 3, N, gen)
    say("front mode", level_dims, dtype, T)
    vis, plan = gpu_vis(level_dims, raw, dtype)
    assert '"mode":"front"' in plan.describe()
    assert rel_err(vis, oracle_vis(raw, dtype, level_dims)) <= TOL["fp32"]


@pytest.mark.parametrize(
    "level_dims,dtype,form,T,chunk_T,kernel",
    [
        ([[4, 4], [4, 4], [4, 4]], "ci8", "fp32", 150, 40, "fused_fp32"),  # general kernel, 4 chunks
        ([[4, 4], [4, 4], [4, 4]], "ci4", "fp32", 7, 2, "fused_fp32"),  # ragged last chunk of 1 sample
        ([[2, 2], [8, 8], [4, 4]], "ci8", "fp32", 70, 20, "fused_ct_fp32"),  # compile-time-shape kernel
        ([[2, 16], [16, 16]], "ci4", "mixed", 9, 3, "fused16x3_mixed"),  # (16,16,16) matrix-core kernel
        ([[2, 16], [16, 16]], "ci8", "mixed", 70, 20, "fused16x3_mixed"),
        ([[2, 2], [8, 8], [4, 4]], "ci4", "mixed", 9, 3, "fused8844_mixed"),  # (8,8,4,4) matrix-core kernel
        ([[2, 2], [8, 8], [4, 4]], "ci8", "mixed", 70, 20, "fused8844_mixed"),
    ],
)
def test_front_chunks_full_oracle(level_dims, dtype, form, T, chunk_T, kernel):
    """Front passes over at least three time chunks (the later chunks add into the first chunk's partial sums,
    or the general kernel reduces after every chunk): every lag against the oracle."""
    N = math.prod(dims_of(level_dims))
    gen = torch.Generator().manual_seed(N + T + chunk_T)
    raw = random_raw(dtype, T, 2, N, gen)
    plan = omni.Plan(level_dims, None, 2, dtype, form, time_block=4, chunk_T=chunk_T)
    desc = plan.describe()
    say("front chunks", level_dims, dtype, form, "T", T, "chunk_T", chunk_T, desc[:160])
    assert f'"kernel":"{kernel}"' in desc
    assert chunk_count(plan, T) >= 3
    vis = plan.correlate(raw.cuda())
    torch.cuda.synchronize()
    err = rel_err(vis.cpu().numpy(), oracle_vis(raw, dtype, level_dims))
    say("front chunks error", err)
    assert err <= TOL[form]


@pytest.mark.parametrize(
    "level_dims,kernel",
    [
        ([[8, 8], [8, 8]], "fused8x4_mixed"),
        ([[2, 16], [16, 16]], "fused16x3_mixed"),
        ([[2, 2], [8, 8], [4, 4]], "fused8844_mixed"),
        ([[32, 32]], "grid32_mixed"),
        ([[64, 64]], "grid64_mixed"),
        ([[128, 128]], "grid128_mixed"),
    ],
)
def test_mixed_kernels_zero_and_one_sample(level_dims, kernel):
    """Each matrix-core kernel with T = 0 (the output is cleared) and T = 1 (one sample: the prologue and the
    software-pipelined loop run once, the loads that run ahead are clamped to that sample) against the oracle."""
    N = math.prod(dims_of(level_dims))
    plan = omni.Plan(level_dims, None, 2, "ci4", "mixed")
    assert f'"kernel":"{kernel}"' in plan.describe()
    out = torch.full(plan.vis_shape(), 7.0 + 1j, dtype=torch.complex64, device="cuda")
    plan.correlate_into(0, 0, out)
    torch.cuda.synchronize()
    assert not out.abs().max().item()
    gen = torch.Generator().manual_seed(N + 1)
    raw = random_raw("ci4", 1, 2, N, gen)
    say("one sample", level_dims, kernel)
    vis = plan.correlate(raw.cuda())
    torch.cuda.synchronize()
    err = rel_err(vis.cpu().numpy(), oracle_vis(raw, "ci4", level_dims))
    say("one sample error", err)
    assert err <= TOL["mixed"]


@pytest.mark.parametrize(
    "level_dims,dtype,kernel",
    [
        ([[8, 8], [8, 8]], "ci8", "fused8x4_mixed"),
        ([[2, 16], [16, 16]], "ci8", "fused16x3_mixed"),
        ([[2, 16], [16, 16]], "ci4", "fused16x3_mixed"),
        ([[32, 32]], "ci4", "grid32_mixed"),
    ],
)
def test_mixed_quiet_and_loud_channels(level_dims, dtype, kernel):
    """The mixed form applies no per-channel gain: a channel of unit-level samples (-1, 0, 1) beside one at the
    format's full scale, each within the tolerance of its own zero-lag power (float16 keeps its relative precision
    at any level, and the stage scales keep a unit sample out of its subnormal range)."""
    dims = dims_of(level_dims)
    N = math.prod(dims)
    T, F = 9, 2
    gen = torch.Generator().manual_seed(N + len(dtype))
    full = 127 if dtype == "ci8" else 7
    parts = [torch.randint(lo, hi + 1, (T, 1, N, 2), generator=gen, dtype=torch.int16) for lo, hi in ((-1, 1), (-full, full))]
    x = torch.cat(parts, dim=1)
    raw = x.to(torch.int8).contiguous() if dtype == "ci8" else skysim.pack_ci4(x[..., 0], x[..., 1])
    say("quiet and loud channels", level_dims, dtype)
    vis, plan = gpu_vis(level_dims, raw, dtype, form="mixed")
    assert f'"kernel":"{kernel}"' in plan.describe()
    err = rel_err(vis, oracle_vis(raw, dtype, level_dims))
    say("quiet and loud channels error", err)
    assert err <= TOL["mixed"]


@pytest.mark.parametrize("dtype", ["ci4", "cf32"])
def test_front_pass_fold_by_four(dtype):
    """A front axis of 32 antennas (m = 64, folded into four residue classes of 16-point DFTs) on the
    32x32-of-16x16 array (N = 262144, M = 4.2M cells), over three time chunks: sampled cells against the oracle."""
    level_dims = [[32, 32], [16, 16]]
    dims = dims_of(level_dims)
    N = math.prod(dims)
    T, F = 3, 1
    gen = torch.Generator().manual_seed(N + len(dtype))
    raw = random_raw(dtype, T, F, N, gen)
    plan = omni.Plan(level_dims, None, F, dtype, "fp32", chunk_T=1)
    desc = plan.describe()
    say("fold by four", dtype, desc[:200])
    assert '"mode":"front"' in desc and '"n_front":1' in desc  # the front pass takes the first axis (32 antennas)
    assert chunk_count(plan, T) >= 3
    vis = plan.correlate(raw.cuda())
    torch.cuda.synchronize()
    x = oracle.decode(raw.numpy(), dtype, T, F, N)
    check_cells(vis.cpu().numpy(), x, dims, "fp32", n_random=64, seed=N, tag="fold by four " + dtype)


@pytest.mark.parametrize("shape", [[[64, 64]], [[128, 128]]])
def test_large_single_level_grids(shape):
    N = math.prod(dims_of(shape))
    gen = torch.Generator().manual_seed(N)
    raw = random_raw("ci4", 6, 2, N, gen)
    say("single level", shape)
    vis, _ = gpu_vis(shape, raw, "ci4")
    assert rel_err(vis, oracle_vis(raw, "ci4", shape)) <= TOL["fp32"]


def check_cells(V, x, dims, form, n_random=256, seed=0, tag=""):
    """The oracle one cell at a time (all |Delta_k| <= 1 plus ``n_random`` random cells), and a few Fourier cells
    of the visibility grid against the oracle's time-summed power (Wiener-Khinchin).  V: [F, 2n_1-1, ...]."""
    F = V.shape[0]
    rng = np.random.default_rng(seed)
    near = np.array(np.meshgrid(*[[-1, 0, 1]] * len(dims), indexing="ij")).reshape(len(dims), -1).T
    far = np.stack([rng.integers(-(n - 1), n, n_random) for n in dims], axis=1)
    deltas = np.concatenate([near, far])
    ref = oracle.visibility_cells(x, dims, deltas)
    got = np.stack([V[(slice(None),) + tuple(dl + np.array(dims) - 1)] for dl in deltas], axis=1)
    z = np.abs(ref[:, len(near) // 2])  # Delta = 0 is the centre of the near block
    err = float(np.max(np.abs(got - ref) / z[:, None]))
    say(tag, "sampled-cell error", err, "over", len(deltas), "cells")
    assert err <= TOL[form]
    kap = rng.integers(0, 2 * np.array(dims), (3, len(dims)))
    P = oracle.fourier_power(x, dims, kap)
    G = np.meshgrid(*[np.arange(-(n - 1), n) for n in dims], indexing="ij", sparse=True)
    for q, k in enumerate(kap):
        ph = sum(kk * g / (2 * n) for kk, g, n in zip(k, G, dims))
        wk = np.exp(-2j * np.pi * ph)
        for f in range(F):
            val = np.sum(V[f].astype(np.complex128) * wk)
            assert abs(val - P[f, q]) <= (1e-4 if form == "fp32" else 2e-3) * np.sum(np.abs(x[:, f]) ** 2), (f, k)


def sampled_cells_check(w, T, F, n_random=256, seed=0, form="fp32", kernel=None, chunk_T=0):
    """Full-size geometry, few samples: the oracle one cell at a time, and Fourier cells (check_cells)."""
    dims = w.dims
    raw = skysim.make_voltages(w, T=T, nchan=F, device="cuda")
    plan = omni.Plan(w.level_dims, w.A, F, w.dtype, form, chunk_T=chunk_T)
    desc = plan.describe()
    say(w.name, desc[:200])
    if kernel:
        assert f'"kernel":"{kernel}"' in desc
    if chunk_T:
        assert chunk_count(plan, T) >= 3
    vis = plan.correlate(raw)
    torch.cuda.synchronize()
    x = oracle.decode(raw.cpu().numpy(), w.dtype, T, F, w.N)
    check_cells(vis.cpu().numpy(), x, dims, form, n_random, seed, w.name)


def test_hier3_sampled_cells():
    """The three-level 16x16 / 8x8 / 4x4 hierarchy (N = 262144, M = 16.8M cells) at full N, 3 time chunks."""
    sampled_cells_check(skysim.WORKLOADS["hier3"], T=12, F=2, chunk_T=4)


def test_hier16x16_sampled_cells():
    """The two-level 16x16-of-16x16 array of the batched workload (N = 65536, M = 1M cells)."""
    sampled_cells_check(skysim.WORKLOADS["hier16x16"], T=10, F=3)


def test_mixed_16x3_small_full_oracle():
    """Mixed form behind a front pass: (2, 16, 16, 16) grid (float16 front workspace, the (16,16,16) matrix-core
    kernel), every lag against the oracle, several float32 time blocks in one chunk."""
    level_dims = [[2, 16], [16, 16]]
    N = math.prod(dims_of(level_dims))
    for dtype, T in (("ci4", 7), ("ci8", 70)):
        gen = torch.Generator().manual_seed(N + T)
        raw = random_raw(dtype, T, 2, N, gen)
        say("mixed 16x3", level_dims, dtype, T)
        vis, plan = gpu_vis(level_dims, raw, dtype, form="mixed", time_block=16)
        assert '"kernel":"fused16x3_mixed"' in plan.describe()
        err = rel_err(vis, oracle_vis(raw, dtype, level_dims))
        say("mixed 16x3 error", err)
        assert err <= TOL["mixed"]


def test_mixed_8844_small_full_oracle():
    """Mixed form behind two front passes: (2, 2, 8, 8, 4, 4) grid (float16 front workspace, the (8,8,4,4)
    matrix-core kernel), every lag against the oracle, several float32 time blocks in one chunk."""
    level_dims = [[2, 2], [8, 8], [4, 4]]
    N = math.prod(dims_of(level_dims))
    for dtype, T in (("ci4", 9), ("ci8", 70)):
        gen = torch.Generator().manual_seed(N + T + 1)
        raw = random_raw(dtype, T, 2, N, gen)
        say("mixed 8844", level_dims, dtype, T)
        vis, plan = gpu_vis(level_dims, raw, dtype, form="mixed", time_block=16)
        assert '"kernel":"fused8844_mixed"' in plan.describe()
        err = rel_err(vis, oracle_vis(raw, dtype, level_dims))
        say("mixed 8844 error", err)
        assert err <= TOL["mixed"]


def test_mixed_hier3_sampled_cells():
    """The three-level hierarchy in the mixed form at full N (fused 16x16 front pass, 3 time chunks): sampled
    cells and Fourier cells."""
    sampled_cells_check(skysim.WORKLOADS["hier3"], T=12, F=2, form="mixed", kernel="fused8844_mixed", chunk_T=4)


def test_mixed_hier16x16_sampled_cells():
    """The 16x16-of-16x16 array in the mixed form at full N (4 time chunks): sampled cells and Fourier cells."""
    sampled_cells_check(skysim.WORKLOADS["hier16x16"], T=10, F=3, form="mixed", kernel="fused16x3_mixed", chunk_T=3)


@pytest.mark.parametrize("level_dims,kernel", [([[32, 32]], "fused_ct_fp32"), ([[16, 32]], "fused_fp32")])
def test_autotuned_plan_matches_oracle(level_dims, kernel):
    """A plan made with the autotuner still agrees with the oracle (schedule only changes speed)."""
    gen = torch.Generator().manual_seed(31)
    N = math.prod(level_dims[0])
    raw = random_raw("ci4", 21, 2, N, gen)
    plan = omni.Plan(level_dims, None, 2, "ci4", "fp32", tune=True)
    d = plan.describe()
    say("tuned", d)
    assert f'"kernel":"{kernel}"' in d
    assert '"tuned_ms":0.000000' not in d
    vis = plan.correlate(raw.cuda())
    torch.cuda.synchronize()
    assert rel_err(vis.cpu().numpy(), oracle_vis(raw, "ci4", level_dims)) <= TOL["fp32"]


@pytest.mark.parametrize(
    "level_dims,dtype,form,kernel",
    [
        ([[32, 32]], "ci4", "mixed", "grid32_mixed"),
        ([[64, 64]], "ci4", "mixed", "grid64_mixed"),
        ([[128, 128]], "ci4", "mixed", "grid128_mixed"),
        ([[8, 8], [8, 8]], "ci8", "mixed", "fused8x4_mixed"),
        ([[8, 8], [8, 8]], "ci8", "fp32", "fused8x4_fp32"),
    ],
)
def test_autotuned_sliced_kernels(level_dims, dtype, form, kernel, tmp_path):
    """The autotuner's search over time slicing x float32 block of the fixed-shape kernels: the tuned plan
    agrees with the oracle, its schedule is stored in the cache file, and a plan made from the cache takes the
    same schedule without searching.  The float32 form keeps its 64-sample block."""
    import json

    gen = torch.Generator().manual_seed(41)
    N = math.prod(dims_of(level_dims))
    T = 40
    raw = random_raw(dtype, T, 2, N, gen)
    cache = str(tmp_path / "tune.txt")
    plan = omni.Plan(level_dims, None, 2, dtype, form, tune="search", tune_cache=cache)
    a = json.loads(plan.describe())["arrays"][0]
    say("tuned", kernel, a["wg_target"], a["block"], a["tuned_ms"])
    assert a["kernel"] == kernel and a["tuned_ms"] > 0
    assert a["block"] in ((256, 1024) if form == "mixed" else (64,))
    vis = plan.correlate(raw.cuda())
    torch.cuda.synchronize()
    N_full = 4096  # above this, the oracle one cell at a time
    if N <= N_full:
        ref_err = lambda v: rel_err(v, oracle_vis(raw, dtype, level_dims))  # noqa: E731
    else:
        x = oracle.decode(raw.numpy(), dtype, T, 2, N)
        ref_err = lambda v: check_cells(v, x, dims_of(level_dims), form, 256, 5, kernel) or 0.0  # noqa: E731
    assert ref_err(vis.cpu().numpy()) <= TOL[form]
    line = open(cache).read().split()
    assert int(line[1]) == a["block"] and int(line[2]) == a["wg_target"]
    again = omni.Plan(level_dims, None, 2, dtype, form, tune="cache", tune_cache=cache)
    b = json.loads(again.describe())["arrays"][0]
    assert (b["wg_target"], b["block"], b["tuned_ms"]) == (a["wg_target"], a["block"], 0.0)
    vis2 = again.correlate(raw.cuda())
    torch.cuda.synchronize()
    assert torch.equal(vis2, vis)  # same schedule, same launch, same bytes


@pytest.mark.parametrize(
    "level_dims,dtype,kernel",
    [
        ([[32, 32]], "ci4", "fused_ct_fp32"),
        ([[64, 64]], "ci8", "fused_ct_fp32"),
        ([[32, 32]], "cf32", "fused_ct_fp32"),
        ([[2, 2], [8, 8], [4, 4]], "ci8", "fused_ct_fp32"),  # front pass on a word-unaligned source
        ([[4, 4], [4, 4], [4, 4]], "ci4", "fused_fp32"),
    ],
)
def test_unaligned_input_pointer(level_dims, dtype, kernel):
    """A source pointer that is 4- but not 16-byte aligned takes the unstaged loads and gives the same result."""
    N = math.prod(dims_of(level_dims))
    gen = torch.Generator().manual_seed(N + 7)
    raw = random_raw(dtype, 11, 2, N, gen)
    flat = raw.reshape(-1)
    pad = 4 // raw.element_size()  # 4 bytes: the library accepts 4-byte aligned sources
    big = torch.empty(flat.numel() + pad, dtype=raw.dtype, device="cuda")
    big[pad:].copy_(flat.cuda())
    shifted = big[pad:].view(raw.shape)
    assert shifted.data_ptr() % 16 != 0 and shifted.is_contiguous()
    say("unaligned", level_dims, dtype, shifted.data_ptr() % 16)
    plan = omni.Plan(level_dims, None, 2, dtype, "fp32")
    assert f'"kernel":"{kernel}"' in plan.describe()
    got = plan.correlate(shifted)
    ref = plan.correlate(raw.cuda())
    torch.cuda.synchronize()
    assert rel_err(got.cpu().numpy(), ref.cpu().numpy()) <= 1e-6
    assert rel_err(got.cpu().numpy(), oracle_vis(raw, dtype, level_dims)) <= TOL["fp32"]


BATCH = [([[8, 8]], None, 3), ([[4, 4], [4, 4]], None, 2), ([[32, 32]], None, 2), ([[2, 2], [8, 8], [4, 4]], None, 2)]


def batch_raw(dtype, T, seed):
    gen = torch.Generator().manual_seed(seed)
    return [random_raw(dtype, T, F, math.prod(dims_of(ld)), gen) for ld, _, F in BATCH]


def test_batch_plan_matches_oracle_per_array():
    """One batch plan over arrays of different shapes equals the oracle array by array."""
    raws = batch_raw("ci8", 23, 5)
    plan = omni.Plan(batch=BATCH, dtype="ci8")
    say("batch", [ld for ld, _, _ in BATCH])
    outs = plan.correlate_batch([r.cuda() for r in raws])
    torch.cuda.synchronize()
    for (ld, _, _), r, o in zip(BATCH, raws, outs):
        assert rel_err(o.cpu().numpy(), oracle_vis(r, "ci8", ld)) <= TOL["fp32"]


def test_graph_batch_replays_match_sequential():
    """A graph plan (arrays as parallel branches of one captured graph) gives the sequential plan's bytes on
    every replay, with eager work and synchronisations between replays; a call of another shape is refused."""
    raws = batch_raw("ci4", 41, 6)
    volts = [r.cuda() for r in raws]
    seq = omni.Plan(batch=BATCH, dtype="ci4")
    ref = [o.clone() for o in seq.correlate_batch(volts)]
    gp = omni.Plan(batch=BATCH, dtype="ci4", graph=True, timing=True)
    outs = [torch.empty(gp.vis_shape(i), dtype=torch.complex64, device="cuda") for i in range(len(BATCH))]
    for rep in range(4):
        for o in outs:
            o.zero_()
        gp.correlate_batch(volts, outs=outs)
        junk = torch.randn(1 << 20, device="cuda") * 2.0  # eager work between replays
        torch.cuda.synchronize()
        del junk
        for a, b in zip(outs, ref):
            assert torch.equal(a, b), f"replay {rep}"
    assert len(gp.stage_times("call")) == 4
    with pytest.raises(omni.OmniError):
        gp.stage_times("forward")
    # another T is refused before anything is captured
    with pytest.raises(omni.OmniError) as ei:
        gp.correlate_batch([v[:17].contiguous() for v in volts])
    assert omni.STATUS[ei.value.code] == "OMNI_E_STATE"
    # the plan still replays its call afterwards
    gp.correlate_batch(volts, outs=outs)
    torch.cuda.synchronize()
    for a, b in zip(outs, ref):
        assert torch.equal(a, b)


def test_graph_batch_without_outs_reuses_its_outputs():
    """Calls of a graph plan without ``outs`` replay one captured graph: the binding hands back the same output
    tensors every time (the graph writes fixed addresses), and each call's result equals the sequential plan's."""
    raws = batch_raw("ci4", 23, 4)
    volts = [r.cuda() for r in raws]
    ref = [o.clone() for o in omni.Plan(batch=BATCH, dtype="ci4").correlate_batch(volts)]
    gp = omni.Plan(batch=BATCH, dtype="ci4", graph=True)
    first = gp.correlate_batch(volts)
    torch.cuda.synchronize()
    snap = [o.clone() for o in first]
    second = gp.correlate_batch(volts)
    torch.cuda.synchronize()
    assert all(a.data_ptr() == b.data_ptr() for a, b in zip(first, second))
    for a, b, r in zip(snap, second, ref):
        assert torch.equal(a, r) and torch.equal(b, r)


@pytest.mark.skip(reason="re-capturing a live graph plan crashed the process on the GPU (a segfault inside the "
                  "fourth capture of one plan, cause not found); re-capture is switched off and returns OMNI_E_STATE")
def test_graph_batch_recapture():
    """A graph plan re-captured for a new T, then for a split integration (NO_FINALIZE, then NO_RESET)."""
    raws = batch_raw("ci4", 41, 6)
    volts = [r.cuda() for r in raws]
    seq = omni.Plan(batch=BATCH, dtype="ci4")
    gp = omni.Plan(batch=BATCH, dtype="ci4", graph=True)
    gp.correlate_batch(volts)
    short = [v[:17].contiguous() for v in volts]
    ref2 = [o.clone() for o in seq.correlate_batch(short)]
    got2 = gp.correlate_batch(short)
    torch.cuda.synchronize()
    for a, b in zip(got2, ref2):
        assert torch.equal(a, b)
    gp.correlate_batch([v[:20].contiguous() for v in volts], flags=omni.NO_FINALIZE)
    got3 = gp.correlate_batch([v[20:].contiguous() for v in volts], flags=omni.NO_RESET)
    torch.cuda.synchronize()
    for (ld, _, _), r, o in zip(BATCH, raws, got3):
        assert rel_err(o.cpu().numpy(), oracle_vis(r, "ci4", ld)) <= TOL["fp32"]


def test_graph_batch_resumes_an_integration():
    """A graph plan continues (OMNI_NO_RESET) an integration checkpointed from another plan through
    omni_accumulator_get / set."""
    raws = batch_raw("ci8", 41, 8)
    volts = [r.cuda() for r in raws]
    first = omni.Plan(batch=BATCH, dtype="ci8")
    first.correlate_batch([v[:20].contiguous() for v in volts], flags=omni.NO_FINALIZE)
    torch.cuda.synchronize()
    second = omni.Plan(batch=BATCH, dtype="ci8", graph=True)
    nb = first.accumulator_bytes()
    assert second.accumulator_bytes() == nb
    ck = np.zeros(nb // 8)
    first.accumulator_get(ck)
    second.accumulator_set(ck)
    got = second.correlate_batch([v[20:].contiguous() for v in volts], flags=omni.NO_RESET)
    torch.cuda.synchronize()
    for (ld, _, _), r, o in zip(BATCH, raws, got):
        assert rel_err(o.cpu().numpy(), oracle_vis(r, "ci8", ld)) <= TOL["fp32"]


# ---------------------------------------------------------------------------
# GPU direct N^2 correlator (comparison baseline): exact integer sums, rounded once to float32


def assert_rounded_once(got, ref):
    """Each component of `got` is the float32 rounding of the exact `ref` (|error| <= 2^-24 |ref|)."""
    got = got.astype(np.complex128)
    for part in (np.real, np.imag):
        g, r = part(got), part(ref)
        assert np.all(np.abs(g - r) <= np.abs(r) * 2.0**-24), float(np.max(np.abs(g - r)))


@pytest.mark.parametrize("dtype", ["ci8", "ci4"])
@pytest.mark.parametrize(
    "level_dims,T,F",
    [([[16, 16]], 77, 3), ([[4, 4], [4, 4]], 40, 2), ([[2, 8], [4, 4]], 33, 1), ([[8, 16]], 1, 2),
     ([[2, 2], [4, 4], [2, 4]], 35, 2)],
    ids=["16x16", "4x4x4x4", "2x8x4x4", "8x16_T1", "2x2x4x4x2x4"],
)
def test_direct_correlator_matches_oracle(level_dims, T, F, dtype):
    gen = torch.Generator().manual_seed(11)
    N = math.prod(dims_of(level_dims))
    raw = random_raw(dtype, T, F, N, gen)
    say("direct correlator", level_dims, dtype, "T", T, "F", F)
    plan = omni.Plan(level_dims, None, F, dtype, "fp32")
    vis = plan.direct_correlate(raw.cuda())
    torch.cuda.synchronize()
    assert_rounded_once(vis.cpu().numpy(), oracle_vis(raw, dtype, level_dims))


def test_direct_correlator_extremes_two_launches():
    """ci8 -128 everywhere over T = 40000 > 32768 samples (two launches, largest int32 pair sums)."""
    T, F, level_dims = 40000, 1, [[8, 16]]
    raw = torch.full((T, F, 128, 2), -128, dtype=torch.int8)
    raw[::3, :, ::5, 1] = 127
    say("direct correlator extremes T", T)
    plan = omni.Plan(level_dims, None, F, "ci8", "fp32")
    vis = plan.direct_correlate(raw.cuda())
    torch.cuda.synchronize()
    assert_rounded_once(vis.cpu().numpy(), oracle_vis(raw, "ci8", level_dims))


def test_direct_correlator_empty_and_errors():
    plan = omni.Plan([[16, 16]], None, 2, "ci8", "fp32")
    vis = plan.direct_correlate(torch.zeros((0, 2, 256, 2), dtype=torch.int8, device="cuda"))
    torch.cuda.synchronize()
    assert not vis.abs().any()
    with pytest.raises(omni.OmniError) as e:
        omni.Plan([[16, 16]], None, 1, "cf32", "fp32").direct_correlate(torch.zeros((4, 1, 256, 2), device="cuda"))
    assert e.value.code == -7  # OMNI_E_STATE: float samples
    with pytest.raises(omni.OmniError, match="multiple of 128"):
        omni.Plan([[10, 10]], None, 1, "ci8", "fp32").direct_correlate(
            torch.zeros((4, 1, 100, 2), dtype=torch.int8, device="cuda"))


def test_direct_correlator_agrees_with_fft_forms_full_size():
    """hier8x8 at full size (F=64, T=4096, ci8): direct (exact) vs the float32 and mixed FFT forms."""
    w = skysim.WORKLOADS["hier8x8"]
    say("direct correlator vs FFT forms: hier8x8 full size")
    raw = skysim.make_voltages(w, device="cuda")
    d = omni.Plan(w.level_dims, w.A, w.nchan, w.dtype, "fp32").direct_correlate(raw)
    for form in ("fp32", "mixed"):
        v = omni.Plan(w.level_dims, w.A, w.nchan, w.dtype, form).correlate(raw)
        torch.cuda.synchronize()
        e = rel_err(v.cpu().numpy(), d.cpu().numpy().astype(np.complex128))
        say("direct vs", form, e)
        assert e <= TOL[form]
    xf = raw.double()
    power = (xf**2).sum(dim=(0, 2, 3)).cpu().numpy()
    dh = d.cpu().numpy().reshape(w.nchan, -1)
    assert np.array_equal(dh[:, dh.shape[1] // 2].real, power.astype(np.float32))


@pytest.mark.parametrize("perm", [(1, 0, 3, 2), (2, 3, 0, 1)], ids=["swap_xy", "swap_levels"])
def test_axis_permutation_equivariance(perm):
    """Permuting the antenna axes (within or between levels) permutes the visibility axes."""
    level_dims, T, F = [[4, 8], [2, 4]], 48, 2
    dims = dims_of(level_dims)
    gen = torch.Generator().manual_seed(5)
    raw = random_raw("ci8", T, F, math.prod(dims), gen)
    vis, _ = gpu_vis(level_dims, raw, "ci8")
    pdims = [dims[k] for k in perm]
    praw = raw.reshape(T, F, *dims, 2).permute(0, 1, *[2 + k for k in perm], 2 + len(dims)).contiguous()
    praw = praw.reshape(T, F, -1, 2)
    plevels = [[pdims[0], pdims[1]], [pdims[2], pdims[3]]]
    pvis, _ = gpu_vis(plevels, praw, "ci8")
    want = np.transpose(vis, (0,) + tuple(1 + k for k in perm))
    assert rel_err(pvis, want) <= TOL["fp32"]


@pytest.mark.parametrize("name", ["hier16x16", "hier3"])
def test_fft_forms_against_direct_full_size(name):
    """Every cell at full size: both FFT forms against the exact direct correlator (integer sums, rounded once)."""
    w = skysim.WORKLOADS[name]
    say(name, "full size: generating")
    raw = skysim.make_voltages(w, device="cuda")
    say(name, "full size: direct correlator")
    d = omni.Plan(w.level_dims, w.A, w.nchan, w.dtype, "fp32").direct_correlate(raw).reshape(w.nchan, -1)
    torch.cuda.synchronize()
    z = d[:, d.shape[1] // 2].real.double()
    power = torch.zeros(w.nchan, dtype=torch.float64, device="cuda")
    for f in range(w.nchan):  # exact total power per channel: sum |x|^2 of the ci4 samples
        b = raw[:, f].to(torch.int16)
        re, im = ((b << 8) >> 12).double(), ((b << 12) >> 12).double()  # signed high and low nibbles
        power[f] = (re * re + im * im).sum()
    assert torch.equal(z, power.float().double())
    for form in ("fp32", "mixed"):
        say(name, "full size:", form)
        v = omni.Plan(w.level_dims, w.A, w.nchan, w.dtype, form).correlate(raw).reshape(w.nchan, -1)
        torch.cuda.synchronize()
        e = float(((v - d).abs().amax(dim=1).double() / z).max())
        say(name, form, "max |V - V_direct| / V[0]:", e)
        assert e <= TOL[form]
        del v


# ---------------------------------------------------------------------------
# Every cell of a full-size three-level grid against the oracle, on a subset of the input (2 channels x 16
# samples of the three-level workload's bytes), and the batched workload's four shapes as one mixed graph plan.


@pytest.fixture(scope="module")
def hier3_subset():
    w = skysim.WORKLOADS["hier3"]
    T, F = 16, 2
    raw = skysim.make_voltages(w, T=T, nchan=F, device="cuda")
    x = oracle.decode(raw.cpu().numpy(), w.dtype, T, F, w.N)
    say("hier3 subset: oracle on every cell (pair sum grouped by the outer level's lag)")
    ref = oracle.visibilities_by_outer_lag(x, w.dims, 2)
    say("hier3 subset: oracle done")
    return w, raw, ref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("form,kernel", [("mixed", "fused8844_mixed"), ("fp32", "fused_ct_fp32")])
def test_hier3_every_cell_on_input_subset(hier3_subset, form, kernel):
    """N = 262144 at full size, 2 channels x T = 16 in 4 time chunks (5 + 5 + 5 + 1 samples): all 10.6M cells
    per channel against the exact oracle."""
    w, raw, ref = hier3_subset
    plan = omni.Plan(w.level_dims, w.A, 2, w.dtype, form, chunk_T=5)
    assert f'"kernel":"{kernel}"' in plan.describe()
    assert chunk_count(plan, 16) == 4
    say("hier3 subset:", form)
    vis = plan.correlate(raw)
    torch.cuda.synchronize()
    err = rel_err(vis.cpu().numpy(), ref)
    say("hier3 subset", form, "max error / zero lag over every cell", err)
    assert err <= TOL[form]


C5_SHAPES = [[[32, 32]], [[64, 64]], [[128, 128]], [[16, 16], [16, 16]]]


@pytest.mark.timeout(600)
def test_mixed_batch_graph_c5_shapes():
    """The batched workload's four arrays (32x32, 64x64, 128x128, 16x16-of-16x16) as one mixed-form graph plan at
    reduced T and F: every lag of 32x32 and 64x64 against the oracle, sampled and Fourier cells of 128x128 and of
    16^4 (3 time chunks); replays equal; a split integration (NO_FINALIZE then NO_RESET) in a second graph plan."""
    T, F = 40, 2
    gen = torch.Generator().manual_seed(2048)
    raws = [random_raw("ci4", T, F, math.prod(dims_of(ld)), gen) for ld in C5_SHAPES]
    volts = [r.cuda() for r in raws]
    batch = [(ld, None, F) for ld in C5_SHAPES]
    gp = omni.Plan(batch=batch, dtype="ci4", form="mixed", graph=True, chunk_T=16)
    say("c5 mixed graph", gp.describe()[:400])
    assert chunk_count(gp, T, 3) >= 3
    outs = gp.correlate_batch(volts)
    torch.cuda.synchronize()
    first = [o.clone() for o in outs]
    for ld, r, o in zip(C5_SHAPES, raws, first):
        dims = dims_of(ld)
        x = oracle.decode(r.numpy(), "ci4", T, F, math.prod(dims))
        if math.prod(dims) <= 4096:
            err = rel_err(o.cpu().numpy(), oracle.visibilities(x, dims).reshape(o.shape))
            say("c5 mixed graph", ld, "every lag", err)
            assert err <= TOL["mixed"]
        else:
            check_cells(o.cpu().numpy(), x, dims, "mixed", 256, 7, f"c5 mixed graph {ld}")
    # a replay without outputs reuses the plan's output tensors and gives the same bytes
    again = gp.correlate_batch(volts)
    torch.cuda.synchronize()
    assert all(a.data_ptr() == b.data_ptr() for a, b in zip(again, outs))
    assert all(torch.equal(a, b) for a, b in zip(again, first))
    # split integration through two graph plans (one per call shape)
    gp1 = omni.Plan(batch=batch, dtype="ci4", form="mixed", graph=True, chunk_T=16)
    gp2 = omni.Plan(batch=batch, dtype="ci4", form="mixed", graph=True, chunk_T=16)
    gp1.correlate_batch([v[:17].contiguous() for v in volts], flags=omni.NO_FINALIZE)
    ck = torch.empty(gp1.accumulator_bytes() // 8, dtype=torch.float64, device="cuda")
    gp1.accumulator_get(ck)
    gp2.accumulator_set(ck)
    split = gp2.correlate_batch([v[17:].contiguous() for v in volts], flags=omni.NO_RESET)
    torch.cuda.synchronize()
    for ld, a, b in zip(C5_SHAPES, split, first):
        e = rel_err(a.cpu().numpy(), b.cpu().numpy().astype(np.complex128))
        say("c5 mixed graph split vs whole", ld, e)
        assert e <= 1e-5


# ---------------------------------------------------------------------------
# Matrix-core kernels of the single-level grids (mixed form).


@pytest.mark.parametrize(
    "level_dims,T,F,time_block,kernel",
    [
        ([[128, 128]], 21, 3, 4, "grid128_mixed"),  # 6 (slice, channel) groups: plain work-group order
        ([[128, 128]], 16, 8, 0, "grid128_mixed"),  # 16 groups: the two halves of a channel on one XCD
        ([[64, 64]], 37, 3, 4, "grid64_mixed"),
        ([[64, 64]], 9, 2, 0, "grid64_mixed"),
        ([[32, 32]], 37, 3, 4, "grid32_mixed"),
        ([[32, 32]], 1, 1, 0, "grid32_mixed"),  # a single sample
    ],
)
def test_single_level_mixed_full_oracle(level_dims, T, F, time_block, kernel):
    """Every lag of a single-level grid in the mixed form against the oracle (ragged T, several float32
    blocks)."""
    N = math.prod(dims_of(level_dims))
    gen = torch.Generator().manual_seed(N + T + F)
    raw = random_raw("ci4", T, F, N, gen)
    say("single level mixed", level_dims, "T", T, "F", F)
    vis, plan = gpu_vis(level_dims, raw, "ci4", "mixed", time_block=time_block)
    assert f'"kernel":"{kernel}"' in plan.describe()
    err = rel_err(vis, oracle_vis(raw, "ci4", level_dims))
    say("single level mixed", level_dims, "error", err)
    assert err <= TOL["mixed"]


def test_single_level_mixed_unaligned_and_sky():
    """The 128x128 mixed kernel on a 4- but not 16-byte aligned source gives the aligned result; on the
    sky-plus-noise workload bytes (64 channels, 24 samples) sampled cells agree with the oracle."""
    w = skysim.WORKLOADS["grid128"]
    raw = skysim.make_voltages(w, T=24, nchan=64, device="cuda")
    plan = omni.Plan(w.level_dims, w.A, 64, "ci4", "mixed")
    assert '"kernel":"grid128_mixed"' in plan.describe()
    ref = plan.correlate(raw).clone()
    flat = raw.reshape(-1)
    big = torch.empty(flat.numel() + 4, dtype=raw.dtype, device="cuda")
    big[4:].copy_(flat)
    shifted = big[4:].view(raw.shape)
    assert shifted.data_ptr() % 16 != 0
    got = plan.correlate(shifted)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    x = oracle.decode(raw.cpu().numpy(), "ci4", 24, 64, w.N)
    check_cells(ref.cpu().numpy()[:4], x[:, :4], w.dims, "mixed", 256, 3, "grid128 sky")
