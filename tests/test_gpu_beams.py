"""Parity of the beam-space variant (Appendix A steps 4-5; HIP, through the C ABI) with the
oracle (oracle/beams.py).

Bar: per channel and pointing, max over the outer lags of |V_gpu - V_oracle| relative to that
pointing's zero-lag power, <= 1e-5 (float32 form) or 2e-3 (mixed form).
"""

import math
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_0909_0001_amd as omni
from oracle import beams

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "mixed": 2e-3}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def random_raw(dtype, T, F, N, gen):
    if dtype == "cf32":
        return torch.randn((T, F, N, 2), generator=gen).float()
    if dtype == "ci8":
        return torch.randint(-127, 128, (T, F, N, 2), generator=gen, dtype=torch.int16).to(torch.int8)
    re = torch.randint(-7, 8, (T, F, N), generator=gen, dtype=torch.int16)
    im = torch.randint(-7, 8, (T, F, N), generator=gen, dtype=torch.int16)
    return ((re & 0xF) << 4 | (im & 0xF)).to(torch.uint8)


def beam_err(got, ref, level_dims):
    """max over channels and pointings of (max over lags |got - ref|) / ref[zero lag]."""
    F = ref.shape[0]
    nb = level_dims[-1][0] * level_dims[-1][1]
    g = np.moveaxis(got.reshape((F, -1, nb)), 2, 1)  # [F, nb, lags]
    r = np.moveaxis(ref.reshape((F, -1, nb)), 2, 1)
    c = r.shape[2] // 2
    z = np.abs(r[:, :, c])
    z[z == 0] = 1.0
    return float(np.max(np.abs(g - r).max(axis=2) / z))


# (level_dims, dtype, form, T, F, route): "unpadded" = the general kernel with the blocks' axes unpadded;
# "subset" = the ordinary plan's fixed-shape kernel, pointings taken as its even Fourier cells
CASES = [
    ([[4, 4], [8, 8]], "ci8", "fp32", 20, 2, "unpadded"),
    ([[4, 4], [8, 8]], "ci4", "mixed", 20, 2, "unpadded"),
    ([[2, 3], [3, 3], [4, 4]], "ci4", "fp32", 9, 3, "unpadded"),
    ([[3, 3], [5, 5]], "cf32", "fp32", 7, 2, "unpadded"),  # odd block sides: unpadded 5-point transforms
    ([[4, 1], [1, 8]], "ci8", "fp32", 11, 2, "unpadded"),  # one-dimensional blocks
    ([[16, 16], [16, 16]], "ci4", "fp32", 12, 2, "subset"),  # 256 pointings, compile-time-shape kernel
    ([[16, 16], [16, 16]], "ci4", "mixed", 12, 2, "subset"),  # the matrix-core kernel behind a front pass
    ([[8, 8], [8, 8]], "ci8", "mixed", 16, 3, "subset"),  # 8x8x8x8 matrix-core kernel
    ([[1, 64], [64, 1]], "ci4", "mixed", 10, 2, "subset"),  # one-dimensional blocks on the 64 x 64 kernel
]


@pytest.mark.parametrize("level_dims,dtype,form,T,F,route", CASES)
def test_beam_space_matches_oracle(level_dims, dtype, form, T, F, route):
    import json

    dims = [v for ld in level_dims for v in ld]
    N = math.prod(dims)
    gen = torch.Generator().manual_seed(N + T)
    raw = random_raw(dtype, T, F, N, gen)
    say(f"[beams] case {level_dims} {dtype} {form} T={T} F={F}")
    plan = omni.Plan(level_dims, None, F, dtype, form, beams=True)
    assert json.loads(plan.describe())["arrays"][0]["beams"] == route
    shape = plan.vis_shape()
    assert shape == (F,) + tuple(2 * v - 1 for v in dims[:-2]) + tuple(dims[-2:])
    vis = plan.correlate(raw.cuda())
    torch.cuda.synchronize()
    x = oracle.decode(raw.numpy(), dtype, T, F, N)
    ref = beams.beam_visibilities(x, level_dims)
    err = beam_err(vis.cpu().numpy(), ref, level_dims)
    say(f"[beams] {level_dims}: err {err:.3g}")
    assert err <= TOL[form]


def test_beam_space_front_chunks():
    """The 16 x 16-of-16 x 16 beam-space plan takes a front pass over its outer axes; three time chunks."""
    import json

    level_dims = [[16, 16], [16, 16]]
    T, F, N = 12, 2, 65536
    gen = torch.Generator().manual_seed(77)
    raw = random_raw("ci8", T, F, N, gen)
    plan = omni.Plan(level_dims, None, F, "ci8", "fp32", beams=True, chunk_T=4)
    a = json.loads(plan.describe())["arrays"][0]
    assert a["mode"] == "front" and -(-T // a["chunk_T"]) == 3
    vis = plan.correlate(raw.cuda())
    torch.cuda.synchronize()
    x = oracle.decode(raw.numpy(), "ci8", T, F, N)
    err = beam_err(vis.cpu().numpy(), beams.beam_visibilities(x, level_dims), level_dims)
    say(f"[beams] front chunks: err {err:.3g}")
    assert err <= TOL["fp32"]


def test_beam_space_split_integration():
    """Two calls (NO_RESET on the second) equal one call over all samples (linearity in time)."""
    level_dims = [[4, 4], [8, 8]]
    gen = torch.Generator().manual_seed(3)
    raw = random_raw("ci8", 24, 2, 1024, gen).cuda()
    plan = omni.Plan(level_dims, None, 2, "ci8", "fp32", beams=True)
    whole = plan.correlate(raw).clone()
    plan.correlate(raw[:10].contiguous(), flags=omni.NO_FINALIZE)
    split = plan.correlate(raw[10:].contiguous(), flags=omni.NO_RESET)
    torch.cuda.synchronize()
    assert beam_err(split.cpu().numpy(), whole.cpu().numpy().astype(np.complex128), level_dims) <= 1e-6


def test_beam_space_refusals():
    level_dims = [[4, 4], [8, 8]]
    A = np.stack([np.eye(2) * 8.0, np.eye(2)])
    plan = omni.Plan(level_dims, A, 1, "ci8", "fp32", beams=True)
    with pytest.raises(omni.OmniError):
        plan.baselines()
    with pytest.raises(omni.OmniError):
        omni.Fold(plan)
    raw = torch.zeros((2, 1, 1024, 2), dtype=torch.int8, device="cuda")
    with pytest.raises(omni.OmniError):
        plan.direct_correlate(raw)
    with pytest.raises(omni.OmniError):
        omni.Plan([[8, 8]], None, 1, "ci8", "fp32", beams=True)


def test_beam_space_bench_size_sampled():
    """The bench's configuration (16 x 16-of-16 x 16, 4-bit, 64 channels, T = 2048, mixed form, subset route):
    one channel's pointings against the oracle, for a handful of pointings (each pointing is the outer-grid
    correlation of its own block beams, so it needs only those)."""
    import json

    level_dims = [[16, 16], [16, 16]]
    T, F, N = 2048, 64, 65536
    gen = torch.Generator(device="cuda").manual_seed(4242)
    re = torch.randint(-7, 8, (T, F, N), generator=gen, device="cuda", dtype=torch.int16)
    im = torch.randint(-7, 8, (T, F, N), generator=gen, device="cuda", dtype=torch.int16)
    raw = ((re & 0xF) << 4 | (im & 0xF)).to(torch.uint8)
    del re, im
    say("[beams] bench size: 16x16-of-16x16, F=64, T=2048, mixed")
    plan = omni.Plan(level_dims, None, F, "ci4", "mixed", beams=True)
    assert json.loads(plan.describe())["arrays"][0]["beams"] == "subset"
    vis = plan.correlate(raw)
    torch.cuda.synchronize()
    f = 29
    x = oracle.decode(raw[:, f:f + 1].contiguous().cpu().numpy(), "ci4", T, 1, N)
    del raw
    B = beams.pointings(x, level_dims)[:, 0]  # [T, 256 blocks, 16, 16]
    del x
    picks = [(0, 0), (1, 0), (7, 13), (15, 15)]
    xb = np.stack([B[:, :, bx, by] for bx, by in picks], axis=1)  # [T, 4, 256]
    del B
    ref = oracle.visibilities(xb, [16, 16])  # [4, 31, 31]
    got = vis[f].cpu().numpy()  # [31, 31, 16, 16]
    for k, (bx, by) in enumerate(picks):
        g, r = got[:, :, bx, by], ref[k]
        err = float(np.abs(g - r).max() / abs(r[15, 15]))
        say(f"[beams] bench size pointing ({bx},{by}): err {err:.3g}")
        assert err <= TOL["mixed"]
