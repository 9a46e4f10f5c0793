"""Parity of the F-engine (HIP, through the C ABI) with the oracle (oracle/fengine.py,
Appendix A steps 2-3), and the F-engine feeding the correlator.

Bar: the codes are integers decided by rounding float values, so they must equal the oracle's
except where the exact (float64) value lies within the kernel's error of a rounding boundary;
there either neighbouring code is a correct result.  The bound used per element is
eps = |gain| * 1e-5 * sum_j |raw_j| + 1e-6 * |Y|: the kernel's products and sums are exact int32
ones of int8 samples and a three-part int8 split of the DFT coefficients (at most 6.1e-8 off
each), followed by a few float32 roundings of the output, so its error stays far inside that.
Every other code is bit-exact, and near-boundary codes are rare (checked).
"""

import math
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_0909_0001_amd as omni
from oracle import fengine as fe

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def make_raw(N, F, T, seed, sigma=20.0):
    """Noise plus a few tones, int8, antenna-major [N, 2 F T]."""
    gen = torch.Generator().manual_seed(seed)
    S = 2 * F * T
    x = torch.randn((N, S), generator=gen) * sigma
    j = torch.arange(S, dtype=torch.float64)
    for q in range(3):
        k0 = (7 * q + 3) % F + 0.25 * q
        x += (30.0 * torch.cos(2 * math.pi * k0 * j / (2 * F) + q)).float()
    return torch.clamp(torch.round(x), -128, 127).to(torch.int8)


def make_gains(N, F, dtype, seed, sigma=20.0):
    gen = torch.Generator().manual_seed(seed + 1)
    target = 2.5 if dtype == "ci4" else 32.0
    mag = target / (sigma * math.sqrt(F)) * (0.7 + 0.6 * torch.rand((N, F), generator=gen))
    ph = 2 * math.pi * torch.rand((N, F), generator=gen)
    return torch.polar(mag, ph).to(torch.complex64)


def check_codes(out_gpu, raw, F, gains, dtype):
    T = raw.shape[1] // (2 * F)
    N = raw.shape[0]
    ref, Y = fe.fengine(raw.numpy(), F, gains.numpy().astype(np.complex128), dtype)
    got = oracle.decode(out_gpu.cpu().numpy(), dtype, T, F, N)
    want = oracle.decode(ref, dtype, T, F, N)
    # per-element error bound of the float32 transform
    blk = np.abs(raw.numpy().astype(np.float64)).reshape(N, T, 2 * F).sum(axis=-1)  # [N, T]
    eps = np.abs(gains.numpy())[None, :, :].transpose(0, 2, 1) * 1e-5 * blk.T[:, None, :] + 1e-6 * np.abs(Y)
    bad = 0
    for part in ("real", "imag"):
        g, w, v = getattr(got, part), getattr(want, part), getattr(Y, part)
        diff = g != w
        if diff.any():
            dist = np.abs(np.abs(v - np.floor(v)) - 0.5)  # distance to the nearest rounding boundary
            assert np.all(np.abs(g - w)[diff] == 1), "a code off by more than one"
            assert np.all(dist[diff] <= eps[diff]), f"a code differs away from a boundary: {dist[diff].max()}"
            bad += int(diff.sum())
    say(f"[fengine] F={F} {dtype} N={N} T={T}: {bad} of {2 * got.size} codes at a rounding boundary")
    assert bad <= max(2, 1e-3 * 2 * got.size)
    return got


@pytest.mark.parametrize("N", [300, 336])
@pytest.mark.parametrize("F", [16, 32, 64])
@pytest.mark.parametrize("dtype", ["ci4", "ci8"])
def test_fengine_matches_oracle(F, dtype, N):
    """Ragged antenna counts (masked lanes): 300 takes the code-by-code stores, 336 (a multiple of 16, not of
    a work-group's antennas) the 16-byte row stores with a partly valid last group; several time chunks."""
    T = 9
    raw = make_raw(N, F, T, seed=F)
    gains = make_gains(N, F, dtype, seed=F)
    say(f"[fengine] case F={F} {dtype} N={N}")
    out = omni.fengine(raw.cuda(), F, gains.cuda(), dtype)
    torch.cuda.synchronize()
    check_codes(out, raw, F, gains, dtype)


def test_fengine_clipping_and_extremes():
    """Full-scale input (-128 and 127) and large gains: most codes clip to the format's edge, never to -8."""
    F, N, T = 64, 64, 3
    raw = torch.full((N, 2 * F * T), 127, dtype=torch.int8)
    raw[::2, ::3] = -128
    gains = torch.full((N, F), 0.05 + 0.05j, dtype=torch.complex64)
    out = omni.fengine(raw.cuda(), F, gains.cuda(), "ci4")
    torch.cuda.synchronize()
    got = check_codes(out, raw, F, gains, "ci4")
    assert got.real.min() >= -7 and got.imag.min() >= -7
    assert (np.abs(got.real) == 7).any()


@pytest.mark.parametrize("dtype", ["ci4", "ci8"])
def test_fengine_large_T_and_N(dtype):
    """A size with many work-groups and time chunks: 4096 antennas, 512 blocks of 128 samples (sampled check
    of 64 antennas against the oracle, since the layout and every code path are the same)."""
    F, N, T = 64, 4096, 512
    raw = make_raw(N, F, T, seed=5)
    gains = make_gains(N, F, dtype, seed=5)
    say(f"[fengine] large case {dtype}")
    out = omni.fengine(raw.cuda(), F, gains.cuda(), dtype)
    torch.cuda.synchronize()
    idx = torch.arange(0, N, 64)
    sub_out = out[:, :, idx].contiguous()
    check_codes(sub_out, raw[idx].contiguous(), F, gains[idx].contiguous(), dtype)


def test_fengine_feeds_the_correlator():
    """F-engine codes of a 16 x 16 grid (F = 16 channels, T = 24 blocks) correlated on the GPU (mixed form):
    the correlator's visibilities equal the oracle's of the same codes to the mixed form's tolerance."""
    F, T = 16, 24
    level_dims = [[16, 16]]
    N = 256
    raw = make_raw(N, F, T, seed=9)
    gains = make_gains(N, F, "ci4", seed=9)
    volt = omni.fengine(raw.cuda(), F, gains.cuda(), "ci4")
    plan = omni.Plan(level_dims, None, F, "ci4", "mixed")
    vis = plan.correlate(volt)
    torch.cuda.synchronize()
    x = oracle.decode(volt.cpu().numpy(), "ci4", T, F, N)
    ref = oracle.visibilities(x, [16, 16])
    g = vis.cpu().numpy().reshape(F, -1)
    r = ref.reshape(F, -1)
    c = r.shape[1] // 2
    err = float(np.max(np.abs(g - r).max(axis=1) / np.abs(r[:, c])))
    say(f"[fengine] correlator on F-engine output: err {err:.3g}")
    assert err <= 2e-3


def test_fengine_argument_errors():
    raw = torch.zeros((8, 2 * 64 * 2), dtype=torch.int8, device="cuda")
    gains = torch.zeros((8, 64), dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError):
        omni.fengine(raw, 48, gains)
    with pytest.raises(ValueError):
        omni.fengine(raw, 64, gains[:, :32].contiguous())
    with pytest.raises(ValueError):
        omni.fengine(raw.to(torch.int16), 64, gains)
    out = omni.fengine(raw, 64, gains, "ci8")
    torch.cuda.synchronize()
    assert out.shape == (2, 64, 8, 2) and int(out.abs().max()) == 0


@pytest.mark.parametrize("dtype", ["ci4", "ci8"])
def test_fengine_bench_size_sampled(dtype):
    """The bench's configuration (16384 antennas, T = 2048 blocks of 128 samples -> 64 channels; 16-byte row
    stores, every work-group and time chunk of the launch): 48 antennas spread over the array, all blocks and
    channels, against the oracle on those antennas' samples (each antenna's codes depend on its own samples
    and gains only)."""
    F, N, T = 64, 16384, 2048
    gen = torch.Generator(device="cuda").manual_seed(31 if dtype == "ci4" else 32)
    raw = torch.randint(-128, 128, (N, 2 * F * T), generator=gen, device="cuda", dtype=torch.int16).to(torch.int8)
    gains = make_gains(N, F, dtype, seed=7, sigma=74.0).cuda()
    say(f"[fengine] bench size {dtype}")
    out = omni.fengine(raw, F, gains, dtype)
    torch.cuda.synchronize()
    idx = torch.cat([torch.arange(0, N, 409)[:40], torch.tensor([63, 64, 8191, 8192, 16320, 16383, 1, 127])])
    sub_out = out[:, :, idx.cuda()].contiguous()
    check_codes(sub_out, raw[idx.cuda()].cpu(), F, gains[idx.cuda()].cpu(), dtype)
