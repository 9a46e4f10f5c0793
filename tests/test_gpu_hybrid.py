"""Parity of hybrid tiles (Sec. III; HIP, through the C ABI) with the oracle (oracle/hybrid.py).

Cases run both forms of the pair stage: with the y-axis transform fused in (P m_y <= 512 and m_x a
multiple of its rows per work-group) and as a separate front pass.

Bar: per channel and tile pair, max over index differences of |C_gpu - C_oracle| relative to
sqrt(C_pp[0] C_qq[0]) (the Cauchy-Schwarz bound of |C_pq|), <= 1e-5: the transforms and the per-cell
cross-power sums are float32 within a chunk of samples, float64 across chunks and in the inverse.
"""

import math
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_0909_0001_amd as omni
from oracle import hybrid

pytestmark = pytest.mark.gpu


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


def pair_err(got, ref, nx, ny):
    F, P = ref.shape[0], ref.shape[1]
    c = (nx - 1, ny - 1)
    zero = np.abs(ref[:, np.arange(P), np.arange(P), c[0], c[1]])  # [F, P]
    scale = np.sqrt(zero[:, :, None] * zero[:, None, :])
    scale[scale == 0] = 1.0
    return float((np.abs(got - ref).reshape(F, P, P, -1).max(axis=-1) / scale).max())


CASES = [
    (4, 8, 8, "ci8", 20, 2),
    (2, 4, 4, "ci4", 300, 1),  # two chunks of samples
    (2, 1, 8, "cf32", 9, 3),  # one-antenna-wide tiles
    (8, 4, 16, "ci4", 11, 2),
    (16, 16, 16, "ci4", 8, 2),  # 16 tiles of 16 x 16
    (32, 2, 4, "ci8", 6, 1),
    (32, 2, 16, "ci4", 5, 1),  # P m_y above 512: separate y-axis pass and pair stage
    (4, 16, 2, "ci8", 12, 2),  # n_y = 2: the y-axis DFT on the vector units (n_y = 4 .. 16 use the matrix cores)
    (8, 16, 1, "ci4", 10, 2),  # n_y = 1
    (8, 2, 32, "ci4", 7, 1),  # n_y = 32, P n_y = 256: vector-unit y-axis DFT inside the pair stage
]


@pytest.mark.parametrize("P,nx,ny,dtype,T,F", CASES)
def test_hybrid_matches_oracle(P, nx, ny, dtype, T, F):
    N = P * nx * ny
    gen = torch.Generator().manual_seed(N + T)
    raw = random_raw(dtype, T, F, N, gen)
    say(f"[hybrid] case P={P} {nx}x{ny} {dtype} T={T} F={F}")
    h = omni.Hybrid(P, nx, ny, F, dtype)
    vis = h.correlate(raw.cuda())
    torch.cuda.synchronize()
    x = oracle.decode(raw.numpy(), dtype, T, F, N)
    ref = hybrid.tile_cross_correlations(x, P, nx, ny)
    err = pair_err(vis.cpu().numpy(), ref, nx, ny)
    say(f"[hybrid] P={P} {nx}x{ny}: err {err:.3g}")
    assert err <= 1e-5


def test_hybrid_split_integration_and_empty_call():
    P, nx, ny, F = 4, 8, 4, 2
    gen = torch.Generator().manual_seed(5)
    raw = random_raw("ci8", 30, F, P * nx * ny, gen).cuda()
    h = omni.Hybrid(P, nx, ny, F, "ci8")
    whole = h.correlate(raw).clone()
    h.correlate(raw[:13].contiguous(), flags=omni.NO_FINALIZE)
    split = h.correlate(raw[13:].contiguous(), flags=omni.NO_RESET)
    torch.cuda.synchronize()
    assert pair_err(split.cpu().numpy(), whole.cpu().numpy().astype(np.complex128), nx, ny) <= 1e-6
    empty = h.correlate(raw[:0].contiguous())
    torch.cuda.synchronize()
    assert float(empty.abs().max()) == 0.0


def test_hybrid_baselines_metadata():
    P, nx, ny = 2, 2, 4
    off = np.array([[0.0, 0.0], [13.25, -4.5]])
    A = np.array([[1.0, 0.2], [0.0, 0.9]])
    h = omni.Hybrid(P, nx, ny, 1, "ci8", offsets=off, A=A)
    uv = h.baselines()
    for p in range(P):
        for q in range(P):
            for dx in range(-(nx - 1), nx):
                for dy in range(-(ny - 1), ny):
                    want = off[p] - off[q] + A @ np.array([dx, dy])
                    assert np.allclose(uv[p, q, dx + nx - 1, dy + ny - 1], want)
    with pytest.raises(omni.OmniError):
        omni.Hybrid(P, nx, ny, 1, "ci8").baselines()


def test_hybrid_argument_errors():
    h = omni.Hybrid(2, 4, 4, 1, "ci8")
    with pytest.raises(ValueError):
        h.correlate(torch.zeros((3, 1, 31, 2), dtype=torch.int8, device="cuda"))
    with pytest.raises(ValueError):
        h.correlate(torch.zeros((3, 1, 32), dtype=torch.uint8, device="cuda"))


def test_hybrid_bench_size_sampled():
    """The bench's configuration (16 tiles of 16 x 16, F = 64, T = 2048, 4-bit, 8 chunks of samples): every tile
    pair of two channels for three tile pairs against the oracle run on just those two tiles (a pair's
    correlation depends on its two tiles' samples only), the diagonal blocks included."""
    P, nx, ny, F, T = 16, 16, 16, 64, 2048
    N = P * nx * ny
    gen = torch.Generator(device="cuda").manual_seed(20260)
    re = torch.randint(-7, 8, (T, F, N), generator=gen, device="cuda", dtype=torch.int16)
    im = torch.randint(-7, 8, (T, F, N), generator=gen, device="cuda", dtype=torch.int16)
    raw = ((re & 0xF) << 4 | (im & 0xF)).to(torch.uint8)
    del re, im
    say("[hybrid] bench size: 16 tiles of 16x16, F=64, T=2048")
    h = omni.Hybrid(P, nx, ny, F, "ci4")
    vis = h.correlate(raw)
    torch.cuda.synchronize()
    M = nx * ny
    for f in (0, 37):
        for p, q in ((0, 1), (5, 12), (15, 3)):
            cols = torch.cat([torch.arange(p * M, (p + 1) * M), torch.arange(q * M, (q + 1) * M)]).cuda()
            sub = raw[:, f:f + 1, :].index_select(2, cols).cpu().numpy()
            x = oracle.decode(sub, "ci4", T, 1, 2 * M)
            ref = hybrid.tile_cross_correlations(x, 2, nx, ny)  # [1, 2, 2, 31, 31]
            idx = torch.tensor([p, q]).cuda()
            got = vis[f:f + 1].index_select(1, idx).index_select(2, idx).cpu().numpy()
            err = pair_err(got, ref, nx, ny)
            say(f"[hybrid] bench size f={f} tiles ({p},{q}): err {err:.3g}")
            assert err <= 1e-5
    h.close()
