"""Seeded synthetic sky-plus-noise voltages for hierarchical antenna grids.

This module is shared by the tests, the benchmark and the oracle's callers.  It
holds no correlator arithmetic: it only places antennas on a hierarchical grid
(r = sum_levels A_l (i_lx, i_ly), Sec. II.D Eq. GridEq), draws point sources
(and optionally a diffuse field) in random sky directions, forms the voltage
each antenna sees, adds complex Gaussian noise and quantises to the sample
formats the library accepts:

* ``cf32``: float32 (re, im) pairs          -> torch.float32 [T, F, N, 2]
* ``ci8`` : int8 (re, im) pairs             -> torch.int8    [T, F, N, 2]
* ``ci4`` : one byte, re high nibble, im low nibble, two's complement, values
  in [-7, 7]                                -> torch.uint8   [T, F, N]

Generation runs on CPU or on a GPU through torch; the seed fixes the bytes for
a given device.  Consumers always check results against the exact bytes the
library consumed, so CPU and GPU streams need not agree.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np
import torch

__all__ = [
    "lattice",
    "positions",
    "Workload",
    "WORKLOADS",
    "make_voltages",
    "pack_ci4",
    "quantise",
    "PAPER_LAYOUTS",
]


def lattice(scale: float, theta_deg: float = 0.0, shear: float = 0.0) -> np.ndarray:
    """2x2 lattice matrix s R(theta) [[1, h], [0, 1]]; its columns are the two lattice vectors."""
    t = math.radians(theta_deg)
    R = np.array([[math.cos(t), -math.sin(t)], [math.sin(t), math.cos(t)]])
    return scale * R @ np.array([[1.0, shear], [0.0, 1.0]])


def positions(level_dims: Sequence[Sequence[int]], A) -> np.ndarray:
    """Antenna positions [N, 2] (wavelengths at the reference frequency), row-major over
    (level 0 x, level 0 y, level 1 x, ...) index tuples."""
    A = np.asarray(A, dtype=np.float64).reshape(len(level_dims), 2, 2)
    dims = [int(n) for ld in level_dims for n in ld]
    idx = np.indices(dims).reshape(len(dims), -1).T.astype(np.float64)
    r = np.zeros((idx.shape[0], 2))
    for lvl in range(len(level_dims)):
        r += idx[:, 2 * lvl : 2 * lvl + 2] @ A[lvl].T
    return r


@dataclass
class Workload:
    """A named synthetic workload: geometry, sizes, sample format and sky."""

    name: str
    level_dims: list  # [[n_x, n_y], ...] outer level first
    A: np.ndarray  # [levels, 2, 2]
    nchan: int
    T: int
    dtype: str  # cf32 | ci8 | ci4
    n_src: int
    form: str = "fp32"  # fp32 | mixed
    diffuse: bool = False
    seed: int = 20090831
    note: str = ""

    @property
    def dims(self) -> list:
        return [int(n) for ld in self.level_dims for n in ld]

    @property
    def N(self) -> int:
        return math.prod(self.dims)

    @property
    def levels(self) -> int:
        return len(self.level_dims)

    def antenna_samples(self) -> int:
        return self.N * self.T * self.nchan


def _stack(*mats) -> np.ndarray:
    return np.stack([np.asarray(m, dtype=np.float64) for m in mats])


WORKLOADS = {
    # 16x16 unit-spaced grid, one channel, float voltages.
    "grid16": Workload("grid16", [[16, 16]], _stack(lattice(1.0)), 1, 1024, "cf32", 8, "fp32", seed=20090832),
    # 8x8 tiles of 8x8 antennas: inner 0.5 lambda; outer 5 lambda, rotated 15 deg, shear 0.2.
    "hier8x8": Workload(
        "hier8x8", [[8, 8], [8, 8]], _stack(lattice(5.0, 15.0, 0.2), lattice(0.5)), 64, 4096, "ci8", 64, "fp32",
        seed=20090833,
    ),
    "hier8x8-mixed": Workload(
        "hier8x8-mixed", [[8, 8], [8, 8]], _stack(lattice(5.0, 15.0, 0.2), lattice(0.5)), 64, 4096, "ci8", 64,
        "mixed", seed=20090833,
    ),
    # Three levels 16x16 (25 deg) / 8x8 (10 deg) / 4x4 (0 deg), 4-bit voltages, diffuse sky.
    "hier3": Workload(
        "hier3", [[16, 16], [8, 8], [4, 4]],
        _stack(lattice(24.0, 25.0), lattice(2.5, 10.0), lattice(0.5)), 16, 1024, "ci4", 256, "mixed", diffuse=True,
        seed=20090834,
    ),
    # The four arrays of the batched workload (64 channels each, T=2048, 4-bit).
    "grid32": Workload("grid32", [[32, 32]], _stack(lattice(0.5)), 64, 2048, "ci4", 32, "mixed", seed=20090835),
    "grid64": Workload("grid64", [[64, 64]], _stack(lattice(0.5)), 64, 2048, "ci4", 32, "mixed", seed=20090836),
    "grid128": Workload("grid128", [[128, 128]], _stack(lattice(0.5)), 64, 2048, "ci4", 32, "mixed", seed=20090837),
    "hier16x16": Workload(
        "hier16x16", [[16, 16], [16, 16]], _stack(lattice(10.0), lattice(0.5)), 64, 2048, "ci4", 32, "mixed",
        seed=20090838,
    ),
}

#: The four hierarchical example layouts of Sec. III (Figs. ThreeLevelFig, BlocksFig, PlankFig,
#: StripsFig), in metres (the minimum antenna spacing is 1 m): name -> (level_dims, A), outer level
#: first, the columns of each A_l the level's two lattice vectors.  The 3-level layout is the one of
#: Fig. 1 (a_1 = (1,0) with five positions and a_4 = (0,1); a_2 = (8,0), a_5 = (2,8); a_3 = (40,10),
#: a_6 = (-10,40), three positions each).
PAPER_LAYOUTS = {
    "3-level": ([[3, 3], [3, 3], [5, 3]], _stack([[40, -10], [10, 40]], [[8, 2], [0, 8]], [[1, 0], [0, 1]])),
    "Blocks": ([[2, 2], [16, 16]], _stack([[200, 0], [0, 200]], [[1, 0], [0, 1]])),
    "Plank": ([[512, 32]], _stack([[1, 0], [0, 1]])),
    "Strips": ([[32, 512]], _stack([[16, 0], [0, 1]])),
}

#: Target pre-clip RMS per real component for each integer format (clip at +-127 / +-7).
_TARGET_RMS = {"ci8": 32.0, "ci4": 2.5}
_CLIP = {"ci8": 127, "ci4": 7}


def channel_ratios(F: int) -> np.ndarray:
    """nu_f / nu_0 for F channels spread over +-10% of the reference frequency (1.0 for F = 1)."""
    if F == 1:
        return np.ones(1)
    return 0.9 + 0.2 * (np.arange(F) + 0.5) / F


def _sky(n_src: int, rng: np.random.Generator, diffuse: bool):
    """Direction cosines (l, m) and fluxes of the incoherent sky components."""
    cosz = 1.0 - rng.random(n_src)  # in (0, 1]
    sinz = np.sqrt(1.0 - cosz**2)
    phi = rng.random(n_src) * 2 * np.pi
    l = sinz * np.cos(phi)
    m = sinz * np.sin(phi)
    flux = rng.uniform(0.5, 2.0, n_src)
    if diffuse:
        # 64x64 pixels over |l|,|m| <= 0.7: log-normal intensity from a unit-variance
        # Gaussian random field with P(k) ~ k^-2, scaled to 25% of the point flux.
        g = 64
        kx = np.fft.fftfreq(g)[:, None]
        ky = np.fft.fftfreq(g)[None, :]
        k = np.sqrt(kx**2 + ky**2)
        amp = np.zeros_like(k)
        amp[k > 0] = 1.0 / k[k > 0]
        field_ = np.fft.ifft2(amp * (rng.standard_normal((g, g)) + 1j * rng.standard_normal((g, g)))).real
        field_ = (field_ - field_.mean()) / field_.std()
        inten = np.exp(field_).ravel()
        inten *= 0.25 * flux.sum() / inten.sum()
        grid = np.linspace(-0.7, 0.7, g)
        gl, gm = np.meshgrid(grid, grid, indexing="ij")
        l = np.concatenate([l, gl.ravel()])
        m = np.concatenate([m, gm.ravel()])
        flux = np.concatenate([flux, inten])
    return l, m, flux


def quantise(v: torch.Tensor, dtype: str, gain: float) -> torch.Tensor:
    """Scale complex voltages, round half to even, clip and pack into the sample format."""
    if dtype == "cf32":
        return torch.view_as_real(v.to(torch.complex64)).contiguous()
    q = torch.view_as_real(v * gain).round().clamp_(-_CLIP[dtype], _CLIP[dtype])
    if dtype == "ci8":
        return q.to(torch.int8)
    return pack_ci4(q[..., 0].to(torch.int16), q[..., 1].to(torch.int16))


def pack_ci4(re: torch.Tensor, im: torch.Tensor) -> torch.Tensor:
    """One byte per sample: re in the high nibble, im in the low nibble, two's complement."""
    return (((re & 0xF) << 4) | (im & 0xF)).to(torch.uint8)


def make_voltages(
    w: Workload,
    device="cpu",
    T: int | None = None,
    nchan: int | None = None,
    seed: int | None = None,
    noise_sigma: float = 1.0,
) -> torch.Tensor:
    """Quantised voltages for workload ``w`` (optionally fewer samples / channels).

    x_{t,f,a} = sum_s sqrt(flux_s) e^{i psi_{s,t,f}} e^{-2 pi i (nu_f/nu_0)(l_s r_ax + m_s r_ay)} + n_{t,f,a}
    with psi uniform per (source, sample, channel) and n ~ CN(0, sigma^2).
    """
    T = w.T if T is None else T
    F = w.nchan if nchan is None else nchan
    seed = w.seed if seed is None else seed
    rng = np.random.default_rng(seed)
    r = positions(w.level_dims, w.A)  # [N, 2]
    l, m, flux = _sky(w.n_src, rng, w.diffuse)
    S = flux.size
    nu = channel_ratios(w.nchan)[:F]
    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    power = float(flux.sum()) + noise_sigma**2
    gain = _TARGET_RMS.get(w.dtype, 1.0) / math.sqrt(power / 2.0)
    N = r.shape[0]
    if w.dtype == "cf32":
        out = torch.empty((T, F, N, 2), dtype=torch.float32, device=dev)
    elif w.dtype == "ci8":
        out = torch.empty((T, F, N, 2), dtype=torch.int8, device=dev)
    else:
        out = torch.empty((T, F, N), dtype=torch.uint8, device=dev)
    sqrt_flux = torch.tensor(np.sqrt(flux), dtype=torch.float32, device=dev)
    lm = torch.tensor(np.stack([l, m], axis=1), dtype=torch.float64, device=dev)  # [S, 2]
    rr = torch.tensor(r, dtype=torch.float64, device=dev)  # [N, 2]
    # antennas are processed in chunks so that the [S, chunk] steering matrix stays small
    chunk = N if S * N <= (1 << 24) else max(256, (1 << 24) // S)
    for f in range(F):
        psi = torch.rand((T, S), generator=gen, device=dev) * (2 * math.pi)
        amp = torch.polar(sqrt_flux.expand(T, S).contiguous(), psi)  # [T, S] complex64
        for a0 in range(0, N, chunk):
            a1 = min(N, a0 + chunk)
            proj = lm @ rr[a0:a1].T  # [S, chunk]: l r_x + m r_y
            steer = torch.exp(-2j * math.pi * float(nu[f]) * proj).to(torch.complex64)
            v = amp @ steer  # [T, chunk]
            noise = torch.randn((T, a1 - a0, 2), generator=gen, device=dev) * (noise_sigma / math.sqrt(2.0))
            v = v + torch.view_as_complex(noise)
            out[:, f, a0:a1] = quantise(v, w.dtype, gain)
    return out
