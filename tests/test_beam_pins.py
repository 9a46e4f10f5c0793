"""Pins of the beam-space oracle (oracle/beams.py, Appendix A steps 4-5): the full hypercube
transformed along the lowest level's lags, plane waves that land in one pointing, a closed-form
sum over pointings, and brute force."""

from __future__ import annotations

import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import beams

RNG = np.random.default_rng(7)


def rand_x(T, F, N, ints=True):
    if ints:
        return RNG.integers(-7, 8, (T, F, N)) + 1j * RNG.integers(-7, 8, (T, F, N))
    return RNG.normal(size=(T, F, N)) + 1j * RNG.normal(size=(T, F, N))


@pytest.mark.parametrize("level_dims", [[[3, 2], [4, 4]], [[2, 2], [2, 3], [4, 2]], [[5, 1], [3, 4]]])
def test_pointings_are_the_hypercube_along_the_block_lags(level_dims):
    """V_b[D'] = sum_{D_in} exp(-2 pi i b.D_in / n) V[D', D_in]: the beam-space result is the full
    hypercube (Sec. II.D) Fourier transformed, unpadded, along the lowest level's lag axes."""
    dims = [v for ld in level_dims for v in ld]
    x = rand_x(3, 2, math.prod(dims))
    Vb = beams.beam_visibilities(x, level_dims)
    V = oracle.visibilities(x, dims)  # [F, lags...]
    nx, ny = dims[-2], dims[-1]
    dx = np.arange(-(nx - 1), nx)
    dy = np.arange(-(ny - 1), ny)
    for bx, by in itertools.product(range(nx), range(ny)):
        ph = np.exp(-2j * np.pi * (bx * dx[:, None] / nx + by * dy[None, :] / ny))
        ref = np.tensordot(V, ph, axes=([-2, -1], [0, 1]))
        assert np.allclose(Vb[..., bx, by], ref, atol=1e-8 * np.abs(V).max())


def test_plane_wave_lands_in_one_pointing():
    """A block-level plane wave exp(+2 pi i (k_x j_x / n_x + k_y j_y / n_y)) times an outer pattern u puts
    (n_x n_y)^2 V_u in pointing (k_x, k_y) and nothing elsewhere."""
    level_dims = [[3, 3], [4, 8]]
    nx, ny = 4, 8
    kx, ky = 3, 5
    T = 2
    u = rand_x(T, 1, 9, ints=False)  # outer pattern [T, 1, 9]
    j = np.indices((nx, ny))
    wave = np.exp(2j * np.pi * (kx * j[0] / nx + ky * j[1] / ny)).reshape(-1)
    x = (u[:, :, :, None] * wave[None, None, None, :]).reshape(T, 1, -1)
    Vb = beams.beam_visibilities(x, level_dims)
    Vu = oracle.visibilities(u, [3, 3])
    for bx, by in itertools.product(range(nx), range(ny)):
        want = (nx * ny) ** 2 * Vu if (bx, by) == (kx, ky) else 0.0 * Vu
        assert np.allclose(Vb[..., bx, by], want, atol=1e-8 * (nx * ny) ** 2 * np.abs(Vu).max())


def test_sum_over_pointings_is_zero_block_lag():
    """sum_b V_b[D'] = n_x n_y V[D', 0] (only D_in = 0 survives the sum over all pointings)."""
    level_dims = [[2, 3], [4, 3]]
    dims = [2, 3, 4, 3]
    x = rand_x(4, 2, 72)
    Vb = beams.beam_visibilities(x, level_dims)
    V = oracle.visibilities(x, dims)
    assert np.allclose(Vb.sum(axis=(-2, -1)), 12 * V[..., 3, 2], atol=1e-8 * np.abs(V).max() * 12)


def test_brute_force_tiny():
    level_dims = [[2, 1], [2, 3]]
    outer, (nx, ny) = [2, 1], (2, 3)
    x = rand_x(2, 1, 12)
    Vb = beams.beam_visibilities(x, level_dims)
    xr = x.reshape(2, 1, 2, 1, nx, ny)
    for bx, by in itertools.product(range(nx), range(ny)):
        B = np.zeros((2, 2, 1), complex)
        for t, i0, i1 in itertools.product(range(2), range(2), range(1)):
            B[t, i0, i1] = sum(xr[t, 0, i0, i1, a, c] * np.exp(-2j * np.pi * (bx * a / nx + by * c / ny))
                               for a in range(nx) for c in range(ny))
        for d0, d1 in itertools.product(range(-1, 2), range(1)):
            acc = 0j
            for t, i0, i1 in itertools.product(range(2), range(2), range(1)):
                if 0 <= i0 - d0 < 2 and 0 <= i1 - d1 < 1:
                    acc += B[t, i0, i1] * np.conj(B[t, i0 - d0, i1 - d1])
            assert abs(Vb[0, d0 + 1, d1, bx, by] - acc) < 1e-9


def test_needs_a_level_above_the_blocks():
    with pytest.raises(ValueError):
        beams.beam_visibilities(rand_x(1, 1, 16), [[4, 4]])
