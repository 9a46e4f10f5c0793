"""Pins of the hybrid-tile oracle (oracle/hybrid.py, Sec. III's hybrid tiles): the diagonal is
each tile's hypercube, tiles on a lattice reproduce the two-level hierarchical hypercube, Hermitian
pair symmetry, closed forms and brute force."""

from __future__ import annotations

import itertools

import numpy as np
import pytest

import oracle
from oracle import hybrid

RNG = np.random.default_rng(11)


def rand_x(T, F, N):
    return RNG.integers(-7, 8, (T, F, N)) + 1j * RNG.integers(-7, 8, (T, F, N))


def test_diagonal_is_each_tiles_hypercube():
    P, nx, ny = 3, 4, 3
    x = rand_x(5, 2, P * nx * ny)
    C = hybrid.tile_cross_correlations(x, P, nx, ny)
    for p in range(P):
        xp = x[:, :, p * nx * ny:(p + 1) * nx * ny]
        assert np.array_equal(C[:, p, p], oracle.visibilities(xp, [nx, ny]))


def test_tiles_on_a_lattice_sum_to_the_hierarchical_hypercube():
    """Tiles arranged as an outer Px x Py grid: summing C_pq over the pairs with tile-index difference D gives
    the two-level hypercube V[D, Delta] (Sec. II.D) of the whole array."""
    Px, Py, nx, ny = 2, 3, 3, 2
    P = Px * Py
    x = rand_x(4, 1, P * nx * ny)
    C = hybrid.tile_cross_correlations(x, P, nx, ny)[0]
    V = oracle.visibilities(x, [Px, Py, nx, ny])[0]
    acc = np.zeros_like(V)
    for p, q in itertools.product(range(P), range(P)):
        (px, py), (qx, qy) = divmod(p, Py), divmod(q, Py)
        acc[px - qx + Px - 1, py - qy + Py - 1] += C[p, q]
    assert np.array_equal(acc, V)


def test_pair_symmetry_and_zero_lag():
    """C_qp[Delta] = conj C_pq[-Delta]; C_pp[0] = sum_t sum_j |x_p|^2."""
    P, nx, ny = 4, 3, 5
    x = rand_x(3, 2, P * nx * ny)
    C = hybrid.tile_cross_correlations(x, P, nx, ny)
    assert np.array_equal(np.transpose(C, (0, 2, 1, 3, 4)), np.conj(C[:, :, :, ::-1, ::-1]))
    xp = x.reshape(3, 2, P, nx * ny)
    assert np.array_equal(C[:, np.arange(P), np.arange(P), nx - 1, ny - 1].real, np.sum(np.abs(xp) ** 2, axis=(0, 3)))


def test_plane_waves_closed_form():
    """Tile p carrying a_p exp(2 pi i (k_x j_x / n_x + k_y j_y / n_y)) at every sample:
    C_pq[Delta] = T a_p conj(a_q) exp(2 pi i k.Delta / n) (n_x - |D_x|)(n_y - |D_y|)."""
    P, nx, ny, T = 3, 4, 5, 2
    kx, ky = 0.3, -1.7
    a = np.array([1.0 + 2j, -0.5j, 3.0])
    j = np.indices((nx, ny))
    wave = np.exp(2j * np.pi * (kx * j[0] / nx + ky * j[1] / ny)).reshape(-1)
    x = np.tile((a[:, None] * wave[None, :]).reshape(-1), (T, 1, 1))
    C = hybrid.tile_cross_correlations(x, P, nx, ny)[0]
    D = np.indices((2 * nx - 1, 2 * ny - 1))
    dx, dy = D[0] - (nx - 1), D[1] - (ny - 1)
    base = np.exp(2j * np.pi * (kx * dx / nx + ky * dy / ny)) * (nx - np.abs(dx)) * (ny - np.abs(dy))
    for p, q in itertools.product(range(P), range(P)):
        assert np.allclose(C[p, q], T * a[p] * np.conj(a[q]) * base, atol=1e-9)


def test_brute_force_tiny():
    P, nx, ny = 2, 2, 2
    x = rand_x(2, 1, P * nx * ny)
    C = hybrid.tile_cross_correlations(x, P, nx, ny)[0]
    xr = x.reshape(2, P, nx, ny)
    for p, q, dx, dy in itertools.product(range(P), range(P), range(-1, 2), range(-1, 2)):
        acc = 0j
        for t, ax, ay in itertools.product(range(2), range(nx), range(ny)):
            bx, by = ax - dx, ay - dy
            if 0 <= bx < nx and 0 <= by < ny:
                acc += xr[t, p, ax, ay] * np.conj(xr[t, q, bx, by])
        assert C[p, q, dx + 1, dy + 1] == acc


def test_shape_check():
    with pytest.raises(ValueError):
        hybrid.tile_cross_correlations(rand_x(1, 1, 10), 3, 2, 2)
