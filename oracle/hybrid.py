"""Plain float64 oracle of hybrid tiles (test infrastructure only; no product path may import it).

Sec. III (the hybrid-tile paragraph): the array is a set of P rectangular tiles of M antennas
each, translated relative to one another by arbitrary amounts; correlations inside a tile use the
FFT method, and the tiles' synthesized beams (their Fourier transforms) are correlated between
tiles pair by pair.  What that computes, for every ordered pair of tiles (p, q) and every index
difference Delta inside the tile grid (Delta_k in [-(n_k - 1), n_k - 1]):

    C_pq[Delta] = sum_t sum_{j, j - Delta in tile} x_p[t, j] conj(x_q[t, j - Delta]),

the cross-correlation of tile p with tile q over index differences (physical baseline
o_p - o_q + sum_k Delta_k a_k for tile offsets o); C_pp is tile p's own visibility hypercube
(Sec. II.D, Eq. ProofEq2).  Readings: antennas are tile-major, x[t, f, p M + (i_x n_y + i_y)];
the output holds every ordered pair, [F, P, P, 2n_x - 1, 2n_y - 1]; plain sums as for the
hypercube.
"""

from __future__ import annotations

import numpy as np

__all__ = ["tile_cross_correlations"]


def tile_cross_correlations(x, P: int, nx: int, ny: int) -> np.ndarray:
    """C[f, p, q, Dx + nx - 1, Dy + ny - 1] from the definition: every antenna pair of tiles p and q
    (time summed by one matrix product), binned by index difference."""
    x = np.asarray(x)
    T, F, N = x.shape
    M = nx * ny
    if N != P * M:
        raise ValueError(f"N={N} is not P * nx * ny = {P * M}")
    ix, iy = np.divmod(np.arange(M), ny)
    key = ((ix[:, None] - ix[None, :] + nx - 1) * (2 * ny - 1) + (iy[:, None] - iy[None, :] + ny - 1)).ravel()
    nb = (2 * nx - 1) * (2 * ny - 1)
    out = np.zeros((F, P, P, nb), dtype=np.complex128)
    for f in range(F):
        X = np.asarray(x[:, f, :], dtype=np.complex128).reshape(T, P, M)
        for p in range(P):
            for q in range(P):
                Cm = X[:, p, :].T @ np.conj(X[:, q, :])  # [M, M]: sum_t x_p[j] conj(x_q[j'])
                out[f, p, q] = np.bincount(key, Cm.real.ravel(), nb) + 1j * np.bincount(key, Cm.imag.ravel(), nb)
    return out.reshape(F, P, P, 2 * nx - 1, 2 * ny - 1)
