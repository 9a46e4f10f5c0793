"""Plain float64 oracle of the beam-space ("digital pointing") variant (test infrastructure only;
no product path may import it).

Appendix A, steps 4-5: when the lowest level of the hierarchy consists of fully sampled
n_x x n_y antenna blocks, each block is first Fourier transformed in two dimensions (no zero
padding), which forms n_x n_y simultaneous pointings of every block; the correlation is then done
in all remaining dimensions with the padded-FFT method of Sec. II.  Readings:

* The lowest level is the last level of ``level_dims`` (its two axes are the last two hypercube
  axes, x then y).  Pointing b = (b_x, b_y), b_x < n_x, b_y < n_y, of the block at outer index
  tuple i is  B_b[i] = sum_{j_x, j_y} x[i, j_x, j_y] exp(-2 pi i (b_x j_x / n_x + b_y j_y / n_y))
  (the forward sign of the correlator's own transform).
* Each pointing is correlated like a channel over the outer axes (Sec. II.D, Eq. ProofEq2):
  V[f, Delta', b] = sum_t sum_i B_b[t, f, i] conj(B_b[t, f, i - Delta']), Delta' over the outer
  axes only, plain sums as for the hypercube.
* Output layout [F, 2n_1 - 1, ..., 2n_{d-2} - 1, n_x, n_y].
"""

from __future__ import annotations

import math
from typing import Sequence

import numpy as np

from .correlator import visibilities

__all__ = ["pointings", "beam_visibilities"]


def pointings(x, level_dims: Sequence[Sequence[int]]) -> np.ndarray:
    """B[t, f, i_outer, b_x, b_y]: the unpadded 2-D DFT of every lowest-level block (Appendix A step 4)."""
    x = np.asarray(x)
    T, F, N = x.shape
    dims = [int(v) for ld in level_dims for v in ld]
    if math.prod(dims) != N:
        raise ValueError(f"prod(dims)={math.prod(dims)} != N={N}")
    nx, ny = dims[-2], dims[-1]
    blocks = x.reshape(T, F, N // (nx * ny), nx, ny).astype(np.complex128)
    return np.fft.fft2(blocks, axes=(-2, -1))


def beam_visibilities(x, level_dims: Sequence[Sequence[int]]) -> np.ndarray:
    """V[f, Delta_outer..., b_x, b_y]: each pointing correlated over the outer levels (Appendix A step 5)."""
    x = np.asarray(x)
    T, F, N = x.shape
    dims = [int(v) for ld in level_dims for v in ld]
    if len(level_dims) < 2:
        raise ValueError("the beam-space variant needs at least one level above the blocks")
    outer = dims[:-2]
    nx, ny = dims[-2], dims[-1]
    B = pointings(x, level_dims)  # [T, F, No, nx, ny]
    No = B.shape[2]
    # every (channel, pointing) is a channel of the outer grid
    xb = np.transpose(B, (0, 1, 3, 4, 2)).reshape(T, F * nx * ny, No)
    V = visibilities(xb, outer)  # [F * nx * ny, lags...]
    lag = tuple(2 * n - 1 for n in outer)
    V = V.reshape((F, nx, ny) + lag)
    return np.moveaxis(np.moveaxis(V, 1, -1), 1, -1)  # [F, lags..., nx, ny]
