"""Plain float64 oracle of the physical-baseline fold and the baseline-distribution
experiment (test infrastructure only; no product path may import it).

Sec. II.D proves that the hypercube of index differences G_Delta holds, for a
layout whose antenna separations decompose uniquely, every physical baseline
b = sum_k Delta_k a_k exactly once; where two index differences land on the
same physical separation (the Fig. 1 layout does this), the physical
correlation is the sum of the hypercube cells that share it.  Sec. III draws
each example layout's two-dimensional baseline distribution d, the layout map
l (one at every antenna) correlated with its parity reversal, d = l * l^-,
with the origin set to zero and an intensity scale proportional to
asinh(4 d / d_max); it then bins d radially into a one-dimensional
distribution, smoothed in the comparison figure with a 5 m sliding boxcar.

Readings where the paper does not fix the detail:

* Pixels.  A baseline b = (b_x, b_y) is folded into pixel
  (rint(b_x / du), rint(b_y / dv)), rint rounding half to even.  With
  integer lattice vectors and du = dv = 1 this is the exact fold of Sec. II.D.
  Images are [ny, nx] arrays, row = y, column = x, with the zero baseline at
  (cy, cx) = (rint(Y / dv), rint(X / du)), X = sum |a_x| (n - 1) over the
  lattice vectors (the largest |b_x|), likewise Y.
* Radial bins.  Pixel (ix, iy) (offsets from the centre) lies in bin
  k = floor(sqrt((ix du)^2 + (iy dv)^2) * scale / dr): bins of width dr after
  the radii are multiplied by ``scale`` (the comparison figure rescales every
  layout to the same largest baseline).  Bin k sums the pixels' values.
* Boxcar.  A centred sliding mean over ``width`` (odd) bins, bins beyond
  either end counting as zero.
* asinh map.  d_max is the largest pixel after the origin is zeroed; the map
  is asinh(4 d / d_max), per channel.
"""

from __future__ import annotations

from typing import Sequence

import numpy as np

from .correlator import baselines

__all__ = [
    "layout_positions",
    "image_centre",
    "baseline_distribution",
    "fold",
    "zero_origin",
    "asinh_map",
    "radial_profile",
    "boxcar",
]


def layout_positions(level_dims: Sequence[Sequence[int]], A) -> np.ndarray:
    """Antenna positions r = sum_levels A_l (i_lx, i_ly) (Sec. II.D Eq. GridEq), [N, 2],
    row-major over (level 0 x, level 0 y, level 1 x, ...)."""
    level_dims = [tuple(int(v) for v in ld) for ld in level_dims]
    A = np.asarray(A, dtype=np.float64).reshape(len(level_dims), 2, 2)
    dims = [n for ld in level_dims for n in ld]
    idx = np.indices(dims).reshape(len(dims), -1).T
    r = np.zeros((idx.shape[0], 2), dtype=np.float64)
    for lvl in range(len(level_dims)):
        ix = idx[:, 2 * lvl].astype(np.float64)
        iy = idx[:, 2 * lvl + 1].astype(np.float64)
        r[:, 0] += A[lvl, 0, 0] * ix + A[lvl, 0, 1] * iy
        r[:, 1] += A[lvl, 1, 0] * ix + A[lvl, 1, 1] * iy
    return r


def image_centre(level_dims: Sequence[Sequence[int]], A, du: float = 1.0, dv: float = 1.0) -> tuple[int, int]:
    """(cy, cx): pixel of the zero baseline; the image is (2 cy + 1) x (2 cx + 1)."""
    level_dims = [tuple(int(v) for v in ld) for ld in level_dims]
    A = np.asarray(A, dtype=np.float64).reshape(len(level_dims), 2, 2)
    X = Y = 0.0
    for lvl, (nx, ny) in enumerate(level_dims):
        X += abs(A[lvl, 0, 0]) * (nx - 1) + abs(A[lvl, 0, 1]) * (ny - 1)
        Y += abs(A[lvl, 1, 0]) * (nx - 1) + abs(A[lvl, 1, 1]) * (ny - 1)
    return int(np.rint(Y / dv)), int(np.rint(X / du))


def baseline_distribution(level_dims: Sequence[Sequence[int]], A, chunk: int = 256) -> np.ndarray:
    """d = l * l^- for a layout on the integer grid (Sec. III): d[r] counts the ordered
    antenna pairs (a, b) with r_a - r_b = r, straight from the positions.

    Returns int64 [2 cy + 1, 2 cx + 1] with the zero separation at (cy, cx).
    The origin holds N (each antenna paired with itself).  Positions must be
    integers.
    """
    r = layout_positions(level_dims, A)
    if not np.all(r == np.rint(r)):
        raise ValueError("baseline_distribution needs integer antenna positions")
    r = r.astype(np.int64)
    cy, cx = image_centre(level_dims, A)
    ny, nx = 2 * cy + 1, 2 * cx + 1
    counts = np.zeros(ny * nx, dtype=np.int64)
    for s in range(0, r.shape[0], chunk):
        dx = r[s : s + chunk, None, 0] - r[None, :, 0]
        dy = r[s : s + chunk, None, 1] - r[None, :, 1]
        counts += np.bincount(((dy + cy) * nx + (dx + cx)).ravel(), minlength=ny * nx)
    return counts.reshape(ny, nx)


def fold(vis, level_dims: Sequence[Sequence[int]], A, du: float = 1.0, dv: float = 1.0) -> np.ndarray:
    """Physical-baseline fold of the hypercube (Sec. II.D): g[pixel] = sum of the cells
    Delta whose baseline b(Delta) = sum_k Delta_k a_k falls in that pixel.

    ``vis``: [F, 2n_1 - 1, ...] (the hypercube, centred).  Returns complex128
    [F, 2 cy + 1, 2 cx + 1].
    """
    vis = np.asarray(vis)
    b = baselines(level_dims, A)
    if vis.shape[1:] != b.shape[:-1]:
        raise ValueError(f"visibility cells {vis.shape[1:]} do not match the layout {b.shape[:-1]}")
    cy, cx = image_centre(level_dims, A, du, dv)
    ny, nx = 2 * cy + 1, 2 * cx + 1
    px = np.rint(b[..., 0] / du).astype(np.int64).ravel() + cx
    py = np.rint(b[..., 1] / dv).astype(np.int64).ravel() + cy
    out = np.zeros((vis.shape[0], ny, nx), dtype=np.complex128)
    for f in range(vis.shape[0]):
        np.add.at(out[f], (py, px), vis[f].ravel())
    return out


def zero_origin(image) -> np.ndarray:
    """Copy of ``image`` [..., ny, nx] with the central (zero-baseline) pixel set to 0 (Sec. III)."""
    out = np.array(image, copy=True)
    ny, nx = out.shape[-2:]
    out[..., ny // 2, nx // 2] = 0
    return out


def asinh_map(d) -> np.ndarray:
    """asinh(4 d / d_max) per leading index (Sec. III's intensity scale); all-zero planes map to 0."""
    d = np.asarray(d, dtype=np.float64)
    dmax = d.reshape(d.shape[:-2] + (-1,)).max(axis=-1)
    dmax = np.where(dmax > 0, dmax, 1.0)
    return np.arcsinh(4.0 * d / dmax[..., None, None])


def radial_profile(d, du: float = 1.0, dv: float = 1.0, dr: float = 1.0, scale: float = 1.0) -> np.ndarray:
    """One-dimensional baseline distribution (Sec. III): the pixels of ``d`` [..., ny, nx]
    summed in radial bins k = floor(|b| * scale / dr), b the pixel's baseline.
    Returns [..., nbins] with nbins = (largest k) + 1."""
    d = np.asarray(d, dtype=np.float64)
    ny, nx = d.shape[-2:]
    iy, ix = np.indices((ny, nx))
    bx = (ix - nx // 2).astype(np.float64) * du
    by = (iy - ny // 2).astype(np.float64) * dv
    k = np.floor(np.sqrt(bx * bx + by * by) * scale / dr).astype(np.int64).ravel()
    nb = int(k.max()) + 1
    flat = d.reshape(-1, ny * nx)
    out = np.stack([np.bincount(k, weights=row, minlength=nb) for row in flat])
    return out.reshape(d.shape[:-2] + (nb,))


def boxcar(h, width: int = 5) -> np.ndarray:
    """Centred sliding mean over ``width`` (odd) bins; bins beyond the ends count as zero
    (Sec. III's comparison figure smooths with a 5 m sliding bin)."""
    if width < 1 or width % 2 == 0:
        raise ValueError("boxcar width must be odd and positive")
    h = np.asarray(h, dtype=np.float64)
    half = width // 2
    pad = np.zeros(h.shape[:-1] + (h.shape[-1] + 2 * half,))
    pad[..., half : half + h.shape[-1]] = h
    out = np.zeros_like(h)
    for j in range(width):
        out += pad[..., j : j + h.shape[-1]]
    return out / width
