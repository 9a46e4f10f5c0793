"""Pins of the baseline-fold oracle (oracle/layout.py) against closed forms, library
routines and brute force (Sec. II.D's fold, Sec. III's baseline distributions)."""

from __future__ import annotations

import itertools

import numpy as np
import pytest
import scipy.signal

import oracle
import skysim

LAYOUTS = skysim.PAPER_LAYOUTS


def _layout_map(level_dims, A):
    """The layout map l of Sec. III: one at every antenna position, as a 0/1 image (row y, column x)."""
    r = np.rint(oracle.layout_positions(level_dims, A)).astype(np.int64)
    r -= r.min(axis=0)
    img = np.zeros((r[:, 1].max() + 1, r[:, 0].max() + 1))
    img[r[:, 1], r[:, 0]] = 1.0
    return img


def _ones_vis(level_dims):
    dims = [n for ld in level_dims for n in ld]
    x = np.ones((1, 1, int(np.prod(dims))), dtype=np.complex128)
    return oracle.visibilities(x, dims)


@pytest.mark.parametrize("name", ["3-level", "Blocks"])
def test_distribution_is_scipy_correlation_of_the_layout_map(name):
    """d = l * l^- (Sec. III) equals scipy's FFT 2-D correlation of the 0/1 layout image."""
    ld, A = LAYOUTS[name]
    d = oracle.baseline_distribution(ld, A)
    img = _layout_map(ld, A)
    ref = scipy.signal.correlate(img, img, mode="full", method="fft")
    assert ref.shape == d.shape
    assert np.array_equal(np.rint(ref).astype(np.int64), d)


def test_plank_closed_form():
    """Plank (single 512 x 32 block, unit lattice): d(x, y) = (512 - |x|)(32 - |y|) (the all-ones
    hypercube of one level, Sec. II.D)."""
    ld, A = LAYOUTS["Plank"]
    d = oracle.baseline_distribution(ld, A)
    y, x = np.indices(d.shape)
    assert d.shape == (63, 1023)
    assert np.array_equal(d, (512 - np.abs(x - 511)) * (32 - np.abs(y - 31)))


def test_strips_and_blocks_closed_forms():
    """Strips: nonzero only at x = 16 i, d = (32 - |i|)(512 - |y|).  Blocks (lattice 200 > 2 * 15, so
    every difference decomposes uniquely): d = (2-|D1|)(2-|D2|)(16-|D3|)(16-|D4|) at
    (200 D1 + D3, 200 D2 + D4)."""
    ld, A = LAYOUTS["Strips"]
    d = oracle.baseline_distribution(ld, A)
    cy, cx = d.shape[0] // 2, d.shape[1] // 2
    ref = np.zeros_like(d)
    for i in range(-31, 32):
        ref[:, cx + 16 * i] = (32 - abs(i)) * (512 - np.abs(np.arange(d.shape[0]) - cy))
    assert np.array_equal(d, ref)
    ld, A = LAYOUTS["Blocks"]
    d = oracle.baseline_distribution(ld, A)
    cy, cx = d.shape[0] // 2, d.shape[1] // 2
    ref = np.zeros_like(d)
    for D1, D2, D3, D4 in itertools.product(range(-1, 2), range(-1, 2), range(-15, 16), range(-15, 16)):
        ref[cy + 200 * D2 + D4, cx + 200 * D1 + D3] = (2 - abs(D1)) * (2 - abs(D2)) * (16 - abs(D3)) * (16 - abs(D4))
    assert np.array_equal(d, ref)


def test_distribution_brute_force_small_three_level():
    """Pure-Python pair loop on a reduced 3-level layout (same lattice vectors, fewer positions)."""
    ld = [[2, 2], [2, 2], [3, 2]]
    A = LAYOUTS["3-level"][1]
    r = [tuple(int(v) for v in p) for p in np.rint(oracle.layout_positions(ld, A))]
    d = oracle.baseline_distribution(ld, A)
    cy, cx = d.shape[0] // 2, d.shape[1] // 2
    ref = np.zeros_like(d)
    for a in r:
        for b in r:
            ref[cy + a[1] - b[1], cx + a[0] - b[0]] += 1
    assert np.array_equal(d, ref)


@pytest.mark.parametrize("name", ["3-level", "Blocks"])
def test_fold_of_the_hypercube_is_the_distribution(name):
    """Sec. II.D's theorem: folding the index-difference hypercube of an all-ones input by
    b = sum_k Delta_k a_k gives l * l^-, also where cells collide (3-level, Fig. 1)."""
    ld, A = LAYOUTS[name]
    g = oracle.fold(_ones_vis(ld), ld, A)[0]
    d = oracle.baseline_distribution(ld, A)
    assert np.array_equal(g.imag, np.zeros_like(d))
    assert np.array_equal(g.real, d.astype(np.float64))


@pytest.mark.parametrize(
    "ld, A",
    [
        ([[64, 8]], [[[1, 0], [0, 1]]]),  # a reduced Plank
        ([[8, 64]], [[[16, 0], [0, 1]]]),  # reduced Strips
    ],
)
def test_fold_reduced_plank_and_strips(ld, A):
    g = oracle.fold(_ones_vis(ld), ld, A)[0]
    assert np.array_equal(g.real, oracle.baseline_distribution(ld, A).astype(np.float64))


def test_three_level_collisions():
    """The 3-level layout has 28,125 index-difference cells but fewer distinct separations; the fold
    puts the colliding cells into one pixel (e.g. 4 a_1 = -4 a_1 + a_2 = (4, 0))."""
    ld, A = LAYOUTS["3-level"]
    r = np.rint(oracle.layout_positions(ld, A)).astype(np.int64)
    diffs = {(int(a[0] - b[0]), int(a[1] - b[1])) for a in r for b in r}
    d = oracle.baseline_distribution(ld, A)
    assert int((d > 0).sum()) == len(diffs) < 28125
    V = _ones_vis(ld)[0]
    # cell (level 2 x lag +1, level 2 y lag 0, level 3 x lag -4) and (level 3 x lag +4)
    c0 = [2, 2, 2, 2, 4, 2]
    a = list(c0)
    a[4] += 4
    b = list(c0)
    b[2] += 1
    b[4] -= 4
    g = oracle.fold(V[None], ld, A)[0]
    cy, cx = g.shape[0] // 2, g.shape[1] // 2
    assert g[cy, cx + 4].real == V[tuple(a)].real + V[tuple(b)].real == d[cy, cx + 4]


def test_fold_of_sky_visibilities_conserves_sum_and_symmetry():
    """For any input the fold keeps the sum over cells and maps the Hermitian hypercube to a
    Hermitian image g(-b) = conj g(b)."""
    ld, A = [[3, 2], [4, 3]], [[[9, -2], [3, 7]], [[1, 0], [0, 1]]]
    dims = [n for l in ld for n in l]
    rng = np.random.default_rng(5)
    x = rng.integers(-7, 8, (4, 2, int(np.prod(dims)))) + 1j * rng.integers(-7, 8, (4, 2, int(np.prod(dims))))
    V = oracle.visibilities(x, dims)
    g = oracle.fold(V, ld, A)
    assert np.allclose(g.sum(axis=(1, 2)), V.reshape(2, -1).sum(axis=1), atol=1e-9)
    assert np.allclose(g, np.conj(g[:, ::-1, ::-1]), atol=1e-9)


def test_fold_coarse_pixels_groups_by_rounded_baseline():
    """du = dv = 4: a cell lands in pixel rint(b / 4) (brute force over cells)."""
    ld, A = LAYOUTS["Blocks"]
    V = _ones_vis(ld)
    g = oracle.fold(V, ld, A, du=4.0, dv=4.0)[0]
    b = oracle.baselines(ld, A)
    cy, cx = oracle.image_centre(ld, A, 4.0, 4.0)
    ref = np.zeros(g.shape)
    for idx in np.ndindex(V.shape[1:]):
        bx, by = b[idx]
        ref[cy + int(np.rint(by / 4.0)), cx + int(np.rint(bx / 4.0))] += V[(0,) + idx].real
    assert np.array_equal(g.real, ref)
    assert g.real.sum() == 1024**2


def test_radial_profile_closed_form_plank():
    """Bin 0 holds the origin (N), bin 1 the pixels with 1 <= |b| < 2: (+-1, 0), (0, +-1), (+-1, +-1)."""
    ld, A = LAYOUTS["Plank"]
    y, x = np.indices((63, 1023))
    d = ((512 - np.abs(x - 511)) * (32 - np.abs(y - 31))).astype(np.float64)
    h = oracle.radial_profile(d)
    assert h[0] == 16384
    assert h[1] == 2 * 511 * 32 + 2 * 512 * 31 + 4 * 511 * 31
    assert h.sum() == 16384**2
    assert h.shape[0] == int(np.floor(np.hypot(511, 31))) + 1


def test_radial_profile_brute_force_and_scale():
    rng = np.random.default_rng(2)
    d = rng.random((2, 7, 9))
    for du, dv, dr, scale in [(1.0, 1.0, 1.0, 1.0), (2.0, 0.5, 1.5, 0.7)]:
        h = oracle.radial_profile(d, du, dv, dr, scale)
        ref = np.zeros_like(h)
        for c in range(2):
            for iy in range(7):
                for ix in range(9):
                    r = ((((ix - 4) * du) ** 2 + ((iy - 3) * dv) ** 2) ** 0.5) * scale / dr
                    ref[c, int(r // 1)] += d[c, iy, ix]
        assert np.allclose(h, ref, atol=1e-12)


def test_boxcar_against_convolution():
    rng = np.random.default_rng(3)
    h = rng.random((3, 40))
    for w in (1, 3, 5, 9):
        ref = np.stack([np.convolve(row, np.ones(w) / w, mode="same") for row in h])
        assert np.allclose(oracle.boxcar(h, w), ref, atol=1e-12)
    ones = oracle.boxcar(np.ones(10), 5)
    assert np.allclose(ones, [3 / 5, 4 / 5, 1, 1, 1, 1, 1, 1, 4 / 5, 3 / 5])
    with pytest.raises(ValueError):
        oracle.boxcar(h, 4)


def test_zero_origin_and_asinh_map():
    ld, A = LAYOUTS["Blocks"]
    d = oracle.zero_origin(oracle.baseline_distribution(ld, A)[None].astype(np.float64))
    assert d[0, 215, 215] == 0 and d.sum() == 1024**2 - 1024
    m = oracle.asinh_map(d)
    assert np.isclose(m.max(), np.arcsinh(4.0)) and m[0, 215, 215] == 0
    # the map is invertible: d = d_max sinh(m) / 4
    assert np.allclose(np.sinh(m) * d.max() / 4.0, d, rtol=1e-12, atol=1e-9)
    assert np.array_equal(np.argsort(m.ravel(), kind="stable"), np.argsort(d.ravel(), kind="stable"))
