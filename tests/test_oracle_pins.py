"""Pins of the CPU oracle against things other than itself.

Each pin is a function of a visibility routine ``vis(x, dims)`` so that the
same pins can be run against deliberately broken copies of the oracle (the
mutation tests at the bottom): every plausible mistake -- a dropped conjugate,
a flipped sign of Delta, the wrong strides, a transposed product, a lost
autocorrelation -- must fail at least one pin.
"""

import itertools
import math

import numpy as np
import pytest
import scipy.signal

import oracle
import skysim
from oracle import correlator as oc
from tests.conftest import load_golden

RNG = np.random.default_rng(1234)


def rand_cplx(shape, rng=RNG, ints=True):
    if ints:
        return rng.integers(-7, 8, shape) + 1j * rng.integers(-7, 8, shape)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def lag_grids(dims):
    return np.meshgrid(*[np.arange(-(n - 1), n) for n in dims], indexing="ij")


# ---------------------------------------------------------------------------
# Pins, each parameterised by the routine under test.
# ---------------------------------------------------------------------------


def pin_paper_example(vis):
    """Sec. II.C Eqs. ConvolutionExampleEq1/Eq2: the printed integer results."""
    g = load_golden("paper_toy_example.txt")
    v1 = np.array(g["voltages_1d"][0])
    out1 = vis(v1.reshape(1, 1, -1).astype(complex), (v1.size,))[0]
    assert np.array_equal(out1.real, np.array(g["vis_1d"][0])) and not out1.imag.any()
    h = np.array(g["hypercube"])
    out2 = vis(h.reshape(1, 1, -1).astype(complex), h.shape)[0]
    assert np.array_equal(out2.real, np.array(g["vis_2d"])) and not out2.imag.any()


def pin_plane_wave(vis):
    """Closed form: x_j = A e^{i phi_t} e^{2 pi i kappa.j} gives V = T|A|^2 e^{2 pi i kappa.Delta} prod(n_k-|Delta_k|)."""
    dims = (3, 4, 2)
    kappa = np.array([0.137, -0.291, 0.402])
    T, Aamp = 5, 1.7
    idx = np.indices(dims).reshape(3, -1).T
    base = Aamp * np.exp(2j * np.pi * idx @ kappa)
    phis = RNG.uniform(0, 2 * np.pi, T)
    x = (np.exp(1j * phis)[:, None] * base[None, :])[:, None, :]
    V = vis(x, dims)[0]
    G = lag_grids(dims)
    weight = np.prod([n - np.abs(g) for n, g in zip(dims, G)], axis=0)
    expect = T * Aamp**2 * np.exp(2j * np.pi * sum(k * g for k, g in zip(kappa, G))) * weight
    assert np.allclose(V, expect, rtol=0, atol=1e-9)


def pin_all_ones(vis):
    """The layout map of ones (Sec. III baseline distribution): V = T prod(n_k - |Delta_k|); sum V = T N^2."""
    dims = (3, 2, 4)
    T = 3
    N = math.prod(dims)
    V = vis(np.ones((T, 1, N), complex), dims)[0]
    G = lag_grids(dims)
    assert np.array_equal(V.real, T * np.prod([n - np.abs(g) for n, g in zip(dims, G)], axis=0))
    assert V.real.sum() == T * N * N


def pin_zero_lag_and_sum(vis):
    """V[0] = sum |x|^2 (total power) and sum_Delta V = sum_t |sum_a x_a|^2, exactly for integers."""
    dims = (4, 3, 3)
    T, F = 4, 2
    x = rand_cplx((T, F, math.prod(dims)))
    V = vis(x, dims)
    centre = tuple(n - 1 for n in dims)
    for f in range(F):
        assert V[f][centre] == np.sum(x[:, f].real ** 2 + x[:, f].imag ** 2)
        s = x[:, f].sum(axis=1)
        assert V[f].sum() == np.sum(s.real**2 + s.imag**2)


def pin_hermitian(vis):
    """V[-Delta] = conj V[Delta] for complex voltages."""
    dims = (3, 5)
    x = rand_cplx((3, 1, 15))
    V = vis(x, dims)[0]
    assert np.array_equal(V[::-1, ::-1], V.conj())


def pin_two_deltas(vis):
    """Voltages at antennas p and q only: V[p-q] = x_p conj(x_q), V[q-p] = its conjugate, V[0] = |x_p|^2+|x_q|^2."""
    dims = (3, 4, 2)
    p, q = (2, 1, 0), (0, 3, 1)
    xp, xq = 2 + 3j, -1 + 5j
    x = np.zeros(dims, complex)
    x[p], x[q] = xp, xq
    V = vis(x.reshape(1, 1, -1), dims)[0]
    expect = np.zeros(V.shape, complex)
    c = tuple(n - 1 for n in dims)
    expect[tuple(a - b + o for a, b, o in zip(p, q, c))] = xp * np.conj(xq)
    expect[tuple(b - a + o for a, b, o in zip(p, q, c))] = xq * np.conj(xp)
    expect[c] = (xp * np.conj(xp) + xq * np.conj(xq)).real
    assert np.array_equal(V, expect)


def pin_separable(vis):
    """x = u (x) v gives V = V_u (x) V_v (single sample)."""
    du, dv = (3, 2), (4,)
    u = rand_cplx(du)
    v = rand_cplx(dv)
    x = np.multiply.outer(u, v)
    V = vis(x.reshape(1, 1, -1), du + dv)[0]
    Vu = vis(u.reshape(1, 1, -1), du)[0]
    Vv = vis(v.reshape(1, 1, -1), dv)[0]
    assert np.array_equal(V, np.multiply.outer(Vu, Vv))


def pin_axis_permutation_and_time_linearity(vis):
    """Permuting the antenna axes permutes the visibility axes; the time sum splits into sub-sums."""
    dims = (3, 2, 4)
    T = 3
    x = np.stack([rand_cplx(dims) for _ in range(T)])  # [T, *dims]
    V = vis(x.reshape(T, 1, -1), dims)[0]
    perm = (2, 0, 1)
    xp = np.transpose(x, (0,) + tuple(1 + k for k in perm))
    Vp = vis(np.ascontiguousarray(xp).reshape(T, 1, -1), tuple(dims[k] for k in perm))[0]
    assert np.array_equal(Vp, np.transpose(V, perm))
    V1 = vis(x[:1].reshape(1, 1, -1), dims)[0]
    V2 = vis(x[1:].reshape(T - 1, 1, -1), dims)[0]
    assert np.array_equal(V, V1 + V2)


def pin_library_correlate(vis):
    """numpy.correlate (1-D) and scipy.signal.correlate (N-D, direct) of a single sample."""
    a = rand_cplx(7)
    V = vis(a.reshape(1, 1, -1), (7,))[0]
    assert np.array_equal(V, np.correlate(a, a, mode="full"))
    dims = (3, 4, 2)
    x = rand_cplx(dims)
    V = vis(x.reshape(1, 1, -1), dims)[0]
    assert np.array_equal(V, scipy.signal.correlate(x, x, mode="full", method="direct"))


def pin_padded_fft(vis):
    """Zero-pad 2x, FFT, square modulus, inverse FFT (numpy fftn), summed over time: rounds to the integers."""
    dims = (4, 3, 2)
    T = 3
    x = rand_cplx((T, 1, math.prod(dims)))
    V = vis(x, dims)[0]
    m = tuple(2 * n for n in dims)
    P = np.zeros(m)
    for t in range(T):
        P += np.abs(np.fft.fftn(x[t, 0].reshape(dims), s=m, axes=tuple(range(len(m))))) ** 2
    g = np.fft.ifftn(P)
    # lag Delta sits at index Delta mod m_k
    G = lag_grids(dims)
    got = g[tuple(np.mod(gk, mk) for gk, mk in zip(G, m))]
    assert np.array_equal(np.round(got.real) + 1j * np.round(got.imag), V)


def brute_force(x, dims):
    """Pure-Python double loop over all antenna pairs (tiny inputs only)."""
    T, F, N = x.shape
    idx = list(itertools.product(*[range(n) for n in dims]))
    out = np.zeros((F,) + tuple(2 * n - 1 for n in dims), complex)
    for f in range(F):
        for t in range(T):
            for a in range(N):
                for b in range(N):
                    cell = tuple(ia - ib + n - 1 for ia, ib, n in zip(idx[a], idx[b], dims))
                    out[(f,) + cell] += x[t, f, a] * np.conj(x[t, f, b])
    return out


def pin_brute_force(vis):
    """Pure-Python pair loop on tiny grids with d up to 6."""
    for dims in [(2,), (3, 2), (2, 3, 2), (2, 1, 3), (2, 2, 2, 2, 2, 2), (3, 1, 2, 2)]:
        N = math.prod(dims)
        x = rand_cplx((2, 2, N))
        assert np.array_equal(vis(x, dims), brute_force(x, dims)), dims


def pin_sparse_embedding(vis):
    """The hypercube theorem (Sec. II.B, II.D): correlating antennas placed in a mostly empty
    physical grid equals G mapped through b(Delta) = sum_k Delta_k a_k, summed over colliding cells.

    Layouts: the toy (a=(1,0),(6,0)), the interleaved grid (a=(5,0),(7,0), i in 1..4, Sec. II.D),
    the four "Blocks" (Sec. III) scaled down to 6x6 blocks, and the 3-level layout of Fig. 1."""
    cases = [
        # (level_dims, A per level) -- columns of A are the lattice vectors of that level
        ([[2, 1], [3, 1]], [[[6, 0], [0, 1]], [[1, 0], [0, 1]]]),
        ([[4, 1], [4, 1]], [[[7, 0], [0, 1]], [[5, 0], [0, 1]]]),
        ([[2, 2], [6, 6]], [[[30, 0], [0, 30]], [[1, 0], [0, 1]]]),
        ([[3, 3], [3, 3], [5, 3]], [[[40, -10], [10, 40]], [[8, 2], [0, 8]], [[1, 0], [0, 1]]]),
    ]
    for level_dims, A in cases:
        dims = [n for ld in level_dims for n in ld]
        N = math.prod(dims)
        x = rand_cplx((2, 1, N))
        V = vis(x, dims)[0]
        pos = np.rint(skysim.positions(level_dims, A)).astype(int)
        lo = pos.min(axis=0)
        ext = pos.max(axis=0) - lo + 1
        P = np.zeros(tuple(2 * ext))
        for t in range(2):
            img = np.zeros(tuple(ext), complex)
            img[pos[:, 0] - lo[0], pos[:, 1] - lo[1]] = x[t, 0]
            P += np.abs(np.fft.fft2(img, s=tuple(2 * ext))) ** 2
        g = np.fft.ifft2(P)
        g = np.round(g.real) + 1j * np.round(g.imag)
        b = np.rint(oracle.baselines(level_dims, A)).astype(int)
        folded = np.zeros(g.shape, complex)
        np.add.at(folded, (np.mod(b[..., 0], 2 * ext[0]), np.mod(b[..., 1], 2 * ext[1])), V)
        assert np.array_equal(folded, g), level_dims


PINS = [
    pin_paper_example,
    pin_plane_wave,
    pin_all_ones,
    pin_zero_lag_and_sum,
    pin_hermitian,
    pin_two_deltas,
    pin_separable,
    pin_axis_permutation_and_time_linearity,
    pin_library_correlate,
    pin_padded_fft,
    pin_brute_force,
    pin_sparse_embedding,
]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_oracle_pin(pin):
    pin(oracle.visibilities)


def _grouped(x, dims):
    """visibilities_by_outer_lag with the outer half of the axes as tiles (a 1-D grid gains a unit outer axis)."""
    dims = tuple(int(n) for n in dims)
    if len(dims) == 1:
        v = oracle.visibilities_by_outer_lag(x, (1,) + dims, 1)
        return v.reshape((v.shape[0],) + oracle.lag_shape(dims))
    return oracle.visibilities_by_outer_lag(x, dims, max(1, len(dims) // 2))


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_grouped_oracle_pin(pin):
    """The pair sum grouped by outer-level lag (used at full three-level size) passes every pin itself."""
    pin(_grouped)


@pytest.mark.parametrize("dims,n_outer", [((3, 2, 4, 3), 1), ((3, 2, 4, 3), 3), ((2, 2, 3, 3, 2, 2), 2)])
def test_grouped_oracle_every_split(dims, n_outer):
    x = rand_cplx((3, 2, math.prod(dims)))
    assert np.array_equal(oracle.visibilities_by_outer_lag(x, dims, n_outer), oracle.visibilities(x, dims))


def test_panelled_equals_unpanelled():
    dims = (4, 4, 3)
    x = rand_cplx((3, 2, 48))
    assert np.array_equal(oracle.visibilities(x, dims, panel=5), oracle.visibilities(x, dims, panel=4096))


# ---------------------------------------------------------------------------
# The per-cell and Fourier-cell oracles, pinned to the full oracle and to fftn.
# ---------------------------------------------------------------------------


def test_visibility_cells_match_full():
    dims = (3, 4, 2)
    x = rand_cplx((3, 2, 24))
    V = oracle.visibilities(x, dims)
    G = lag_grids(dims)
    cells = np.stack([g.ravel() for g in G], axis=1)
    got = oracle.visibility_cells(x, dims, cells)
    assert np.array_equal(got, V.reshape(2, -1))
    # out-of-range lags are empty
    assert not oracle.visibility_cells(x, dims, [[3, 0, 0], [0, -4, 0]]).any()


def test_fourier_power_matches_fftn_and_wiener_khinchin():
    dims = (3, 4)
    T = 4
    x = rand_cplx((T, 1, 12), ints=False)
    m = (6, 8)
    kap = np.array([[0, 0], [1, 3], [5, 7], [2, 0]])
    P = oracle.fourier_power(x, dims, kap, m)[0]
    ref = sum(np.abs(np.fft.fftn(x[t, 0].reshape(dims), s=m, axes=tuple(range(len(m))))) ** 2 for t in range(T))
    assert np.allclose(P, ref[kap[:, 0], kap[:, 1]], rtol=1e-12)
    V = oracle.visibilities(x, dims)[0]
    G = lag_grids(dims)
    for q, k in enumerate(kap):
        wk = np.sum(V * np.exp(-2j * np.pi * (k[0] * G[0] / m[0] + k[1] * G[1] / m[1])))
        assert abs(wk - P[q]) < 1e-9 * abs(P[q]) + 1e-9
        assert abs(wk.imag) < 1e-9 * abs(P[q]) + 1e-9


def test_baselines_are_position_differences():
    level_dims = [[3, 2], [2, 4]]
    A = np.stack([skysim.lattice(5.0, 15.0, 0.2), skysim.lattice(0.5, 0.0, 0.0)])
    pos = skysim.positions(level_dims, A)
    b = oracle.baselines(level_dims, A)
    dims = [n for ld in level_dims for n in ld]
    idx = np.indices(dims).reshape(4, -1).T
    for a, c in RNG.integers(0, pos.shape[0], (40, 2)):
        cell = tuple(idx[a] - idx[c] + np.array(dims) - 1)
        assert np.allclose(b[cell], pos[a] - pos[c], atol=1e-12)


def test_fig1_layout_has_colliding_cells():
    """In the 3-level layout of Fig. 1 some distinct index differences share a physical baseline,
    e.g. (level-1 x lag 4) and (level-1 x lag -4, level-2 x lag 1): 4 a_1 = a_2 - 4 a_1 ... per Eq. GridEq."""
    level_dims = [[3, 3], [3, 3], [5, 3]]
    A = [[[40, -10], [10, 40]], [[8, 2], [0, 8]], [[1, 0], [0, 1]]]
    b = np.rint(oracle.baselines(level_dims, A)).astype(int).reshape(-1, 2)
    assert len({tuple(v) for v in b}) < b.shape[0]


# ---------------------------------------------------------------------------
# Sample formats.
# ---------------------------------------------------------------------------


def test_decoders_hand_values():
    raw = np.array([0x7F, 0x88, 0x01, 0xF9], dtype=np.uint8)
    got = oracle.decode_ci4(raw, 1, 1, 4)[0, 0]
    assert list(got) == [7 - 1j, -8 - 8j, 0 + 1j, -1 - 7j]
    raw8 = np.array([127, -128, -3, 5], dtype=np.int8)
    assert list(oracle.decode_ci8(raw8, 1, 1, 2)[0, 0]) == [127 - 128j, -3 + 5j]
    rawf = np.array([1.5, -2.25], dtype=np.float32)
    assert list(oracle.decode_cf32(rawf, 1, 1, 1)[0, 0]) == [1.5 - 2.25j]


# ---------------------------------------------------------------------------
# Mutation tests: broken oracles must fail at least one pin.
# ---------------------------------------------------------------------------


def _mutant(kind):
    def vis(x, dims):
        x = np.asarray(x, dtype=complex)
        T, F, N = x.shape
        out_shape = tuple(2 * n - 1 for n in dims)
        idx = np.indices(dims).reshape(len(dims), -1).T
        strides = oc._row_major_strides(out_shape)
        if kind == "input_strides":
            strides = oc._row_major_strides(dims)
        c = idx @ strides
        c0 = int(np.sum((np.asarray(dims) - 1) * strides))
        V = np.zeros((F, math.prod(out_shape)), complex)
        for f in range(F):
            X = x[:, f, :]
            if kind == "no_conj":
                C = X.T @ X
            elif kind == "transposed":
                C = X.T.conj() @ X
            else:
                C = X.T @ X.conj()
            if kind == "no_autos":
                np.fill_diagonal(C, 0)
            sgn = -1 if kind == "flip_sign" else 1
            key = sgn * (c[:, None] - c[None, :]) + c0
            key = np.clip(key, 0, V.shape[1] - 1).ravel()
            V[f] += np.bincount(key, C.real.ravel(), V.shape[1]) + 1j * np.bincount(key, C.imag.ravel(), V.shape[1])
        return V.reshape((F,) + out_shape)

    return vis


@pytest.mark.parametrize("kind", ["no_conj", "transposed", "flip_sign", "input_strides", "no_autos"])
def test_pins_catch_planted_mistake(kind):
    bad = _mutant(kind)
    failed = []
    for pin in PINS:
        try:
            pin(bad)
        except (AssertionError, ValueError, IndexError):
            failed.append(pin.__name__)
    assert failed, f"no pin caught mutant {kind}"


def test_mutant_harness_is_faithful():
    """The unmutated copy used by the mutation tests passes every pin (so failures above are the mutation's)."""
    good = _mutant("none")
    for pin in PINS:
        pin(good)
