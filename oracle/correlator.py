"""Plain float64 oracle of the hierarchical-grid correlator (test infrastructure only).

Notation follows the paper.  An antenna sits at r = i_1 a_1 + i_2 a_2 + ...
(Sec. II.D, Eq. GridEq); its voltage at one time and one frequency band is
F_{i_1 i_2 ...}.  The visibility hypercube is

    G_Delta = sum_{i'} F_{i'} conj(F_{i' - Delta}),   Delta_k in [-(n_k-1), n_k-1]

(Sec. II.D, Eq. ProofEq2, with the index range stated right after it), i.e.
the product of every antenna pair summed over all pairs that share the same
index difference (Sec. II.A).  The conjugate on the second factor is what the
"square modulus" of Sec. II.A produces for complex voltages; for the paper's
real-valued toy example it is a no-op.  Observations at different times are
combined by summation (Sec. II.A), so every function here also sums over the
time axis.  Autocorrelations are included at Delta = 0 (the central value of
the toy example in Sec. II.C is the sum of squares).

Voltages are arrays x[T, F, N]: T time samples, F frequency channels and N
antennas, the antenna index being row-major over (i_1, ..., i_d).
"""

from __future__ import annotations

import math
from typing import Sequence

import numpy as np

__all__ = [
    "lag_shape",
    "visibilities",
    "visibilities_by_outer_lag",
    "visibility_cells",
    "fourier_power",
    "baselines",
    "decode",
    "decode_cf32",
    "decode_ci8",
    "decode_ci4",
]


def lag_shape(dims: Sequence[int]) -> tuple[int, ...]:
    """Shape of the visibility hypercube: 2 n_k - 1 lags per axis (Sec. II.D)."""
    return tuple(2 * int(n) - 1 for n in dims)


def _row_major_strides(shape: Sequence[int]) -> np.ndarray:
    strides = np.ones(len(shape), dtype=np.int64)
    for k in range(len(shape) - 2, -1, -1):
        strides[k] = strides[k + 1] * shape[k + 1]
    return strides


def _antenna_index_tuples(dims: Sequence[int]) -> np.ndarray:
    """[N, d] integer index tuples (i_1, ..., i_d) in row-major antenna order."""
    return np.indices(tuple(dims)).reshape(len(dims), -1).T.astype(np.int64)


def visibilities(x, dims: Sequence[int], panel: int = 2048) -> np.ndarray:
    """Visibility hypercube per channel, straight from the definition.

    For every channel f:  V_f[Delta] = sum_t sum_{j, j-Delta in grid} x_{t,f,j} conj(x_{t,f,j-Delta}).

    Steps (Sec. II.A; Sec. II.C Eq. ConvolutionDefEq; Sec. II.D Eq. ProofEq2):
      1. C[a, b] = sum_t x_{t,f,a} conj(x_{t,f,b})       (all antenna pairs, time summed)
      2. V[Delta] = sum over pairs (a, b) whose index tuples differ by Delta of C[a, b].

    Step 1 is one matrix product; step 2 is a histogram keyed by the index
    difference.  Rows of C are processed in panels of ``panel`` antennas so
    that the N x N matrix is never held whole.  Returns complex128
    [F, 2n_1-1, ..., 2n_d-1] with Delta_k stored at position Delta_k + n_k - 1.
    For integer voltages every product and partial sum is an integer below
    2**53, so the result is exact whatever order the product sums in.
    """
    x = np.asarray(x)
    T, F, N = x.shape
    dims = tuple(int(n) for n in dims)
    if math.prod(dims) != N:
        raise ValueError(f"prod(dims)={math.prod(dims)} != N={N}")
    out_shape = lag_shape(dims)
    n_cells = math.prod(out_shape)
    idx = _antenna_index_tuples(dims)
    lag_strides = _row_major_strides(out_shape)
    c = idx @ lag_strides  # position of each antenna's index tuple in lag units
    c0 = int(np.sum((np.asarray(dims) - 1) * lag_strides))  # position of Delta = 0
    V = np.zeros((F, n_cells), dtype=np.complex128)
    for f in range(F):
        X = np.asarray(x[:, f, :], dtype=np.complex128)  # T x N
        Xc = X.conj()
        for a0 in range(0, N, panel):
            a1 = min(N, a0 + panel)
            C = X[:, a0:a1].T @ Xc  # C[a, b] = sum_t x_a conj(x_b)
            key = (c[a0:a1, None] - c[None, :] + c0).ravel()
            V[f] += np.bincount(key, weights=C.real.ravel(), minlength=n_cells)
            V[f] += 1j * np.bincount(key, weights=C.imag.ravel(), minlength=n_cells)
    return V.reshape((F,) + out_shape)


def visibilities_by_outer_lag(x, dims: Sequence[int], n_outer: int) -> np.ndarray:
    """The visibility hypercube of ``visibilities``, with the pair sum grouped for large grids.

    Each index tuple j = (p, i) is split into its first ``n_outer`` indices p (a "tile" of the outer
    levels) and the remaining indices i.  The definition
        V[Delta] = sum_t sum_{pairs (j, j') with j - j' = Delta} x_{t,j} conj(x_{t,j'})
    then reads, for Delta = (dp, di),
        V[(dp, di)] = sum_{i - i' = di}  S_dp[i, i'],
        S_dp[i, i'] = sum_{tile pairs (p, q), p - q = dp}  sum_t x_{t,(p,i)} conj(x_{t,(q,i')}),
    because the histogram over di is linear in the pair products: the products of all tile pairs sharing
    one outer difference dp are added first (one matrix product over the tiles stacked along the time axis)
    and binned once.  Only dp on the non-negative half of the outer lag grid (row-major position at or
    after dp = 0) is summed; the rest follows from swapping the two antennas of every pair, which
    conjugates the product and negates Delta:  V[-Delta] = conj V[Delta].  No other step differs from
    ``visibilities``; for integer voltages the result is exact.  Returns complex128
    [F, 2n_1-1, ..., 2n_d-1] like ``visibilities``.
    """
    x = np.asarray(x)
    T, F, N = x.shape
    dims = tuple(int(n) for n in dims)
    if math.prod(dims) != N:
        raise ValueError(f"prod(dims)={math.prod(dims)} != N={N}")
    if not 0 < n_outer < len(dims):
        raise ValueError("n_outer must leave at least one outer and one inner axis")
    outer, inner = dims[:n_outer], dims[n_outer:]
    P, I = math.prod(outer), math.prod(inner)
    out_o, out_i = lag_shape(outer), lag_shape(inner)
    n_o, n_i = math.prod(out_o), math.prod(out_i)
    # inner histogram key of every (i, i') pair: position of i - i' in the inner lag grid
    ci = _antenna_index_tuples(inner) @ _row_major_strides(out_i)
    ci0 = int(np.sum((np.asarray(inner) - 1) * _row_major_strides(out_i)))
    key = (ci[:, None] - ci[None, :] + ci0).ravel()
    # tile pairs grouped by their outer difference dp (position in the outer lag grid)
    po = _antenna_index_tuples(outer)
    co = po @ _row_major_strides(out_o)
    co0 = int(np.sum((np.asarray(outer) - 1) * _row_major_strides(out_o)))
    dpos = (co[:, None] - co[None, :] + co0).ravel()
    pp, qq = np.divmod(np.arange(P * P), P)
    order = np.argsort(dpos, kind="stable")
    bounds = np.searchsorted(dpos[order], np.arange(n_o + 1))
    V = np.zeros((F, n_o, n_i), dtype=np.complex128)
    for f in range(F):
        X = np.asarray(x[:, f, :], dtype=np.complex128).reshape(T, P, I)
        for g in range(co0, n_o):  # the non-negative half of the outer lags
            sel = order[bounds[g] : bounds[g + 1]]
            if sel.size == 0:
                continue
            A = X[:, pp[sel], :].reshape(-1, I)  # [T * pairs, I]: tile p of every pair, stacked
            B = X[:, qq[sel], :].reshape(-1, I)  # tile q of the same pairs, same order
            S = A.T @ B.conj()  # S[i, i'] = sum over pairs and samples of x_(p,i) conj(x_(q,i'))
            V[f, g] = np.bincount(key, weights=S.real.ravel(), minlength=n_i) + 1j * np.bincount(
                key, weights=S.imag.ravel(), minlength=n_i
            )
        # V[-Delta] = conj V[Delta]: in the row-major centred layout -Delta sits at the mirrored position
        V[f, :co0] = np.conj(V[f, ::-1, ::-1][:co0])
    return V.reshape((F,) + lag_shape(dims))


def visibility_cells(x, dims: Sequence[int], deltas) -> np.ndarray:
    """V_f[Delta] for a list of index differences, one overlap sum each.

    For each Delta the antennas j with j - Delta still on the grid form a box;
    the cell is sum_t sum_j x_j conj(x_{j-Delta}) over that box (the same
    definition as ``visibilities``, evaluated cell by cell).  Cost O(N T F)
    per cell, so it serves as a spot check at full size.  ``deltas`` is
    [K, d]; returns complex128 [F, K].
    """
    x = np.asarray(x)
    T, F, N = x.shape
    dims = tuple(int(n) for n in dims)
    if math.prod(dims) != N:
        raise ValueError("prod(dims) != N")
    xr = x.reshape((T, F) + dims)
    deltas = np.atleast_2d(np.asarray(deltas, dtype=np.int64))
    out = np.zeros((F, deltas.shape[0]), dtype=np.complex128)
    for q, delta in enumerate(deltas):
        sl_j, sl_jm = [slice(None), slice(None)], [slice(None), slice(None)]
        empty = False
        for k, (n, dk) in enumerate(zip(dims, delta)):
            if abs(dk) >= n:
                empty = True
                break
            if dk >= 0:  # j in [dk, n), j - dk in [0, n - dk)
                sl_j.append(slice(dk, n))
                sl_jm.append(slice(0, n - dk))
            else:  # j in [0, n + dk), j - dk in [-dk, n)
                sl_j.append(slice(0, n + dk))
                sl_jm.append(slice(-dk, n))
        if empty:
            continue
        a = np.asarray(xr[tuple(sl_j)], dtype=np.complex128).reshape(T, F, -1)
        b = np.asarray(xr[tuple(sl_jm)], dtype=np.complex128).reshape(T, F, -1)
        out[:, q] = np.einsum("tfa,tfa->f", a, b.conj())
    return out


def fourier_power(x, dims: Sequence[int], kappas, m: Sequence[int] | None = None) -> np.ndarray:
    """Time-summed square modulus of the zero-padded DFT at chosen frequency cells.

    P_f[kappa] = sum_t | sum_j x_{t,f,j} exp(-2 pi i sum_k kappa_k j_k / m_k) |^2

    This is the quantity the fast method squares and integrates before its
    inverse transform (Sec. II.A: FFT, square modulus, inverse FFT; Sec. II.C:
    zero-padded FFT then squaring).  ``m`` are the padded lengths (default
    2 n_k).  By the Wiener-Khinchin identity it also equals
    sum_Delta V[Delta] exp(-2 pi i sum_k kappa_k Delta_k / m_k) for any m_k,
    which is how a visibility hypercube is checked one Fourier cell at a time.
    ``kappas`` is [K, d] (integers or reals); returns float64 [F, K].
    """
    x = np.asarray(x)
    T, F, N = x.shape
    dims = tuple(int(n) for n in dims)
    if m is None:
        m = tuple(2 * n for n in dims)
    idx = _antenna_index_tuples(dims).astype(np.float64)  # [N, d]
    kappas = np.atleast_2d(np.asarray(kappas, dtype=np.float64))
    phase = -2.0 * np.pi * (kappas / np.asarray(m, dtype=np.float64)) @ idx.T  # [K, N]
    E = np.exp(1j * phase)
    out = np.zeros((F, kappas.shape[0]), dtype=np.float64)
    for f in range(F):
        X = np.asarray(x[:, f, :], dtype=np.complex128) @ E.T  # [T, K]
        out[f] = np.sum(X.real**2 + X.imag**2, axis=0)
    return out


def baselines(level_dims: Sequence[Sequence[int]], A) -> np.ndarray:
    """Physical baseline of every index-difference cell.

    A layout is r = sum_levels A_l (i_lx, i_ly), the columns of A_l being the
    level's lattice vectors a (Sec. II.D, Eq. GridEq).  Two antennas whose
    index tuples differ by Delta are separated by b(Delta) = sum_l A_l
    (Delta_lx, Delta_ly) (Sec. II.D: the lattice vectors only label which
    physical separation a hypercube cell is).  Returns float64
    [2n_1-1, ..., 2n_d-1, 2] with axes ordered (level 0 x, level 0 y, ...).
    """
    level_dims = [tuple(int(v) for v in ld) for ld in level_dims]
    A = np.asarray(A, dtype=np.float64).reshape(len(level_dims), 2, 2)
    dims = [n for ld in level_dims for n in ld]
    shape = lag_shape(dims)
    grids = np.meshgrid(*[np.arange(-(n - 1), n) for n in dims], indexing="ij")
    b = np.zeros(shape + (2,), dtype=np.float64)
    for lvl in range(len(level_dims)):
        dx = grids[2 * lvl]
        dy = grids[2 * lvl + 1]
        b[..., 0] += A[lvl, 0, 0] * dx + A[lvl, 0, 1] * dy
        b[..., 1] += A[lvl, 1, 0] * dx + A[lvl, 1, 1] * dy
    return b


# ---------------------------------------------------------------------------
# Sample formats.  Written from the format definitions, independently of the
# HIP decoders: cf32 = interleaved float32 (re, im); ci8 = interleaved int8
# (re, im); ci4 = one byte per sample, re in the high nibble and im in the low
# nibble, both two's complement.
# ---------------------------------------------------------------------------


def decode_cf32(raw, T: int, F: int, N: int) -> np.ndarray:
    a = np.asarray(raw).view(np.float32).reshape(T, F, N, 2).astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]


def decode_ci8(raw, T: int, F: int, N: int) -> np.ndarray:
    a = np.asarray(raw).view(np.int8).reshape(T, F, N, 2).astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]


def _nibble(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.int64)
    return np.where(v >= 8, v - 16, v)


def decode_ci4(raw, T: int, F: int, N: int) -> np.ndarray:
    b = np.asarray(raw).view(np.uint8).reshape(T, F, N)
    re = _nibble(b >> 4)
    im = _nibble(b & 0x0F)
    return re.astype(np.float64) + 1j * im.astype(np.float64)


def decode(raw, dtype: str, T: int, F: int, N: int) -> np.ndarray:
    return {"cf32": decode_cf32, "ci8": decode_ci8, "ci4": decode_ci4}[dtype](raw, T, F, N)
