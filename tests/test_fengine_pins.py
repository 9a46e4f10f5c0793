"""Pins of the F-engine oracle (oracle/fengine.py, Appendix A step 2): brute-force DFT, closed
forms (tone, impulse, constant), rounding and clipping by hand, the sample-format round trip and
the corner-turned layout."""

from __future__ import annotations

import cmath
import math

import numpy as np
import pytest

import oracle
from oracle import fengine as fe


def test_channelise_brute_force():
    rng = np.random.default_rng(1)
    N, F, T = 3, 4, 2
    raw = rng.integers(-128, 128, (N, 2 * F * T))
    X = fe.channelise(raw, F)
    assert X.shape == (N, T, F)
    for n in range(N):
        for t in range(T):
            for k in range(F):
                ref = sum(int(raw[n, 2 * F * t + j]) * cmath.exp(-2j * math.pi * j * k / (2 * F)) for j in range(2 * F))
                assert abs(X[n, t, k] - ref) < 1e-9


def test_channelise_closed_forms():
    F = 16
    j = np.arange(2 * F)
    # a cosine at bin k0 puts A F at k0 and nothing elsewhere
    for k0 in (1, 5, F - 1):
        X = fe.channelise((3.0 * np.cos(2 * np.pi * k0 * j / (2 * F)))[None], F)[0, 0]
        ref = np.zeros(F, complex)
        ref[k0] = 3.0 * F
        assert np.allclose(X, ref, atol=1e-9)
    # an impulse at j0: X_k = exp(-2 pi i j0 k / 2F) (the forward sign)
    j0 = 3
    imp = np.zeros(2 * F)
    imp[j0] = 1.0
    X = fe.channelise(imp[None], F)[0, 0]
    assert np.allclose(X, np.exp(-2j * np.pi * j0 * np.arange(F) / (2 * F)), atol=1e-12)
    # a constant c: 2F c in bin 0 only
    X = fe.channelise(np.full((1, 4 * F), 5.0), F)[0]
    assert np.allclose(X[:, 0], 2 * F * 5.0) and np.allclose(X[:, 1:], 0.0, atol=1e-9)
    with pytest.raises(ValueError):
        fe.channelise(np.zeros((1, 3 * F)), F)


def test_requantise_by_hand():
    re, im = fe.requantise(np.array([2.5 + 3.5j, -2.5 - 0.5j, 7.6 - 9.0j, 0.49 + 6.5j]), "ci4")
    assert list(re) == [2, -2, 7, 0] and list(im) == [4, 0, -7, 6]
    re, im = fe.requantise(np.array([127.4 - 200.0j, -127.5 + 126.5j]), "ci8")
    assert list(re) == [127, -127] and list(im) == [-127, 126]


def test_pack_hand_bytes_and_round_trip():
    b = fe.pack(np.array([-1, -7, 7, 0]), np.array([7, 1, -7, -1]), "ci4")
    assert list(b) == [0xF7, 0x91, 0x79, 0x0F]
    rng = np.random.default_rng(2)
    re, im = rng.integers(-7, 8, (2, 3, 5)), rng.integers(-7, 8, (2, 3, 5))
    assert np.array_equal(oracle.decode_ci4(fe.pack(re, im, "ci4"), 2, 3, 5), re + 1j * im)
    re8, im8 = rng.integers(-127, 128, (2, 3, 5)), rng.integers(-127, 128, (2, 3, 5))
    assert np.array_equal(oracle.decode_ci8(fe.pack(re8, im8, "ci8"), 2, 3, 5), re8 + 1j * im8)


@pytest.mark.parametrize("dtype", ["ci4", "ci8"])
def test_fengine_layout_brute_force(dtype):
    """Element (t, k, n) of the output is the requantised g[n, k] X[n, t, k] (explicit loops)."""
    rng = np.random.default_rng(3)
    N, F, T = 5, 8, 3
    raw = rng.integers(-40, 41, (N, 2 * F * T))
    g = (rng.normal(size=(N, F)) + 1j * rng.normal(size=(N, F))) * (0.05 if dtype == "ci4" else 0.5)
    out, Y = fe.fengine(raw, F, g, dtype)
    q = 7 if dtype == "ci4" else 127
    dec = oracle.decode(out, dtype, T, F, N)
    for t in range(T):
        for k in range(F):
            for n in range(N):
                x = sum(int(raw[n, 2 * F * t + j]) * cmath.exp(-2j * math.pi * j * k / (2 * F)) for j in range(2 * F))
                y = g[n, k] * x
                assert abs(Y[t, k, n] - y) < 1e-9 * (1 + abs(y))
                want = complex(min(q, max(-q, round(y.real))), min(q, max(-q, round(y.imag))))
                assert dec[t, k, n] == want
