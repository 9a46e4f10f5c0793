"""Plain float64 oracle of the F-engine ahead of the correlator (test infrastructure only; no product
path may import it).

Appendix A, step 2: the data of each antenna are Fourier transformed in the time domain (and
calibrated as necessary); step 3 then arranges, for each frequency bin, the antennas' values into
the hypercube that the correlator takes.  Readings where the paper gives no detail:

* Raw samples are real (one int8 per antenna and sampling instant), antenna-major:
  raw[n][s], s = 0 .. 2 F T - 1 (each antenna's digitiser stream contiguous).
* Channelisation: consecutive blocks of L = 2F samples, one real DFT per block, no window;
  block t gives bins k = 0 .. F - 1 (the Nyquist bin is dropped):
      X[n, t, k] = sum_{j < 2F} raw[n][2F t + j] exp(-2 pi i j k / (2F)).
* Calibration: one complex gain per antenna and channel, which also carries the requantisation
  scale: Y = g[n, k] X[n, t, k].
* Requantisation: real and imaginary parts rounded to the nearest integer, ties to even, then
  clipped to [-7, 7] (ci4) or [-127, 127] (ci8).
* Corner turn: the codes are written in the correlator's layout [t][k][n] (ci4: one byte, re in the
  high nibble and im in the low nibble, two's complement; ci8: (re, im) int8 pairs).
"""

from __future__ import annotations

import numpy as np

__all__ = ["channelise", "requantise", "pack", "fengine"]

_QMAX = {"ci4": 7, "ci8": 127}


def channelise(raw, F: int) -> np.ndarray:
    """X[n, t, k] of real blocks of 2F samples (k < F), complex128 [N, T, F]."""
    raw = np.asarray(raw)
    N, S = raw.shape
    if S % (2 * F):
        raise ValueError(f"{S} samples per antenna is not a whole number of {2 * F}-sample blocks")
    blocks = raw.reshape(N, S // (2 * F), 2 * F).astype(np.float64)
    return np.fft.rfft(blocks, axis=-1)[..., :F]


def requantise(Y, dtype: str) -> tuple[np.ndarray, np.ndarray]:
    """Integer codes (re, im) of complex values: round half to even, clip to the format's range."""
    q = _QMAX[dtype]
    Y = np.asarray(Y)
    return (np.clip(np.rint(Y.real), -q, q).astype(np.int64), np.clip(np.rint(Y.imag), -q, q).astype(np.int64))


def pack(re, im, dtype: str) -> np.ndarray:
    """Codes [T, F, N] -> the correlator's bytes: ci4 uint8 [T, F, N], ci8 int8 [T, F, N, 2]."""
    if dtype == "ci4":
        return (((np.asarray(re) & 0xF) << 4) | (np.asarray(im) & 0xF)).astype(np.uint8)
    return np.stack([re, im], axis=-1).astype(np.int8)


def fengine(raw, F: int, gains, dtype: str):
    """The whole step: channelise, calibrate, requantise, corner-turn.  Returns (bytes in [T, F, N] layout,
    the calibrated float64 values Y [T, F, N] before rounding)."""
    X = channelise(raw, F)  # [N, T, F]
    Y = X * np.asarray(gains)[:, None, :]
    Y = np.transpose(Y, (1, 2, 0))  # corner turn -> [T, F, N]
    re, im = requantise(Y, dtype)
    return pack(re, im, dtype), Y
