"""CPU oracle for the hierarchical-grid correlator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, tables or helpers) and imports nothing from it.

Everything here is a plain, slow, float64 transcription of what the paper
defines, written so it can be checked against the paper by eye:

* ``visibilities``      -- the visibility hypercube G, i.e. the correlation of
  every antenna pair summed over pairs sharing the same index difference
  (Sec. II.A; Sec. II.C Eq. ConvolutionDefEq; Sec. II.D Eq. ProofEq2).
* ``visibilities_by_outer_lag`` -- the same hypercube with the pair sum
  grouped by the outer levels' index difference (large grids).
* ``visibility_cells``  -- the same quantity for a list of individual index
  differences, one overlap sum per cell (for spot checks at full size).
* ``fourier_power``     -- the time-summed square modulus of the padded
  Fourier transform at chosen frequency cells (Sec. II.A: FFT, square
  modulus, inverse FFT); by Wiener-Khinchin it equals the DFT of G.
* ``baselines``         -- the physical separation of each index-difference
  cell, sum_k Delta_k a_k (Sec. II.D Eq. GridEq).
* ``decode_*``          -- the voltage sample formats (independent decoders).
* ``layout``            -- the physical-baseline fold of the hypercube and the
  baseline-distribution experiment of Sec. III (d = l * l^- from antenna
  positions, zeroed origin, asinh map, radial bins, boxcar smoothing).
* ``beams``             -- the beam-space variant: unpadded 2-D transform of
  every lowest-level block ("digital pointings"), then each pointing
  correlated over the other levels (Appendix A, steps 4-5).
* ``hybrid``            -- hybrid tiles: every ordered pair of arbitrarily
  translated rectangular tiles cross-correlated over index differences
  (Sec. III, the hybrid-tile paragraph).
* ``fengine``           -- the per-antenna time-domain Fourier transform,
  calibration, requantisation and corner turn ahead of the correlator
  (Appendix A, steps 2-3).

Every function is pinned by tests in ``tests/test_oracle_pins.py`` against
values printed in the paper, closed forms, library routines and brute force.
"""

from .correlator import (  # noqa: F401
    baselines,
    decode,
    decode_cf32,
    decode_ci4,
    decode_ci8,
    fourier_power,
    lag_shape,
    visibilities,
    visibilities_by_outer_lag,
    visibility_cells,
)
from . import beams, fengine, hybrid  # noqa: F401
from .layout import (  # noqa: F401
    asinh_map,
    baseline_distribution,
    boxcar,
    fold,
    image_centre,
    layout_positions,
    radial_profile,
    zero_origin,
)
