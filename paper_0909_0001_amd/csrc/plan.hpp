// Internal plan structures shared by the host planner and the HIP kernels.
//
// Notation (Sec. II.D of the paper): d axes with n_k antennas each; every axis
// is zero-padded to m_k = 2 n_k; M = prod m_k Fourier cells per channel.
//
// The forward transform of one axis is organised as a "fold + short DFT":
// with a fold modulus r_k dividing m_k and L_k = m_k / r_k, the outputs whose
// frequency is congruent to a residue rho (mod r_k) are
//
//   X[r_k q + rho] = sum_{j<L_k} z_j w_{L_k}^{q j},
//   z_j = sum_{l >= 0, j + l L_k < n_k} x[j + l L_k] w_{m_k}^{rho (j + l L_k)},
//
// where w_m = exp(-2 pi i / m).  This is the zero-padded DFT of Sec. II.A/II.C
// split by residue class (decimation in frequency): r_k = 1 is the plain
// pruned DFT, r_k = 2 the usual "even/odd outputs" split.  A work-group can own
// a subset of the residues of one axis (the split axis); it then computes
// exactly the Fourier cells of those residues for every time sample, and
// accumulates their square moduli on chip.  Residues can be divided along
// several axes; the split index c of a work-group is mixed-radix over them.
#pragma once
#include <stdint.h>

namespace omni {

constexpr int kMaxD = 8;
constexpr int kMaxL = 32;  // longest per-thread short DFT

struct AxisP {
  int32_t n;         // antennas along this axis
  int32_t m;         // padded length 2n
  int32_t r;         // fold modulus (divides m)
  int32_t L;         // m / r, the short-DFT length
  int32_t R;         // residues of this axis held by one work-group
  int32_t rho_step;  // residue of the i-th held class = rho0 + i * rho_step
  int32_t split;     // work-groups sharing this axis' residues (rho0 = (c / split_div) % split)
  int32_t split_div; // mixed-radix divisor of this axis' digit in the work-group split index c
  int32_t E;         // extent of this axis inside the work-group after its transform: R * L
  int32_t w_stride;  // stride (complex elements) in the LDS working array
  int32_t p_stride;  // stride (cells) in the LDS power array
  int32_t in_stride; // stride (samples) in one (t, channel) input tile
  int32_t tw_off;    // offset of the w_m^q table (q in [0, m)) in the twiddle array
};

struct PassP {
  int32_t axis;                 // axis transformed by this pass
  int32_t n_other;              // number of other axes
  int32_t ext[kMaxD];           // extents of the other axes at this pass, fastest first
  int32_t w_str[kMaxD];         // their strides in the working array (source and target)
  int32_t src_str[kMaxD];       // their strides in the source (input tile for pass 0)
  int32_t p_str[kMaxD];         // their strides in the power array (last pass)
  int32_t lines;                // product of ext
  int32_t jobs;                 // lines * R of the transformed axis
};

struct FusedP {
  int32_t d;
  int32_t F;             // channels in the source layout
  int32_t N;             // samples per (t, channel) tile
  int32_t n_split;       // work-groups per channel (product of the axes' split factors)
  int32_t n_slices;      // time slices (work-groups per channel along time)
  int32_t cells_wg;      // Fourier cells owned by one work-group
  int32_t w_elems;       // complex elements of the LDS working array
  int32_t n_tw;          // complex twiddles in the table
  int32_t time_block;    // samples summed in float32 before the float64 add
  int32_t xcd_groups;    // 1: XCD-aware block mapping is valid
  AxisP ax[kMaxD];
  PassP pass[kMaxD];     // processing order; pass[0] loads and folds, pass[d-1] squares
};

}  // namespace omni
