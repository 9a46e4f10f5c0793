// Fused mixed-precision correlator for single-level square grids of 128 x 128
// antennas (both axes padded to m = 256, 65536 cells per channel), gfx950.
//
// Each axis' zero-padded 256-point DFT (Sec. II.A/II.C) is split Cooley-Tukey
// style, m = P Q, input j = j_l + P j_h (only j_h < Q/2 carries antennas: the
// padding prunes the first stage), output kappa = Q kappa_a + kappa_b:
//   stage 1   y[kappa_b][j_l] = sum_{j_h < Q/2} w_Q^{kappa_b j_h} x[j_l + P j_h]
//   stage 2   X[Q kappa_a + kappa_b] = sum_{j_l < P} w_m^{(Q kappa_a + kappa_b) j_l} y[kappa_b][j_l]
// (the twiddle w_m^{kappa_b j_l} is folded into the stage-2 matrix, one matrix
// per kappa_b).  Every stage is a real-embedded complex matrix product on the
// matrix cores (float16 operands, float32 accumulation):
//   [Re y ; Im y] = [[Re W, -Im W], [Im W, Re W]] [Re x ; Im x],
// with W split into float16 hi + lo parts (hi = rn(W), lo = rn(W - hi)) and
// scaled by 1 / (number of inputs) (exact powers of two that keep every
// float16 intermediate within the input's range; `out_scale` undoes them on
// |X|^2).
//
// Axis 1 (the contiguous one) runs first with P = 8, Q = 32; the two
// work-groups of a channel split its first stage's outputs (work-group s owns
// kappa_b1 in [16 s, 16 s + 16)), so each owns the 32768 cells with those
// kappa_b1, without repeating any product.  Axis 0 runs second with
// P = Q = 16.  A work-group = (time slice, channel, s), 1024 threads (16
// waves), 32 float32 accumulators per lane for the whole slice.  Per sample:
//   D   decode the 16 KiB 4-bit tile into float16 planes in LDS (Lx)
//   P0  axis-1 stage 1, data x W^T on v_mfma_f32_32x32x16_f16        Lx -> L1
//   P1  axis-1 stage 2, data x W^T on v_mfma_f32_16x16x32_f16 (hi and lo
//       stacked along K; one kappa_b1 per wave)                      L1 -> L2
//   P2  axis-0 stage 1, data x W^T, 32x32x16, in 4 chunks of 32 kappa_1 lines
//                                                                    L2 -> L3
//   P3  axis-0 stage 2, W x data, 32x32x16 (one kappa_b0 per wave), so that
//       the real and imaginary rows of an output land in one lane: |X|^2.
// In P0-P2 the rows of a tile are lines ordered with the next pass' contracted
// index fastest, so each lane stores 4 consecutive values with one 8-byte LDS
// write and the next pass reads 8 values with one 16-byte read.  Every layout
// is XOR-swizzled so that each 8-byte store (16 lanes, 32 banks) and each
// 16-byte load (16 lanes, 64 banks) meets every bank once; where the swizzle
// reorders the 8 values of a read, the order depends on the wave or the
// lane half only, and that lane's matrix fragment uses the same order.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace omni {

namespace g2c {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx16 mfma32(half8 a, half8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma16(half8 a, half8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Real-embedded DFT coefficient of input component im_in in output component im_out.
__device__ __forceinline__ float embed(float2 w, int im_out, int im_in) {
  return !im_out ? (!im_in ? w.x : -w.y) : (!im_in ? w.y : w.x);
}
__device__ __forceinline__ void split16(float v, _Float16& hi, _Float16& lo) {
  hi = (_Float16)v;
  lo = (_Float16)(v - (float)hi);
}

__device__ __forceinline__ half4 to_half4(float a, float b, float c, float d) {
  half4 v;
  v[0] = (_Float16)a;
  v[1] = (_Float16)b;
  v[2] = (_Float16)c;
  v[3] = (_Float16)d;
  return v;
}

}  // namespace g2c

namespace g2m {

constexpr int NT = 1024;
constexpr int SLOTS = 32;  // accumulators per lane
constexpr int CELLS = SLOTS * NT;

// LDS layouts, in halves.  R2 holds Lx then L2, R1 holds L1 then the two L3 chunk buffers.
//   Lx [comp][j_l1 8][i0 128][j_h1 16]: two 16-byte chunks per row, chunk (j_h1 / 8) ^ (i0 & 1); i0's low
//      three bits XOR j_l1
__device__ __forceinline__ int lx_at(int comp, int jl, int i0, int jh) {
  const int i0x = (i0 & ~7) | ((i0 ^ jl) & 7);
  return ((comp * 8 + jl) * 128 + i0x) * 16 + (((jh >> 3) ^ (i0 & 1)) << 3) + (jh & 7);
}
//   L1 [comp][kappa_b1 16][pos(i0) ^ (kappa_b1 & 7)][j_l1 8], pos(i0) = i0 / 16 + 8 (i0 % 16); the two
//      4-value units of a row swapped for kappa_b1 >= 8
__device__ __forceinline__ int l1_row(int comp, int kb, int i0) {
  const int pos = (i0 >> 4) | ((i0 & 15) << 3);
  return ((comp * 16 + kb) * 128 + (pos ^ (kb & 7))) * 8;
}
//   L2 [comp][lambda 128][j_l0 ^ kappa_a1][j_h0 8], lambda = 16 kappa_a1 + (kappa_b1 - 16 s); units swapped
//      for comp 1
__device__ __forceinline__ int l2_row(int comp, int lam, int jl0) {
  return ((comp * 128 + lam) * 16 + (jl0 ^ (lam >> 4))) * 8;
}
//   L3 [comp][kappa_b0 16][j_l0 / 8][kappa_1 local 32 ^ (kappa_b0 & 7)][8]; units swapped for kappa_b0 >= 8
__device__ __forceinline__ int l3_row(int comp, int kb0, int chunk, int k1l) {
  return (((comp * 16 + kb0) * 2 + chunk) * 32 + (k1l ^ (kb0 & 7))) * 8;
}

}  // namespace g2m

// Grid: n_slices * F * 2 work-groups, 1024 threads.  src: [T][F][16384] 4-bit samples (re high nibble);
// tw: w_256^q, q < 256 (float32); partial: [n_slices][F][2][32768] float64, cell order of grid128_cell.
__global__ __launch_bounds__(1024) void grid128_mixed_kernel(const uint8_t* __restrict__ src, int64_t T,
                                                            int64_t t_per_slice, const float2* __restrict__ tw,
                                                            double* __restrict__ partial, int F, int n_slices,
                                                            int time_block, double out_scale, int aligned16) {
  using namespace g2c;
  using namespace g2m;
  __shared__ __attribute__((aligned(16))) _Float16 R1[32768];
  __shared__ __attribute__((aligned(16))) _Float16 R2[32768];
  // the P0 and P2 fragments depend on the lane only (the same in every wave): one copy in LDS, entry j of
  // lane l at j * 64 + l (16 lanes read 16 consecutive 16-byte slots)
  __shared__ half8 WF[6 * 64];
  // the P1 fragment of wave w at WF1[w * 64 + l]
  __shared__ half8 WF1[16 * 64];
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
  const int h = l >> 5, n32 = l & 31, n16 = l & 15, g16 = l >> 4;
  // work-group -> (slice, channel, s); with a multiple of 8 (slice, channel) groups the two halves of a
  // channel land on one XCD (blocks b and b + 8 share an XCD), so its input tile is read once from HBM
  int s, q;
  const int nq = n_slices * F;
  if ((nq & 7) == 0) {
    const int b = blockIdx.x;
    s = (b >> 3) & 1;
    q = (b >> 4) * 8 + (b & 7);
  } else {
    s = blockIdx.x & 1;
    q = blockIdx.x >> 1;
  }
  const int ch = q % F, sl = q / F;
  const int64_t t0 = (int64_t)sl * t_per_slice;
  const int64_t t1 = min(T, t0 + t_per_slice);

  // ---- matrix fragments (fixed for the whole kernel) ----
  // P0: B = W1^T, W1[kappa_b1][j_h1] = w_32^{kappa_b1 j_h1} / 16, kappa_b1 = 16 s + (col & 15), output
  // component col / 16; K step ks, lane half h = input component, entry i = j_h1 8 ks + i.
  // (held in WF: entries 0-1 hi, 2-3 lo by K step)
  // P1: B = W2^T (K = [hi comp 0 | hi comp 1 | lo comp 0 | lo comp 1] over the 8 j_l1), kappa_b1 = 16 s + w,
  // column n16 = (kappa_a1 = n16 & 7, output component n16 >> 3); entry i = j_l1 i ^ (4 (w >> 3)) (L1's units
  // are swapped for kappa_b1 local >= 8).  W2[kappa_a1][j_l1] = w_256^{(32 kappa_a1 + kappa_b1) j_l1} / 8.
  // (held in WF1)
  // P2: B = W1'^T, W1'[kappa_b0][j_h0] = w_16^{kappa_b0 j_h0} / 8, column n32 = (kappa_b0 = n32 & 15, output
  // component n32 >> 4); lane half h = input component, entry i = j_h0 i ^ 4h (L2's units swapped for comp 1).
  // (held in WF: entry 4 hi, 5 lo)
  // P3: A = W2'(kappa_b0 = w), W2'[kappa_a0][j_l0] = w_256^{(16 kappa_a0 + w) j_l0} / 16, row n32 =
  // (kappa_a0 = n32 & 15, output component n32 >> 4); K step ks, lane half h = input component, entry i =
  // j_l0 8 ks + (i ^ 4 (w >> 3)).
  half8 w3h[2], w3l[2];
  if (w == 0) {
    const int kb1 = 16 * s + (n32 & 15), co = n32 >> 4;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      half8 fh, fl;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int jh = 8 * ks + i;
        _Float16 hi, lo;
        split16(embed(tw[(8 * kb1 * jh) & 255], co, h) * 0.0625f, hi, lo);
        fh[i] = hi;
        fl[i] = lo;
      }
      WF[ks * 64 + l] = fh;
      WF[(2 + ks) * 64 + l] = fl;
    }
    const int kb0 = n32 & 15;
    half8 fh, fl;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int jh0 = i ^ (4 * h);
      _Float16 hi, lo;
      split16(embed(tw[(16 * kb0 * jh0) & 255], co, h) * 0.125f, hi, lo);
      fh[i] = hi;
      fl[i] = lo;
    }
    WF[4 * 64 + l] = fh;
    WF[5 * 64 + l] = fl;
  }
  {
    const int kb1w = 16 * s + w, ka1 = n16 & 7, co1 = n16 >> 3, ci1 = g16 & 1, lo1 = g16 >> 1;
    half8 f1;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int jl = i ^ (4 * (w >> 3));
      _Float16 hi, lo;
      split16(embed(tw[((32 * ka1 + kb1w) * jl) & 255], co1, ci1) * 0.125f, hi, lo);
      f1[i] = lo1 ? lo : hi;
    }
    WF1[w * 64 + l] = f1;
    const int co = n32 >> 4;
    const int ka0 = n32 & 15;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int jl0 = 8 * ks + (i ^ (4 * (w >> 3)));
        _Float16 hi, lo;
        split16(embed(tw[((16 * ka0 + w) * jl0) & 255], co, h) * 0.0625f, hi, lo);
        w3h[ks][i] = hi;
        w3l[ks][i] = lo;
      }
  }

  // ---- D: thread tid decodes 16 bytes: i0 = tid / 8, i1 in [16 u, 16 u + 16) (u = tid % 8), i.e. j_h1 in
  // {2u, 2u + 1} and all 8 j_l1.  A 4-bit value v becomes the float16 1024 + (v + 8) by placing the biased
  // nibble under the exponent byte 0x64; subtracting 1032 is exact.
  // ---- LDS addresses.  Every access of a pass is a per-lane base combined with a compile-time constant (an
  // XOR on bits the base leaves clear, or an add above them), worked out from the layouts above:
  //   P0 read   lx_at(h, j_l1, i0, 8 ks), i0 = 8w + 4k + g'      = a0 ^ (64 k + 8 ks)
  //   P0 store  l1_row(c, kb, 8w + 4k + g) + 4 (h ^ kb / 8)     = s0 + 256 k + 64 g
  //   P1 read   l1_row(g16 & 1, w, i0(tile, n16))               = a1 + 128 tile
  //   P1 store  l2_row(c, 16 ka + w, 2 tile + g16 / 2) + unit   = s1 ^ 16 tile
  //   P2 read   l2_row(h, 32 c + 2w + n32 / 16, n32 & 15)       = (a2 ^ 16 c) + 4096 c
  //   P2 store  l3_row(c, kb0, g & 1, 2w + g / 2) + unit        = (s2 ^ 8 (g / 2)) + 256 (g & 1) (+ 16384 buffer)
  //   P3 read   l3_row(h, w, ks, n32)                           = a3 + 256 ks (+ 16384 buffer)
  //   D  store  lx_at(comp, j_l1, i0, 2u)                       = (sd ^ 16 j_l1) + 2048 j_l1 + 16384 comp
  // The bases are made opaque by an empty asm at the start of each pass, so that the compiler forms the
  // pass' addresses there (one XOR or none each) instead of holding all of them across the time loop.
  const int gq = n32 >> 3, jl_ = n32 & 7;
  int a0 = (((h * 8 + jl_) * 128 + 8 * w) * 16) + (gq ^ jl_) * 16 + (gq & 1) * 8;
  int s0;
  {
    const int kb = n32 & 15, co = n32 >> 4;
    s0 = (co * 16 + kb) * 1024 + ((w >> 1) ^ (kb & 7)) * 8 + 512 * (w & 1) + 4 * (h ^ (kb >> 3));
  }
  int a1 = ((((g16 & 1) * 16 + w) * 128 + ((4 * ((n16 >> 2) & 1) + (n16 & 3)) ^ (w & 7)) + 8 * (n16 >> 3)) * 8);
  int s1;
  {
    const int ka = n16 & 7, co = n16 >> 3, gb = g16 >> 1, u = (g16 & 1) ^ co;
    s1 = (co * 128 + 16 * ka + w) * 128 + 16 * (ka >> 1) + 8 * (gb ^ (ka & 1)) + 4 * u;
  }
  int a2 = (h * 128 + 2 * w + (n32 >> 4)) * 128 + (((n32 & 15) ^ (w >> 3)) * 8);
  int s2;
  {
    const int kb0 = n32 & 15, co = n32 >> 4;
    s2 = (co * 16 + kb0) * 512 + ((2 * w) ^ (kb0 & 6)) * 8 + 8 * (kb0 & 1) + 4 * (h ^ (kb0 >> 3));
  }
  int a3 = (((h * 16 + w) * 2) * 32 + (n32 ^ (w & 7))) * 8;
  int sd;
  {
    const int i0 = tid >> 3, u = tid & 7;
    sd = ((i0 & ~7) + 0) * 16 + (i0 & 7) * 16 + (((u >> 2) ^ (i0 & 1)) << 3) + ((2 * u) & 7);
  }
  auto opaque = [](int& v) { asm volatile("" : "+v"(v)); };

  // ---- D: thread tid decodes 16 bytes: i0 = tid / 8, i1 in [16 u, 16 u + 16) (u = tid % 8), i.e. j_h1 in
  // {2u, 2u + 1} and all 8 j_l1.  A 4-bit value v becomes the float16 1024 + (v + 8) by placing the biased
  // nibble under the exponent byte 0x64; subtracting 1032 is exact.
  uint4 raw;
  // (a 4-byte aligned source takes four 4-byte loads)
  auto load_raw = [&](int64_t t) {
    const uint8_t* p = src + (t * F + ch) * 16384 + tid * 16;
    if (aligned16) {
      raw = *reinterpret_cast<const uint4*>(p);
    } else {
      const uint32_t* p4 = reinterpret_cast<const uint32_t*>(p);
      raw = make_uint4(p4[0], p4[1], p4[2], p4[3]);
    }
  };
  auto decode = [&]() {
    opaque(sd);
    const uint32_t b[4] = {raw.x ^ 0x88888888u, raw.y ^ 0x88888888u, raw.z ^ 0x88888888u, raw.w ^ 0x88888888u};
    const _Float16 bias = (_Float16)1032.f;
    const half2v bb = {bias, bias};
#pragma unroll
    for (int jl = 0; jl < 8; ++jl) {
      // bytes jl (j_h1 = 2u) and jl + 8 (j_h1 = 2u + 1)
      const uint32_t lo_w = b[jl >> 2], hi_w = b[(jl >> 2) + 2];
      const uint32_t sel = (uint32_t)(jl & 3) | ((uint32_t)(4 + (jl & 3)) << 16) | 0x0c000c00u;
      const uint32_t pair = __builtin_amdgcn_perm(hi_w, lo_w, sel);  // [byte(lo_w), 0, byte(hi_w), 0]
      const uint32_t re = ((pair >> 4) & 0x000f000fu) | 0x64006400u, im = (pair & 0x000f000fu) | 0x64006400u;
      const half2v vr = __builtin_bit_cast(half2v, re) - bb, vi = __builtin_bit_cast(half2v, im) - bb;
      const int at = (sd ^ (16 * jl)) + 2048 * jl;
      *reinterpret_cast<half2v*>(&R2[at]) = vr;
      *reinterpret_cast<half2v*>(&R2[at + 16384]) = vi;
    }
  };

  // ---- P0: tile tt of wave w (tiles 2w, 2w + 1): rows r = 8g + 4h' + e <-> (j_l1 = r & 7, i0 = 4 tile + r / 8)
  auto pass0 = [&]() {
    opaque(a0);
    opaque(s0);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      floatx16 d = {};
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const half8 x = *reinterpret_cast<const half8*>(&R2[a0 ^ (64 * k + 8 * ks)]);
        d = mfma32(x, WF[ks * 64 + l], d);
        d = mfma32(x, WF[(2 + ks) * 64 + l], d);
      }
      // column n32 = (kappa_b1 local = n32 & 15, comp n32 >> 4); rows 8g + 4h + e: j_l1 = 4h + e, i0 = 4 tile + g
#pragma unroll
      for (int g = 0; g < 4; ++g)
        *reinterpret_cast<half4*>(&R1[s0 + 256 * k + 64 * g]) =
            to_half4(d[4 * g], d[4 * g + 1], d[4 * g + 2], d[4 * g + 3]);
    }
  };

  // ---- P1: wave w, kappa_b1 local = w; 8 tiles of 16 lines: row rho <-> i0 = j_l0 + 16 j_h0 with
  // j_h0 = 4 ((rho / 4) & 1) + rho % 4, j_l0 = 2 tile + rho / 8
  auto pass1 = [&]() {
    opaque(a1);
    opaque(s1);
    const half8 w1 = WF1[w * 64 + l];
#pragma unroll 2
    for (int tile = 0; tile < 8; ++tile) {
      const half8 x = *reinterpret_cast<const half8*>(&R1[a1 + 128 * tile]);
      floatx4 d = {};
      d = mfma16(x, w1, d);
      // column n16 = (kappa_a1 = n16 & 7, comp n16 >> 3); rows 4 g16 + i: j_h0 = 4 (g16 & 1) + i,
      // j_l0 = 2 tile + g16 / 2
      *reinterpret_cast<half4*>(&R2[s1 ^ (16 * tile)]) = to_half4(d[0], d[1], d[2], d[3]);
    }
  };

  // ---- P2 of chunk c (lambda in [32 c, 32 c + 32)): tile of wave w = lambda pair 32 c + 2w, +1; rows
  // r = 8g + 4h + e <-> (j_l0 = r & 15, lambda = 32 c + 2w + r / 16) -> L3 buffer c & 1
  auto pass2 = [&](int c) {
    opaque(a2);
    opaque(s2);
    _Float16* L3 = R1 + (c & 1) * 16384;
    const half8 x = *reinterpret_cast<const half8*>(&R2[(a2 ^ (16 * c)) + 4096 * c]);
    floatx16 d = {};
    d = mfma32(x, WF[4 * 64 + l], d);
    d = mfma32(x, WF[5 * 64 + l], d);
    // column n32 = (kappa_b0 = n32 & 15, comp n32 >> 4); rows 8g + 4h + e: j_l0 = 8 (g & 1) + 4h + e,
    // kappa_1 local = 2w + g / 2
#pragma unroll
    for (int g = 0; g < 4; ++g)
      *reinterpret_cast<half4*>(&L3[(s2 ^ (8 * (g >> 1))) + 256 * (g & 1)]) =
          to_half4(d[4 * g], d[4 * g + 1], d[4 * g + 2], d[4 * g + 3]);
  };

  float acc[SLOTS];
#pragma unroll
  for (int i = 0; i < SLOTS; ++i) acc[i] = 0.f;

  // ---- P3 of chunk c: kappa_b0 = w, columns kappa_1 local n32; rows 8g + 4h + e (g < 2) hold Re and rows
  // 16 + 8g + 4h + e Im of kappa_a0 = 8g + 4h + e
  auto pass3 = [&](int c) {
    opaque(a3);
    const _Float16* L3 = R1 + (c & 1) * 16384;
    floatx16 d = {};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const half8 x = *reinterpret_cast<const half8*>(&L3[a3 + 256 * ks]);
      d = mfma32(w3h[ks], x, d);
      d = mfma32(w3l[ks], x, d);
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      float& a = acc[8 * c + r];
      a = fmaf(d[r], d[r], fmaf(d[r + 8], d[r + 8], a));
    }
  };

  double* out = partial + (((int64_t)sl * F + ch) * 2 + s) * (int64_t)CELLS;
  bool flushed = false;
  auto flush = [&]() {
    double* o = out + tid;
    asm volatile("" : "+v"(o));
    if (flushed) {
#pragma unroll
      for (int i0 = 0; i0 < SLOTS; i0 += 8) {
        double prev[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) prev[k] = o[(i0 + k) * NT];
#pragma unroll
        for (int k = 0; k < 8; ++k) o[(i0 + k) * NT] = prev[k] + (double)acc[i0 + k] * out_scale;
      }
    } else {
#pragma unroll
      for (int i = 0; i < SLOTS; ++i) o[i * NT] = (double)acc[i] * out_scale;
    }
#pragma unroll
    for (int i = 0; i < SLOTS; ++i) acc[i] = 0.f;
    flushed = true;
  };

  // Per sample t (barriers marked |):  D(t) | P0 | P1 | P2(0) | P2(1) P3(0) | P2(2) P3(1) | P2(3) P3(2) |
  // P3(3) D(t + 1) | P0(t + 1) ...  Lx and L2 share R2 (D(t + 1) follows P2(3) of t), L1 and the L3
  // buffers share R1 (P0(t + 1) follows P3(3) of t).  The next sample's bytes are loaded one sample ahead.
  if (t0 < t1) {
    load_raw(t0);
    decode();
    load_raw(min(t0 + 1, t1 - 1));
  }
  int blk = 0;
  for (int64_t t = t0; t < t1; ++t) {
    __syncthreads();
    pass0();
    __syncthreads();
    pass1();
    __syncthreads();
    pass2(0);
    __syncthreads();
    // (the scheduling barriers keep one pass' tile registers from overlapping the next pass')
    pass2(1);
    __builtin_amdgcn_sched_barrier(0);
    pass3(0);
    __syncthreads();
    pass2(2);
    __builtin_amdgcn_sched_barrier(0);
    pass3(1);
    __syncthreads();
    pass2(3);
    __builtin_amdgcn_sched_barrier(0);
    pass3(2);
    __syncthreads();
    pass3(3);
    __builtin_amdgcn_sched_barrier(0);
    if (t + 1 < t1) {
      decode();
      load_raw(min(t + 2, t1 - 1));
    }
    if (++blk == time_block) {
      blk = 0;
      flush();
    }
  }
  if (blk > 0 || !flushed) flush();
}

// Natural index kappa_0 * 256 + kappa_1 of cell `cell` (= slot * 1024 + thread) of work-group half s.
int grid128_cell(int s, int cell) {
  const int slot = cell / 1024, tid = cell % 1024;
  const int w = tid >> 6, l = tid & 63, h = l >> 5, n32 = l & 31;
  const int c = slot / 8, r = slot % 8, g = r / 4, e = r % 4;
  const int ka0 = 8 * g + 4 * h + e, k0 = 16 * ka0 + w;
  const int lam = 32 * c + n32, ka1 = lam >> 4, kb1 = 16 * s + (lam & 15);
  return k0 * 256 + 32 * ka1 + kb1;
}

hipError_t launch_grid128_mixed(const void* src, int64_t T, int64_t tps, const float2* tw256, double* partial, int F,
                                int n_slices, int time_block, double out_scale, hipStream_t st) {
  if ((reinterpret_cast<uintptr_t>(src) & 3) != 0 || F < 1 || n_slices < 1) return hipErrorInvalidValue;
  const int aligned16 = (reinterpret_cast<uintptr_t>(src) & 15) == 0;
  hipLaunchKernelGGL(grid128_mixed_kernel, dim3((unsigned)(n_slices * F * 2)), dim3(g2m::NT), 0, st,
                     static_cast<const uint8_t*>(src), T, tps, tw256, partial, F, n_slices, time_block, out_scale,
                     aligned16);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 64 x 64 antennas (m = 128, 16384 cells per channel): both axes P = 8, Q = 16
// (8 inputs per first-stage line, 8 per second-stage line), so every stage has
// 8 inputs and is scaled by 1/8.  One work-group of 1024 threads owns a whole
// channel (16 accumulators per lane).  Passes as for 128 x 128 without the
// split and with 16 waves <-> 16 kappa_b of each axis:
//   D   256 threads decode the 4 KiB tile into Lx [comp][j_l1][i0 ^ 2 j_l1][j_h1]
//   P0  axis-1 stage 1, 32x32x16, 16 tiles (one per wave)           Lx -> L1
//   P1  axis-1 stage 2, 16x16x32 (hi | lo along K), kappa_b1 = w    L1 -> L2
//   P2  axis-0 stage 1, 32x32x16, 2 tiles per wave                  L2 -> L3
//   P3  axis-0 stage 2, W x data on 16x16x32 (hi | lo along K), kappa_b0 = w,
//       rows 2 kappa_a0 + comp so that an output's two rows share a lane.
namespace g64 {
constexpr int NT = 1024;
constexpr int SLOTS = 16;
constexpr int CELLS = SLOTS * NT;
// Lx [comp][jl 8][i0 ^ 2jl (64)][jh 8]                            (rows of 16 bytes)
__device__ __forceinline__ int lx_row(int comp, int jl, int i0) { return ((comp * 8 + jl) * 64 + (i0 ^ (2 * jl))) * 8; }
// L1 [comp][kb 16][pos(i0) ^ (kb & 7)][jl 8], pos(i0) = i0 / 8 + 8 (i0 % 8); units swapped for kb >= 8
__device__ __forceinline__ int l1_row(int comp, int kb, int i0) {
  const int pos = (i0 >> 3) | ((i0 & 7) << 3);
  return ((comp * 16 + kb) * 64 + (pos ^ (kb & 7))) * 8;
}
// L2 [comp][kappa_1 128][jl0 ^ (kappa_1 / 16)][jh0 8]; units swapped for comp 1
__device__ __forceinline__ int l2_row(int comp, int k1, int jl0) { return ((comp * 128 + k1) * 8 + (jl0 ^ (k1 >> 4))) * 8; }
// L3 [comp][kb0 16][kappa_1 ^ (kb0 & 7)][jl0 8]; units swapped for kb0 >= 8
__device__ __forceinline__ int l3_row(int comp, int kb0, int k1) { return ((comp * 16 + kb0) * 128 + (k1 ^ (kb0 & 7))) * 8; }
}  // namespace g64

// Grid: n_slices * F work-groups.  src: [T][F][4096] 4-bit samples; tw: w_128^q, q < 128; partial:
// [n_slices][F][16384] float64 in the cell order of grid64_cell.
__global__ __launch_bounds__(1024) void grid64_mixed_kernel(const uint8_t* __restrict__ src, int64_t T,
                                                           int64_t t_per_slice, const float2* __restrict__ tw,
                                                           double* __restrict__ partial, int F, int time_block,
                                                           double out_scale, int aligned16) {
  using namespace g2c;
  using namespace g64;
  __shared__ __attribute__((aligned(16))) _Float16 R2[16384];  // Lx (8192 halves), then L2
  __shared__ __attribute__((aligned(16))) _Float16 R1[32768];  // L1 (16384 halves), then L3
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
  const int h = l >> 5, n32 = l & 31, n16 = l & 15, g16 = l >> 4;
  const int ch = blockIdx.x % F, sl = blockIdx.x / F;
  const int64_t t0 = (int64_t)sl * t_per_slice;
  const int64_t t1 = min(T, t0 + t_per_slice);

  // Fragments.  Stage 1 of either axis: W1[kb][jh] = w_16^{kb jh} / 8 = w_128^{8 kb jh} / 8 (column n32 =
  // (kb = n32 & 15, output component n32 >> 4), lane half h = input component); P0 reads jh in natural order,
  // P2 with the units swapped for comp 1.
  half8 f0h, f0l, f2h, f2l;
  // P1 (B, 16x16x32): column n16 = (ka = n16 & 7, output comp n16 >> 3), K chunk g16 = (hi | lo, input comp);
  // W2[ka][jl] = w_128^{(16 ka + w) jl} / 8, entry i = jl i ^ 4 (w >> 3).
  half8 f1;
  // P3 (A, 16x16x32): row n16 = (ka0 = n16 >> 1, output comp n16 & 1), K chunk g16 = (hi | lo, input comp);
  // W2'[ka0][jl0] = w_128^{(16 ka0 + w) jl0} / 8, entry i = jl0 i ^ 4 (w >> 3).
  half8 f3;
  {
    const int kb = n32 & 15, co = n32 >> 4;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      _Float16 hi, lo;
      split16(embed(tw[(8 * kb * i) & 127], co, h) * 0.125f, hi, lo);
      f0h[i] = hi;
      f0l[i] = lo;
      const int jh0 = i ^ (4 * h);
      split16(embed(tw[(8 * kb * jh0) & 127], co, h) * 0.125f, hi, lo);
      f2h[i] = hi;
      f2l[i] = lo;
    }
    const int ci = g16 & 1, lo_part = g16 >> 1;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int j = i ^ (4 * (w >> 3));
      _Float16 hi, lo;
      split16(embed(tw[((16 * (n16 & 7) + w) * j) & 127], n16 >> 3, ci) * 0.125f, hi, lo);
      f1[i] = lo_part ? lo : hi;
      split16(embed(tw[((16 * (n16 >> 1) + w) * j) & 127], n16 & 1, ci) * 0.125f, hi, lo);
      f3[i] = lo_part ? lo : hi;
    }
  }

  auto lane_v = [&]() {
    int v = l;
    asm volatile("" : "+v"(v));
    return v;
  };
  // ---- D: threads 0..255, 16 bytes each: i0 = tid / 4, i1 in [16 u, 16 u + 16) (u = tid % 4) -> j_h1 in
  // {2u, 2u + 1}, all 8 j_l1
  uint4 raw = make_uint4(0u, 0u, 0u, 0u);
  auto load_raw = [&](int64_t t) {
    if (tid < 256) {
      const uint8_t* p = src + (t * F + ch) * 4096 + tid * 16;
      if (aligned16) {
        raw = *reinterpret_cast<const uint4*>(p);
      } else {
        const uint32_t* p4 = reinterpret_cast<const uint32_t*>(p);
        raw = make_uint4(p4[0], p4[1], p4[2], p4[3]);
      }
    }
  };
  auto decode = [&]() {
    if (tid < 256) {
      const int tv = lane_v() + 64 * w, i0 = tv >> 2, u = tv & 3;
      const uint32_t b[4] = {raw.x ^ 0x88888888u, raw.y ^ 0x88888888u, raw.z ^ 0x88888888u, raw.w ^ 0x88888888u};
      const _Float16 bias = (_Float16)1032.f;
      const half2v bb = {bias, bias};
#pragma unroll
      for (int jl = 0; jl < 8; ++jl) {
        const uint32_t sel = (uint32_t)(jl & 3) | ((uint32_t)(4 + (jl & 3)) << 16) | 0x0c000c00u;
        const uint32_t pair = __builtin_amdgcn_perm(b[(jl >> 2) + 2], b[jl >> 2], sel);
        const uint32_t re = ((pair >> 4) & 0x000f000fu) | 0x64006400u, im = (pair & 0x000f000fu) | 0x64006400u;
        *reinterpret_cast<half2v*>(&R2[lx_row(0, jl, i0) + 2 * u]) = __builtin_bit_cast(half2v, re) - bb;
        *reinterpret_cast<half2v*>(&R2[lx_row(1, jl, i0) + 2 * u]) = __builtin_bit_cast(half2v, im) - bb;
      }
    }
  };
  // ---- P0: tile w: rows r = 8g + 4h + e <-> (jl = r & 7, i0 = 4w + r / 8)
  auto pass0 = [&]() {
    const int lv = lane_v(), n32 = lv & 31, h = lv >> 5;
    const half8 x = *reinterpret_cast<const half8*>(&R2[lx_row(h, n32 & 7, 4 * w + (n32 >> 3))]);
    floatx16 d = {};
    d = mfma32(x, f0h, d);
    d = mfma32(x, f0l, d);
    const int kb = n32 & 15, co = n32 >> 4;
#pragma unroll
    for (int g = 0; g < 4; ++g)
      *reinterpret_cast<half4*>(&R1[l1_row(co, kb, 4 * w + g) + 4 * (h ^ (kb >> 3))]) =
          to_half4(d[4 * g], d[4 * g + 1], d[4 * g + 2], d[4 * g + 3]);
  };
  // ---- P1: kb1 = w; 4 tiles of 16 lines: row rho <-> i0 = jl0 + 8 jh0, jh0 = 4 ((rho / 4) & 1) + rho % 4,
  // jl0 = 2 tile + rho / 8
  auto pass1 = [&]() {
    const int lv = lane_v(), n16 = lv & 15, g16 = lv >> 4;
#pragma unroll
    for (int tile = 0; tile < 4; ++tile) {
      const int i0 = (2 * tile + (n16 >> 3)) + 8 * (4 * ((n16 >> 2) & 1) + (n16 & 3));
      const half8 x = *reinterpret_cast<const half8*>(&R1[l1_row(g16 & 1, w, i0)]);
      floatx4 d = {};
      d = mfma16(x, f1, d);
      const int ka = n16 & 7, co = n16 >> 3, k1 = 16 * ka + w, jl0 = 2 * tile + (g16 >> 1);
      *reinterpret_cast<half4*>(&R2[l2_row(co, k1, jl0) + 4 * ((g16 & 1) ^ co)]) = to_half4(d[0], d[1], d[2], d[3]);
    }
  };
  // ---- P2: tiles 2w, 2w + 1: rows r = 8g + 4h + e <-> (jl0 = r & 7, kappa_1 = 4 tile + r / 8)
  auto pass2 = [&]() {
    const int lv = lane_v(), n32 = lv & 31, h = lv >> 5;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int tile = 2 * w + k;
      const half8 x = *reinterpret_cast<const half8*>(&R2[l2_row(h, 4 * tile + (n32 >> 3), n32 & 7)]);
      floatx16 d = {};
      d = mfma32(x, f2h, d);
      d = mfma32(x, f2l, d);
      const int kb0 = n32 & 15, co = n32 >> 4;
#pragma unroll
      for (int g = 0; g < 4; ++g)
        *reinterpret_cast<half4*>(&R1[l3_row(co, kb0, 4 * tile + g) + 4 * (h ^ (kb0 >> 3))]) =
            to_half4(d[4 * g], d[4 * g + 1], d[4 * g + 2], d[4 * g + 3]);
    }
  };
  float acc[SLOTS];
#pragma unroll
  for (int i = 0; i < SLOTS; ++i) acc[i] = 0.f;
  // ---- P3: kb0 = w; 8 tiles of 16 kappa_1 columns; rows 4 g16 + i <-> (ka0 = 2 g16 + i / 2, comp i & 1)
  auto pass3 = [&]() {
    const int lv = lane_v(), n16 = lv & 15, g16 = lv >> 4;
#pragma unroll
    for (int tile = 0; tile < 8; ++tile) {
      const half8 x = *reinterpret_cast<const half8*>(&R1[l3_row(g16 & 1, w, 16 * tile + n16)]);
      floatx4 d = {};
      d = mfma16(f3, x, d);
      acc[2 * tile] = fmaf(d[0], d[0], fmaf(d[1], d[1], acc[2 * tile]));
      acc[2 * tile + 1] = fmaf(d[2], d[2], fmaf(d[3], d[3], acc[2 * tile + 1]));
    }
  };

  double* out = partial + ((int64_t)sl * F + ch) * (int64_t)CELLS;
  bool flushed = false;
  auto flush = [&]() {
    double* o = out + tid;
    asm volatile("" : "+v"(o));
#pragma unroll
    for (int i = 0; i < SLOTS; ++i) {
      const double v = (double)acc[i] * out_scale;
      o[i * NT] = flushed ? o[i * NT] + v : v;
      acc[i] = 0.f;
    }
    flushed = true;
  };

  // Per sample: D(t) | P0 | P1 | P2 | P3 and D(t + 1) | ...  (Lx and L2 share R2, L1 and L3 share R1).
  if (t0 < t1) {
    load_raw(t0);
    decode();
    load_raw(min(t0 + 1, t1 - 1));
  }
  int blk = 0;
  for (int64_t t = t0; t < t1; ++t) {
    __syncthreads();
    pass0();
    __syncthreads();
    pass1();
    __syncthreads();
    pass2();
    __syncthreads();
    pass3();
    __builtin_amdgcn_sched_barrier(0);
    if (t + 1 < t1) {
      decode();
      load_raw(min(t + 2, t1 - 1));
    }
    if (++blk == time_block) {
      blk = 0;
      flush();
    }
  }
  if (blk > 0 || !flushed) flush();
}

// Natural index kappa_0 * 128 + kappa_1 of cell `cell` (= slot * 1024 + thread).
int grid64_cell(int cell) {
  const int slot = cell / 1024, tid = cell % 1024;
  const int w = tid >> 6, l = tid & 63, n16 = l & 15, g16 = l >> 4;
  const int tile = slot / 2, j = slot % 2;
  const int ka0 = 2 * g16 + j, k0 = 16 * ka0 + w, k1 = 16 * tile + n16;
  return k0 * 128 + k1;
}

hipError_t launch_grid64_mixed(const void* src, int64_t T, int64_t tps, const float2* tw128, double* partial, int F,
                               int n_slices, int time_block, double out_scale, hipStream_t st) {
  if ((reinterpret_cast<uintptr_t>(src) & 3) != 0 || F < 1 || n_slices < 1) return hipErrorInvalidValue;
  const int aligned16 = (reinterpret_cast<uintptr_t>(src) & 15) == 0;
  hipLaunchKernelGGL(grid64_mixed_kernel, dim3((unsigned)(n_slices * F)), dim3(g64::NT), 0, st,
                     static_cast<const uint8_t*>(src), T, tps, tw128, partial, F, time_block, out_scale, aligned16);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 32 x 32 antennas (m = 64, 4096 cells per channel): each axis' pruned 64-point
// DFT as one dense real-embedded product (32 complex inputs -> 64 outputs,
// K = 64 in four steps, scaled by 1/32).  A work-group of 256 threads (4 waves)
// owns a channel (16 accumulators per lane); wave w owns outputs
// kappa in [16 w, 16 w + 16) of each axis.  The W fragment of wave w serves as
// the B operand of P0 (data x W^T) and the A operand of P1 (W x data): lane l
// holds row / column l % 32 and input chunk l / 32 in both.
//   D   the 1 KiB tile -> Lx [comp][i0][i1] float16
//   P0  axis 1, data x W^T, rows i0 (one tile), columns (kappa_1, comp)     Lx -> L1
//   P1  axis 0, W x data, columns kappa_1 (two tiles) -> |X|^2.
namespace g32 {
constexpr int NT = 256;
constexpr int SLOTS = 16;
constexpr int CELLS = SLOTS * NT;
// Lx [comp][i0 32][chunk ^ ((i0 / 4) & 3)][8]: rows of four 16-byte chunks of i1
__device__ __forceinline__ int lx_at(int comp, int i0, int chunk) { return (comp * 32 + i0) * 32 + ((chunk ^ ((i0 >> 2) & 3)) << 3); }
// L1 [comp][kappa_1 64][chunk ^ ((kappa_1 / 4) & 3)][8]: rows of four 16-byte chunks of i0
__device__ __forceinline__ int l1_at(int comp, int k1, int chunk) { return (comp * 64 + k1) * 32 + ((chunk ^ ((k1 >> 2) & 3)) << 3); }
}  // namespace g32

// Grid: n_slices * F work-groups of 256 threads.  src: [T][F][1024] 4-bit samples; tw: w_64^q, q < 64;
// partial: [n_slices][F][4096] float64 in the cell order of grid32_cell.
__global__ __launch_bounds__(256) void grid32_mixed_kernel(const uint8_t* __restrict__ src, int64_t T,
                                                          int64_t t_per_slice, const float2* __restrict__ tw,
                                                          double* __restrict__ partial, int F, int time_block,
                                                          double out_scale) {
  using namespace g2c;
  using namespace g32;
  __shared__ __attribute__((aligned(16))) _Float16 Lx[2048];
  __shared__ __attribute__((aligned(16))) _Float16 L1[4096];
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
  const int h = l >> 5, n32 = l & 31;
  const int ch = blockIdx.x % F, sl = blockIdx.x / F;
  const int64_t t0 = (int64_t)sl * t_per_slice;
  const int64_t t1 = min(T, t0 + t_per_slice);

  // W[kappa][j] = w_64^{kappa j} / 32, kappa = 16 w + (n32 & 15), output component n32 >> 4, K step ks,
  // input component h, entry i = j 8 ks + i
  half8 fh[4], fl[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      _Float16 hi, lo;
      split16(embed(tw[((16 * w + (n32 & 15)) * (8 * ks + i)) & 63], n32 >> 4, h) * 0.03125f, hi, lo);
      fh[ks][i] = hi;
      fl[ks][i] = lo;
    }

  auto lane_v = [&]() {
    int v = l;
    asm volatile("" : "+v"(v));
    return v;
  };
  // ---- D: thread tid decodes 4 bytes: i0 = tid / 8, i1 in [4 q, 4 q + 4) (q = tid % 8)
  uint32_t raw = 0;
  auto load_raw = [&](int64_t t) { raw = *reinterpret_cast<const uint32_t*>(src + (t * F + ch) * 1024 + tid * 4); };
  auto decode = [&]() {
    const int tv = lane_v() + 64 * w, i0 = tv >> 3, q = tv & 7;
    const uint32_t b = raw ^ 0x88888888u;
    const _Float16 bias = (_Float16)1032.f;
    const half2v bb = {bias, bias};
    const uint32_t p01 = __builtin_amdgcn_perm(b, b, 0x0c010c00u), p23 = __builtin_amdgcn_perm(b, b, 0x0c030c02u);
    const half2v r01 = __builtin_bit_cast(half2v, ((p01 >> 4) & 0x000f000fu) | 0x64006400u) - bb;
    const half2v r23 = __builtin_bit_cast(half2v, ((p23 >> 4) & 0x000f000fu) | 0x64006400u) - bb;
    const half2v i01 = __builtin_bit_cast(half2v, (p01 & 0x000f000fu) | 0x64006400u) - bb;
    const half2v i23 = __builtin_bit_cast(half2v, (p23 & 0x000f000fu) | 0x64006400u) - bb;
    *reinterpret_cast<half4*>(&Lx[lx_at(0, i0, q >> 1) + 4 * (q & 1)]) = __builtin_shufflevector(r01, r23, 0, 1, 2, 3);
    *reinterpret_cast<half4*>(&Lx[lx_at(1, i0, q >> 1) + 4 * (q & 1)]) = __builtin_shufflevector(i01, i23, 0, 1, 2, 3);
  };
  // ---- P0: rows i0 = n32, columns (kappa_1 = 16 w + c % 16, comp c / 16) -> L1, 4 consecutive i0 per store
  auto pass0 = [&]() {
    const int lv = lane_v(), n32 = lv & 31, h = lv >> 5;
    floatx16 d = {};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const half8 x = *reinterpret_cast<const half8*>(&Lx[lx_at(h, n32, ks)]);
      d = mfma32(x, fh[ks], d);
      d = mfma32(x, fl[ks], d);
    }
    const int k1 = 16 * w + (n32 & 15), co = n32 >> 4;
#pragma unroll
    for (int g = 0; g < 4; ++g)  // rows 8g + 4h + e: i0 = 8g + 4h + e, chunk g, unit h
      *reinterpret_cast<half4*>(&L1[l1_at(co, k1, g) + 4 * h]) =
          to_half4(d[4 * g], d[4 * g + 1], d[4 * g + 2], d[4 * g + 3]);
  };
  float acc[SLOTS];
#pragma unroll
  for (int i = 0; i < SLOTS; ++i) acc[i] = 0.f;
  // ---- P1: rows (kappa_0 = 16 w + r % 16, comp r / 16), columns kappa_1 = 32 tile + n32; rows 8g + 4h + e
  // (g < 2) hold Re and rows 16 + 8g + 4h + e Im of kappa_0 = 16 w + 8g + 4h + e
  auto pass1 = [&]() {
    const int lv = lane_v(), n32 = lv & 31, h = lv >> 5;
#pragma unroll
    for (int tile = 0; tile < 2; ++tile) {
      floatx16 d = {};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const half8 x = *reinterpret_cast<const half8*>(&L1[l1_at(h, 32 * tile + n32, ks)]);
        d = mfma32(fh[ks], x, d);
        d = mfma32(fl[ks], x, d);
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        float& a = acc[8 * tile + r];
        a = fmaf(d[r], d[r], fmaf(d[r + 8], d[r + 8], a));
      }
    }
  };

  double* out = partial + ((int64_t)sl * F + ch) * (int64_t)CELLS;
  bool flushed = false;
  auto flush = [&]() {
    double* o = out + tid;
    asm volatile("" : "+v"(o));
#pragma unroll
    for (int i = 0; i < SLOTS; ++i) {
      const double v = (double)acc[i] * out_scale;
      o[i * NT] = flushed ? o[i * NT] + v : v;
      acc[i] = 0.f;
    }
    flushed = true;
  };

  // Per sample: D(t) | P0 | P1 and D(t + 1) | ...
  if (t0 < t1) {
    load_raw(t0);
    decode();
    load_raw(min(t0 + 1, t1 - 1));
  }
  int blk = 0;
  for (int64_t t = t0; t < t1; ++t) {
    __syncthreads();
    pass0();
    __syncthreads();
    pass1();
    if (t + 1 < t1) {
      decode();
      load_raw(min(t + 2, t1 - 1));
    }
    if (++blk == time_block) {
      blk = 0;
      flush();
    }
  }
  if (blk > 0 || !flushed) flush();
}

// Natural index kappa_0 * 64 + kappa_1 of cell `cell` (= slot * 256 + thread).
int grid32_cell(int cell) {
  const int slot = cell / 256, tid = cell % 256;
  const int w = tid >> 6, l = tid & 63, h = l >> 5, n32 = l & 31;
  const int tile = slot / 8, r = slot % 8, g = r / 4, e = r % 4;
  const int k0 = 16 * w + 8 * g + 4 * h + e, k1 = 32 * tile + n32;
  return k0 * 64 + k1;
}

hipError_t launch_grid32_mixed(const void* src, int64_t T, int64_t tps, const float2* tw64, double* partial, int F,
                               int n_slices, int time_block, double out_scale, hipStream_t st) {
  if ((reinterpret_cast<uintptr_t>(src) & 3) != 0 || F < 1 || n_slices < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(grid32_mixed_kernel, dim3((unsigned)(n_slices * F)), dim3(g32::NT), 0, st,
                     static_cast<const uint8_t*>(src), T, tps, tw64, partial, F, time_block, out_scale);
  return hipGetLastError();
}

}  // namespace omni
