// Fused mixed-precision kernel for the (8,8,4,4) grid that remains of the
// three-level 16x16 / 8x8 / 4x4 hierarchy after its two front passes (gfx950,
// float16 matrix cores).
//
// Input: one float16 tile per (time sample, Fourier "channel" of the front
// axes), planar [re | im][a][b][c][d] (8, 8, 4, 4 antennas), scaled by the
// front pass.  The zero-padded DFTs (Sec. II.A/II.C) are dense complex matrix
// products, real-embedded as in the other matrix-core kernels,
//   [Re y ; Im y] = [[Re W, -Im W], [Im W, Re W]] [Re x ; Im x],
// on v_mfma_f32_32x32x16_f16 with W split into float16 hi + lo parts:
//   P1 axes c and d together: the 8x8 outputs of the 4x4 inputs (Kronecker
//      product of two 8 x 4 DFTs, K = 32), lines (a, b), W scaled by 1/16
//   P2 axis b: 16 x 8, lines (a, kappa_cd), W scaled by 1/8
//   P3 axis a: 16 x 8, W x data, lines (kappa_b, kappa_cd), so that the real
//      and imaginary row of an output land in one lane -> |X|^2 in registers.
// The scales keep every float16 intermediate within the input's range;
// `out_scale` undoes them on |X|^2.  Work-group = (time slice, channel), 512
// threads, all 16384 cells of the channel, 32 float32 accumulators per lane.
// LDS rows are padded and their units swapped per row so that the 8-byte
// stores and the 16-byte operand loads (16 lanes at a time each) touch distinct
// banks.  Each lane loads its P1 operands straight from HBM into registers, one
// sample ahead, and the passes are software-pipelined over samples (two
// barriers per sample).
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace omni {

namespace m8844 {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int NT = 512;
constexpr int CELLS = 16384;
constexpr int SLOTS = 32;

__device__ __forceinline__ floatx16 mfma(half8 a, half8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// LB [comp][a 8][kappa_cd 64][b 8]: a-blocks of 64 rows of 8 halves, padded by 16 halves;
// LC [comp][kappa_b 16][kappa_cd 64][a 8]: kappa_b-blocks padded by 8 halves.  Measured on gfx950, an
// 8-byte store is served 16 lanes at a time from 32 banks (a 128-byte window) and a 16-byte load 16
// lanes at a time from 64 banks (256 bytes); the two 4-half units of a row are swapped for rows with
// bit 3 of kappa_cd set (LB) or of kappa_b set (LC), so that the stores of 16 consecutive rows (LB) or
// of one row in 16 blocks (LC) meet every bank once.  The loads take whole rows; the swap is absorbed
// by the DFT operand (the rows a wave loads are all swapped, or none).
constexpr int LB_BLK = 64 * 8 + 16;
constexpr int LB_CMP = 8 * LB_BLK;
constexpr int LC_BLK = 64 * 8 + 8;
constexpr int LC_CMP = 16 * LC_BLK;

__device__ __forceinline__ int lb_at(int comp, int a, int kcd, int b) {
  return comp * LB_CMP + a * LB_BLK + kcd * 8 + (b ^ (4 * ((kcd >> 3) & 1)));
}
__device__ __forceinline__ int lc_at(int comp, int kb, int kcd, int a) {
  return comp * LC_CMP + kb * LC_BLK + kcd * 8 + (a ^ (4 * ((kb >> 3) & 1)));
}

__device__ __forceinline__ half4 to_half4(const floatx16& d, int g) {
  half4 v;
  v[0] = (_Float16)d[4 * g];
  v[1] = (_Float16)d[4 * g + 1];
  v[2] = (_Float16)d[4 * g + 2];
  v[3] = (_Float16)d[4 * g + 3];
  return v;
}

// real-embedded entry: output component co, input component ci of w (scaled)
__device__ __forceinline__ float embed(float2 w, bool co, bool ci) {
  return !co ? (!ci ? w.x : -w.y) : (!ci ? w.y : w.x);
}

}  // namespace m8844

// Grid: n_slices x F work-groups, 512 threads.  src: [T][F][2][1024] halves;
// tw16 / tw8: w_16^q (q < 16) and w_8^q (q < 8), float32; partial:
// [n_slices][F][16384] float64 in the cell order of fused8844_cell.
__global__ __launch_bounds__(512, 4) void fused8844_mixed_kernel(const _Float16* __restrict__ src, int64_t T,
                                                              int64_t t_per_slice, const float2* __restrict__ tw16,
                                                              const float2* __restrict__ tw8,
                                                              double* __restrict__ partial, int F, int time_block,
                                                              int accumulate, double out_scale) {
  using namespace m8844;
  __shared__ __attribute__((aligned(16))) _Float16 LB[2 * LB_CMP];
  __shared__ __attribute__((aligned(16))) _Float16 LC[2 * LC_CMP];
  // (the wave index read as a wave-uniform value: the unit order of the operand loads depends on it alone)
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, h = l >> 5,
            n32 = l & 31;
  const bool co = n32 >= 16;
  const int ch = blockIdx.x % F;
  const int s = blockIdx.x / F;
  const int64_t t0 = (int64_t)s * t_per_slice;
  const int64_t t1 = min(T, t0 + t_per_slice);

  // P1 operand of this wave's column tile ct = w % 4: column n32 = (co, kappa_cd = 16 ct + n32 % 16),
  // K = (ci = h, j = 8 ks + i) with j = 4 c + d; w = w_8^{kc c} w_8^{kd d} / 16
  const int ct = w & 3, mt1 = w >> 2;
  half8 W1h[2], W1l[2];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int kcd = 16 * ct + (n32 & 15), j = 8 * ks + i;
      const int kc = kcd >> 3, kd = kcd & 7, c = j >> 2, d = j & 3;
      const float2 wc = tw8[(kc * c) & 7], wd = tw8[(kd * d) & 7];
      const float2 wv = make_float2(wc.x * wd.x - wc.y * wd.y, wc.x * wd.y + wc.y * wd.x);
      const float v = embed(wv, co, h != 0) * 0.0625f;
      const _Float16 hi = (_Float16)v;
      W1h[ks][i] = hi;
      W1l[ks][i] = (_Float16)(v - (float)hi);
    }
  }
  // P2 / P3 operand: output (co, kappa = n32 % 16), K = (ci = h, j < 8): w_16^{kappa j} / 8.  In odd waves
  // every row that P2 and P3 load from LDS has its two units swapped (bit 3 of kappa_cd, resp. of
  // kappa_b, equals the wave's bit 0), so there the operand takes input j = i ^ 4 at position i instead
  // of swapping the loaded data back.
  const int sw = w & 1;
  half8 W2h, W2l;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float v = embed(tw16[((n32 & 15) * (i ^ (4 * sw))) & 15], co, h != 0) * 0.125f;
    const _Float16 hi = (_Float16)v;
    W2h[i] = hi;
    W2l[i] = (_Float16)(v - (float)hi);
  }

  // P1 operand of this lane: row tile mt1, line mt1 * 32 + n32 = a * 8 + b, component h, 16 halves
  // (j = 4 c + d); read straight from HBM into registers, one sample ahead
  // (a wave-uniform tile address plus a 32-bit lane offset, added at each load: the empty asm keeps
  // the compiler from holding a 64-bit address per lane across the loop)
  const int p1_byte = (h * 1024 + (mt1 * 32 + n32) * 16) * 2;
  auto load_x1 = [&](int64_t t, half8* x1) {
    const char* tile = reinterpret_cast<const char*>(src + (t * F + ch) * 2048);
    int off = p1_byte;
    asm volatile("" : "+v"(off));
    const half8* g = reinterpret_cast<const half8*>(tile + off);
    x1[0] = g[0];
    x1[1] = g[1];
  };

  float acc[SLOTS];
#pragma unroll
  for (int i = 0; i < SLOTS; ++i) acc[i] = 0.f;
  double* out = partial + ((int64_t)s * F + ch) * CELLS;
  bool flushed = false;
  auto flush = [&]() {
    // addresses formed here (the empty asm keeps them out of the time loop); loads in groups of 8
    double* o = out + tid;
    asm volatile("" : "+v"(o));
    if (accumulate || flushed) {
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

  half8 x1[2];
  // ---- P1: row tile mt1 (lines mt1 * 32 + n32 = a * 8 + b), column tile ct
  auto pass1 = [&]() {
    floatx16 d = {};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      d = mfma(x1[ks], W1h[ks], d);
      d = mfma(x1[ks], W1l[ks], d);
    }
    // rows 8g + 4h + e: line mt1 * 32 + 8g + 4h + e -> a = 4 mt1 + g, b = 4h + e
    const int kcd = 16 * ct + (n32 & 15);
#pragma unroll
    for (int g = 0; g < 4; ++g)
      *reinterpret_cast<half4*>(&LB[lb_at(co, 4 * mt1 + g, kcd, 4 * h)]) = to_half4(d, g);
  };
  // ---- P2: row tiles 2w, 2w + 1 (lines mt * 32 + n32: a = n32 % 8, kappa_cd = 4 mt + n32 / 8)
  auto pass2 = [&]() {
#pragma unroll
    for (int jm = 0; jm < 2; ++jm) {
      const int mt = 2 * w + jm;
      const int a_in = n32 & 7, kcd_in = 4 * mt + (n32 >> 3);
      const half8 x = *reinterpret_cast<const half8*>(&LB[h * LB_CMP + a_in * LB_BLK + kcd_in * 8]);
      floatx16 d = {};
      d = mfma(x, W2h, d);
      d = mfma(x, W2l, d);
      // column n32: (co, kappa_b = n32 % 16); rows 8g + 4h + e: a = 4h + e, kappa_cd = 4 mt + g
#pragma unroll
      for (int g = 0; g < 4; ++g)
        *reinterpret_cast<half4*>(&LC[lc_at(co, n32 & 15, 4 * mt + g, 4 * h)]) = to_half4(d, g);
    }
  };
  // ---- P3: four column tiles j of lines (kappa_b, kappa_cd = 32 (j % 2) + n32) with
  //      kappa_b = 8 (w % 2) + 2 (w / 2) + j / 2: bit 3 of kappa_b is the wave's bit 0
  auto pass3 = [&]() {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kb = 8 * sw + 2 * (w >> 1) + (j >> 1), kcd = 32 * (j & 1) + n32;
      const half8 x = *reinterpret_cast<const half8*>(&LC[h * LC_CMP + kb * LC_BLK + kcd * 8]);
      floatx16 d = {};
      d = mfma(W2h, x, d);
      d = mfma(W2l, x, d);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        float& a_ = acc[j * 8 + r];
        a_ = fmaf(d[r], d[r], fmaf(d[r + 8], d[r + 8], a_));
      }
    }
  };

  // Two phases per sample, software-pipelined over samples: phase 1 runs P1 of sample t + 1 and P3 of
  // sample t, phase 2 runs P2 of t + 1.  LB is written in phase 1 and read in phase 2, LC the other way
  // round, so one barrier after each phase suffices.  Operands are loaded one sample ahead of P1; in the
  // last iteration P1 and P2 run on a repeated sample and their outputs are never read.
  if (t0 < t1) {
    load_x1(t0, x1);
    pass1();
    load_x1(min(t0 + 1, t1 - 1), x1);
    __syncthreads();
    pass2();
    __syncthreads();
  }
  int blk = 0;
  for (int64_t t = t0; t < t1; ++t) {
    pass1();
    load_x1(min(t + 2, t1 - 1), x1);
    pass3();
    __syncthreads();
    pass2();
    __syncthreads();
    if (++blk == time_block) {
      blk = 0;
      flush();
    }
  }
  if (blk > 0 || !flushed) flush();
}

// Natural index ((kappa_a * 16 + kappa_b) * 8 + kappa_c) * 8 + kappa_d of cell `cell` (= slot * 512 + thread).
int fused8844_cell(int cell) {
  const int slot = cell / 512, tid = cell % 512;
  const int w = tid >> 6, l = tid & 63, h = l >> 5, n32 = l & 31;
  const int r = slot % 8, j = slot / 8;
  const int kb = 8 * (w & 1) + 2 * (w >> 1) + (j >> 1), kcd = 32 * (j & 1) + n32;
  const int ka = 8 * (r / 4) + 4 * h + (r % 4);
  return (ka * 16 + kb) * 64 + kcd;
}

hipError_t launch_fused8844_mixed(const void* src, int64_t T, int64_t tps, const float2* tw16, const float2* tw8,
                                  double* partial, int F, int n_slices, int time_block, int accumulate,
                                  double out_scale, hipStream_t st) {
  if ((reinterpret_cast<uintptr_t>(src) & 15) != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fused8844_mixed_kernel, dim3((unsigned)(n_slices * F)), dim3(512), 0, st,
                     static_cast<const _Float16*>(src), T, tps, tw16, tw8, partial, F, time_block, accumulate,
                     out_scale);
  return hipGetLastError();
}

}  // namespace omni
