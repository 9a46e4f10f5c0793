// Fused mixed-precision kernel for the (16,16,16) grid that remains of the
// 16x16-of-16x16 array after its front pass (gfx950, float16 matrix cores).
//
// Input: one float16 tile per (time sample, Fourier "channel" of the front
// axis), planar [re | im][a][b][c], 16 antennas per axis, scaled by 1/16.
// Every axis' zero-padded 32-point DFT (Sec. II.A/II.C) is a dense 32 x 16
// complex matrix product per line, real-embedded
//   [Re y ; Im y] = [[Re W, -Im W], [Im W, Re W]] [Re x ; Im x]   (K = 32),
// on v_mfma_f32_32x32x16_f16 (float16 operands, float32 accumulation), with W
// split into float16 hi + lo parts (two MFMAs per product) and scaled by 1/16
// (exact; it keeps every float16 intermediate within the input's range).  The
// |X|^2 accumulators carry those scales; `out_scale` restores them when they
// are written out.
//
// Work-group = (time slice, channel), 1024 threads (16 waves, one work-group
// per CU); it owns all 32768 cells of the channel, 32 float32 accumulators per
// lane.  Per sample:
//   A  axis c, lines (a, b): data x W^T, 8 row tiles, each with both halves
//      of kappa_c, in waves 0-7 -> LB
//   B  axis b, lines (a, kappa_c): data x W^T, one row tile per wave, both
//      halves of kappa_b -> LC
//   C  axis a, lines (kappa_b, kappa_c): W x data, two column tiles per wave,
//      both halves of kappa_a, so that the real and the imaginary row of an
//      output land in the same lane -> |X|^2 in registers.
// Inputs are taken in even-odd order, so each pair of output halves shares
// the product of its even inputs (6 matrix-core instructions per pair
// instead of 8).
// In A and B the rows of a tile are lines ordered with the next pass'
// contracted axis fastest, so a lane stores 4 consecutive values of it with
// one 8-byte LDS write and the next pass reads an operand with one 16-byte
// read.  Each lane loads its pass-A operands straight from HBM into registers,
// one sample ahead, and the passes are software-pipelined over samples (two
// barriers per sample).
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace omni {

namespace m163 {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int NT = 1024;
constexpr int CELLS = 32768;
constexpr int SLOTS = 32;  // accumulators per lane

__device__ __forceinline__ floatx16 mfma(half8 a, half8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// LB [comp][a][kappa_c][b] and LC [comp][kappa_b][kappa_c][a], in halves: rows of 16 halves (four
// 4-half units), blocks of 32 rows padded by 8 halves (so consecutive blocks start 16 bytes apart modulo
// 256).  Measured on gfx950, an 8-byte store is served 16 lanes at a time from 32 banks (a 128-byte
// window) and a 16-byte load 16 lanes at a time from 64 banks (256 bytes).  The units of a row are
// XOR-permuted: in LB by (kappa_c / 4) % 4, in LC by bit 3 of kappa_b (bit 0 of the unit) and bit 3 of
// kappa_c (bit 1).  Then each 8-byte store (16 lanes: 16 consecutive rows of LB, or the same row of
// 16 LC blocks) and each 16-byte load (16 lanes: 16 LB blocks, or 16 consecutive LC rows) meets every
// bank at most once.
constexpr int BLK = 520;         // 32 x 16 + 8
constexpr int CMP = 16 * BLK;    // component stride of LB (16 values of a)
constexpr int CMPC = 32 * BLK;   // component stride of LC (all 32 values of kappa_b)
__device__ __forceinline__ int lb_x(int kc) { return (kc >> 2) & 3; }
__device__ __forceinline__ int lc_x(int kb, int kc) { return ((kb >> 3) & 1) | (((kc >> 3) & 1) << 1); }
__device__ __forceinline__ int lb_at(int comp, int a, int kc, int b) {
  return comp * CMP + a * BLK + kc * 16 + (b ^ (4 * lb_x(kc)));
}
__device__ __forceinline__ int lc_at(int comp, int kb, int kc, int a) {
  return comp * CMPC + kb * BLK + kc * 16 + (a ^ (4 * lc_x(kb, kc)));
}
// the aligned 16 bytes of a row (units permuted by x) that hold its halves j0 .. j0 + 7 (j0 a multiple of
// 8); their two units come in swapped order when x is odd, which the caller's DFT operand absorbs
__device__ __forceinline__ half8 load8(const _Float16* row, int j0, int x) {
  return *reinterpret_cast<const half8*>(row + (j0 ^ (8 * (x >> 1))));
}

__device__ __forceinline__ half4 to_half4(const floatx16& d, int g) {
  half4 v;
  v[0] = (_Float16)d[4 * g];
  v[1] = (_Float16)d[4 * g + 1];
  v[2] = (_Float16)d[4 * g + 2];
  v[3] = (_Float16)d[4 * g + 3];
  return v;
}

}  // namespace m163

// Grid: n_slices x F work-groups (F = channels of this launch), 1024 threads.
// src: [T][F][2][4096] halves; tw: w_32^q, q < 32 (float32); partial:
// [n_slices][F][32768] float64 in the cell order given by fused16x3_cell.
__global__ __launch_bounds__(1024) void fused16x3_mixed_kernel(const _Float16* __restrict__ src, int64_t T,
                                                              int64_t t_per_slice, const float2* __restrict__ tw,
                                                              double* __restrict__ partial, int F, int time_block,
                                                              int accumulate, double out_scale) {
  using namespace m163;
  __shared__ __attribute__((aligned(16))) _Float16 LB[2 * CMP];
  __shared__ __attribute__((aligned(16))) _Float16 LC[2 * CMPC];
  // (the wave index read as a wave-uniform value: the unit order of the operand loads depends on it alone)
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, h = l >> 5,
            n32 = l & 31;
  const int ch = blockIdx.x % F;
  const int s = blockIdx.x / F;
  const int64_t t0 = (int64_t)s * t_per_slice;
  const int64_t t1 = min(T, t0 + t_per_slice);

  // Every contraction takes its 16 inputs in "even-odd" order: position p holds input sig(p) = 2 p for
  // p < 8 and 2 (p - 8) + 1 for p >= 8, so K-step 0 carries the even inputs and K-step 1 the odd ones (the
  // rows of LB and LC are stored in that order: pass A and pass B map their output rows to lines through sig).
  // DFT operand of this lane for K step ks: output (co = n32 / 16, kappa = n32 % 16), input (ci = h,
  // j = sig(8 ks + (i ^ 4 sw))).  The outputs kappa + 16 use the same operand with the odd inputs negated
  // (w_32^{(kappa + 16) j} = (-1)^j w_32^{kappa j}): the whole K-step-1 operand of the data, by flip_all.
  // In waves with sw = 1 every operand row loaded in passes B and C has its two 4-half units swapped (bit 0
  // of the rows' unit permutation equals bit 1 of the wave index, see pass C's tiles), and pass A builds its
  // operand swapped likewise, so the operand takes position 8 ks + (i ^ 4) at element i.
  const int sw = (w >> 1) & 1;
  auto sig = [](int p) { return p < 8 ? 2 * p : 2 * p - 15; };
  half8 Wh[2], Wl[2];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int kap = n32 & 15, j = sig(8 * ks + (i ^ (4 * sw)));
      const float2 wv = tw[(kap * j) & 31];
      const bool co = n32 >= 16, ci = h != 0;
      const float v = (!co ? (!ci ? wv.x : -wv.y) : (!ci ? wv.y : wv.x)) * 0.0625f;
      const _Float16 hi = (_Float16)v;
      Wh[ks][i] = hi;
      Wl[ks][i] = (_Float16)(v - (float)hi);
    }
  }
  // negate every entry (both halves of each 32-bit word) when `mask` is 0x80008000
  auto flip_all = [](half8 v, uint32_t mask) {
    uint4 b = __builtin_bit_cast(uint4, v);
    b.x ^= mask;
    b.y ^= mask;
    b.z ^= mask;
    b.w ^= mask;
    return __builtin_bit_cast(half8, b);
  };

  // pass A: waves w < 8 take row tile rt = w (lines a = 2 rt + n32 / 16, b = sig(n32 % 16)) and both column
  // halves ua (kappa_c in [16 ua, 16 ua + 16)), so the even-input product is formed once for both; waves
  // w >= 8 have no pass-A work.  The lane's operand: component h, the 16 values of c, read straight from HBM
  // into registers, one sample ahead, and put in even-odd order by byte permutes.
  const bool a_wave = w < 8;
  const int rt = w & 7;
  const int a_line = (2 * rt + (n32 >> 4)) * 16 + sig(n32 & 15);
  // (in waves with sw = 1 the two 16-byte halves of the line, c < 8 and c >= 8, are loaded in swapped order)
  // (a wave-uniform tile address plus a 32-bit lane offset, added at each load: the empty asm keeps the
  // compiler from holding 64-bit lane addresses across the loop)
  const int xa_byte = (h * 4096 + a_line * 16) * 2;
  auto load_xa = [&](int64_t t, half8* xa) {
    if (!a_wave) return;
    int off = xa_byte;
    asm volatile("" : "+v"(off));
    const uint2* g = reinterpret_cast<const uint2*>(reinterpret_cast<const char*>(src + (t * F + ch) * 8192) + off);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint2 lo = g[2 * (q ^ sw)], hi = g[2 * (q ^ sw) + 1];
      xa[q] = __builtin_bit_cast(half8, make_uint4(lo.x, lo.y, hi.x, hi.y));
    }
  };
  // even (ks = 0) or odd (ks = 1) entries of the loaded line: each 32-bit word of the result takes the low
  // (even) or high (odd) halves of two consecutive words of the line
  auto even_odd = [](const half8 (&x)[2], int ks) {
    const uint32_t sel = ks ? 0x07060302u : 0x05040100u;
    const uint4 a = __builtin_bit_cast(uint4, x[0]), b = __builtin_bit_cast(uint4, x[1]);
    const uint4 r = make_uint4(__builtin_amdgcn_perm(a.y, a.x, sel), __builtin_amdgcn_perm(a.w, a.z, sel),
                               __builtin_amdgcn_perm(b.y, b.x, sel), __builtin_amdgcn_perm(b.w, b.z, sel));
    return __builtin_bit_cast(half8, r);
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

  half8 xa[2];
  // ---- A: axis c on row tile rt, both halves of kappa_c; this lane's half h reads component h of c
  auto pass_a = [&]() {
    if (!a_wave) return;
    const int co = n32 >> 4;
    const half8 xe = even_odd(xa, 0), xo = even_odd(xa, 1);
    floatx16 e = {};
    e = mfma(xe, Wh[0], e);
    e = mfma(xe, Wl[0], e);
#pragma unroll
    for (int ua = 0; ua < 2; ++ua) {
      const half8 x = ua ? flip_all(xo, 0x80008000u) : xo;
      floatx16 d = mfma(x, Wh[1], e);
      d = mfma(x, Wl[1], d);
      // column n32: (co, kappa_c = 16 ua + n32 % 16); rows 8g + 4h + e: position 8 (g & 1) + 4h + e of b,
      // a = 2 rt + g / 2
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int a = 2 * rt + (g >> 1), b0 = 8 * (g & 1) + 4 * h;
        *reinterpret_cast<half4*>(&LB[lb_at(co, a, 16 * ua + (n32 & 15), b0)]) = to_half4(d, g);
      }
    }
  };
  // ---- B: axis b, row tile mt = w of lines (a = sig(m % 16), kappa_c = 2 mt + m / 16), both halves of
  // kappa_b: the even-input product is formed once, the odd inputs added with and without their sign flip
  auto pass_b = [&]() {
    const int mt = w;
    const int a_in = sig(n32 & 15), kc_in = 2 * mt + (n32 >> 4);
    const _Float16* row = &LB[h * CMP + a_in * BLK + kc_in * 16];
    const half8 xe = load8(row, 0, lb_x(kc_in)), xo = load8(row, 8, lb_x(kc_in));
    floatx16 e = {};
    e = mfma(xe, Wh[0], e);
    e = mfma(xe, Wl[0], e);
    floatx16 d[2];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const half8 x = half ? flip_all(xo, 0x80008000u) : xo;
      d[half] = mfma(x, Wh[1], e);
      d[half] = mfma(x, Wl[1], d[half]);
    }
    const int co = n32 >> 4;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int kb = 16 * half + (n32 & 15);
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int a0 = 8 * (g & 1) + 4 * h, kc = 2 * mt + (g >> 1);
        *reinterpret_cast<half4*>(&LC[lc_at(co, kb, kc, a0)]) = to_half4(d[half], g);
      }
    }
  };
  // ---- C: axis a, column tiles (lines kappa_b, kappa_c = n32), row tiles u; kappa_b takes the bits
  //      (j, w0, w2, w1, w3) of j and the wave index, so that its bit 3 is sw
  auto pass_c = [&]() {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int kb = j + 2 * (w & 1) + 4 * ((w >> 2) & 1) + 8 * sw + 16 * (w >> 3);
      half8 x[2];
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) x[ks] = load8(&LC[h * CMPC + kb * BLK + n32 * 16], 8 * ks, lc_x(kb, n32));
      // the even-input product once; row tile u adds the odd inputs, negated for u = 1 (kappa_a + 16)
      floatx16 e = {};
      e = mfma(Wh[0], x[0], e);
      e = mfma(Wl[0], x[0], e);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const half8 xo = u ? flip_all(x[1], 0x80008000u) : x[1];
        floatx16 d = mfma(Wh[1], xo, e);
        d = mfma(Wl[1], xo, d);
        // rows r < 8 hold Re and rows r + 8 Im of the same kappa_a
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          float& a_ = acc[(j * 2 + u) * 8 + r];
          a_ = fmaf(d[r], d[r], fmaf(d[r + 8], d[r + 8], a_));
        }
      }
    }
  };

  // Two phases per sample, software-pipelined over samples: phase 1 runs A of sample t + 1 and C of
  // sample t, phase 2 runs B of t + 1.  LB is written in phase 1 and read in phase 2, LC the other way
  // round, so one barrier after each phase suffices.  Operands are loaded one sample ahead of A; in the
  // last iteration A and B run on a repeated sample and their outputs are never read.
  if (t0 < t1) {
    load_xa(t0, xa);
    pass_a();
    load_xa(min(t0 + 1, t1 - 1), xa);
    __syncthreads();
    pass_b();
    __syncthreads();
  }
  int blk = 0;
  for (int64_t t = t0; t < t1; ++t) {
    pass_a();
    load_xa(min(t + 2, t1 - 1), xa);
    pass_c();
    __syncthreads();
    pass_b();
    __syncthreads();
    if (++blk == time_block) {
      blk = 0;
      flush();
    }
  }
  if (blk > 0 || !flushed) flush();
}

// Natural index (kappa_a * 32 + kappa_b) * 32 + kappa_c of cell `cell` (= slot * 1024 + thread).
int fused16x3_cell(int cell) {
  const int slot = cell / 1024, tid = cell % 1024;
  const int w = tid >> 6, l = tid & 63, h = l >> 5, n32 = l & 31;
  const int r = slot % 8, u = (slot / 8) % 2, j = slot / 16;
  const int ka = 16 * u + 8 * (r / 4) + 4 * h + (r % 4);
  const int kb = j + 2 * (w & 1) + 4 * ((w >> 2) & 1) + 8 * ((w >> 1) & 1) + 16 * (w >> 3);
  const int kc = n32;
  return (ka * 32 + kb) * 32 + kc;
}

hipError_t launch_fused16x3_mixed(const void* src, int64_t T, int64_t tps, const float2* tw, double* partial, int F,
                                  int n_slices, int time_block, int accumulate, double out_scale, hipStream_t st) {
  if ((reinterpret_cast<uintptr_t>(src) & 15) != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fused16x3_mixed_kernel, dim3((unsigned)(n_slices * F)), dim3(m163::NT), 0, st,
                     static_cast<const _Float16*>(src), T, tps, tw, partial, F, time_block, accumulate, out_scale);
  return hipGetLastError();
}

}  // namespace omni
