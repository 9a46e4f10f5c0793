// Fused mixed-precision correlator for the two-level 8x8-of-8x8 hierarchy
// (four axes of 8 antennas padded to 16, M = 65536 cells per channel), gfx950.
//
// Each axis' zero-padded 16-point DFT (Sec. II.A/II.C) is a dense complex
// matrix-vector product per line, y = W x with W[o][j] = w16^{o j} (16 x 8),
// computed for 32 lines at a time as one real-embedded GEMM on the matrix
// cores (v_mfma_f32_32x32x16_f16: float16 operands, float32 accumulation):
//   rows/columns [Re y ; Im y] = [[Re W, -Im W], [Im W, Re W]] [Re x ; Im x].
// W is split into float16 hi + lo parts (hi = rn(W), lo = rn(W - hi)), two
// MFMAs per tile, so the twiddles carry ~22 bits.  Every stage is scaled by
// 1/8 (folded into W, exact), which bounds every float16 intermediate by the
// input's maximum magnitude; the 2^24 on |X|^2 is undone at the end.
//
// Work-group = (time slice, channel f, residue h of kappa_3 mod 2), 1024
// threads (16 waves).  It owns the 32768 cells with kappa_3 = h (mod 2); each
// lane keeps 32 of them in float32 registers for the whole slice.  Per time
// sample (one 32-line tile per wave and pass, two in P4):
//   P1 axis 3 (i3) straight from HBM; of its 16 outputs the 8 with
//      kappa_3 = 2q + h are kept -> LDS L2
//   P2 axis 2, 16 outputs -> L3
//   P3 axis 1 and P4 axis 0 in two halves of kappa_2: P3 -> L4, then P4 squares
//   the modulus (real and imaginary rows of an output land in the same lane)
//   and accumulates.
// In every pass the 32 lines of a tile are ordered with the next pass'
// contracted axis fastest, so each lane stores 4 consecutive values of it with
// one 8-byte LDS write and the next pass reads an operand with one 16-byte read.
// The next sample's input is prefetched during the current one, and the passes
// are software-pipelined over samples (two barriers per sample).
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace omni {

namespace f8m {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int NT = 1024;
constexpr int CPL = 32;  // cells per lane

__device__ __forceinline__ floatx16 mfma(half8 a, half8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// Real-embedded DFT operand entry for lane column `col` and row k (0..15) of
// the K dimension: output o = col % 16 (real part for col < 16, imaginary part
// otherwise), input j = k % 8 (real part for k < 8, imaginary otherwise).
__device__ __forceinline__ float embed(float2 w, bool im_out, bool im_in) {
  return !im_out ? (!im_in ? w.x : -w.y) : (!im_in ? w.y : w.x);
}

__device__ __forceinline__ void store4(_Float16* p, float a, float b, float c, float d) {
  half4 v;
  v[0] = (_Float16)a;
  v[1] = (_Float16)b;
  v[2] = (_Float16)c;
  v[3] = (_Float16)d;
  *reinterpret_cast<half4*>(p) = v;
}

// Raw input of one P1 operand: 8 samples along i3 (16 bytes of ci8, 8 of ci4),
// converted to float16 without int -> float conversions: a small integer u
// (0 <= u < 1024) becomes the float16 1024 + u by placing u in the low
// mantissa bits under the exponent byte 0x64; subtracting 1024 + bias (bias =
// 128 for int8, 8 for int4, the offset that made u non-negative) is exact.
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t biased_pair(uint32_t bytes, uint32_t sel) {
  return __builtin_amdgcn_perm(0x64646464u, bytes, sel);  // selector byte 4 = 0x64, 0-3 = bytes
}
__device__ __forceinline__ half8 unbias(uint32_t p0, uint32_t p1, uint32_t p2, uint32_t p3, float bias) {
  const _Float16 b = (_Float16)(1024.f + bias);
  const half2v bb = {b, b};
  const half2v h0 = __builtin_bit_cast(half2v, p0) - bb, h1 = __builtin_bit_cast(half2v, p1) - bb;
  const half2v h2 = __builtin_bit_cast(half2v, p2) - bb, h3 = __builtin_bit_cast(half2v, p3) - bb;
  const half4 lo = __builtin_shufflevector(h0, h1, 0, 1, 2, 3), hi = __builtin_shufflevector(h2, h3, 0, 1, 2, 3);
  return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}
template <int FMT>
struct Raw;
template <>
struct Raw<1> {  // word k = [re 2k, im 2k, re 2k+1, im 2k+1] (int8)
  uint4 v;
  __device__ __forceinline__ void load(const void* __restrict__ base, int64_t sample) {
    v = *reinterpret_cast<const uint4*>(reinterpret_cast<const int8_t*>(base) + 2 * sample);
  }
  __device__ __forceinline__ half8 to_half(int comp) const {
    const uint32_t sel = comp ? 0x04030401u : 0x04020400u;
    return unbias(biased_pair(v.x ^ 0x80808080u, sel), biased_pair(v.y ^ 0x80808080u, sel),
                  biased_pair(v.z ^ 0x80808080u, sel), biased_pair(v.w ^ 0x80808080u, sel), 128.f);
  }
};
template <>
struct Raw<2> {  // byte i of word k = sample 4k + i, real part in the high nibble (int4)
  uint2 v;
  __device__ __forceinline__ void load(const void* __restrict__ base, int64_t sample) {
    v = *reinterpret_cast<const uint2*>(reinterpret_cast<const int8_t*>(base) + sample);
  }
  __device__ __forceinline__ half8 to_half(int comp) const {
    const uint32_t x = v.x ^ 0x88888888u, y = v.y ^ 0x88888888u;
    const uint32_t ux = (comp ? x : x >> 4) & 0x0F0F0F0Fu, uy = (comp ? y : y >> 4) & 0x0F0F0F0Fu;
    return unbias(biased_pair(ux, 0x04010400u), biased_pair(ux, 0x04030402u), biased_pair(uy, 0x04010400u),
                  biased_pair(uy, 0x04030402u), 8.f);
  }
};

// LDS layouts (float16).  A 16-byte operand row holds the 8 values of one
// component along the axis the next pass contracts, as two 4-value units.
// Measured on gfx950, an 8-byte store is served 16 lanes at a time from 32
// banks (a 128-byte window) and a 16-byte load 16 lanes at a time from 64 banks
// (256 bytes).  Rows are XOR-permuted within their block, and in L3 the two
// units of a row are swapped for kappa_2 >= 8, so that the stores of each pass
// and the loads of the next meet every bank once (the P3 -> P4 stores: twice).
//   L2 [comp][i0][q][i1 ^ q][i2]                (P1 -> P2)
//   L3 [comp][q][k2][i0 ^ (k2 % 8)][i1]         (P2 -> P3; units swapped for k2 >= 8)
//   L4 [buf][comp][k1][(8 q + k2c) ^ k1][i0]    (P3 -> P4)
__device__ __forceinline__ int l2_row(int comp, int i0, int q, int i1) {
  return ((comp * 8 + i0) * 8 + q) * 8 + (i1 ^ q);
}
__device__ __forceinline__ int l3_row(int comp, int q, int k2, int i0) {
  return ((comp * 8 + q) * 16 + k2) * 8 + (i0 ^ (k2 & 7));
}
__device__ __forceinline__ int l4_row(int comp, int k1, int idx2) {
  return (comp * 16 + k1) * 64 + (idx2 ^ k1);
}

}  // namespace f8m

// One time sample per iteration, 1024 threads (16 waves) in 112 KiB of LDS:
// one work-group per CU, up to 128 VGPRs per lane.
template <int FMT>
__global__ __launch_bounds__(f8m::NT) void fused8x4_mixed_kernel(const void* __restrict__ src, int64_t T,
                                                                int64_t t_per_slice,
                                                                const float2* __restrict__ tw16,
                                                                double* __restrict__ partial, int F,
                                                                int xcd_groups, int time_block) {
  using namespace f8m;
  __shared__ _Float16 L2[2 * 8 * 8 * 8 * 8];
  __shared__ _Float16 L3[2 * 8 * 16 * 8 * 8];
  __shared__ _Float16 L4[2][2 * 16 * 64 * 8];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col = lane & 31, hh = lane >> 5;
  const int b = blockIdx.x;
  int grp, h;
  if (xcd_groups) {
    const int xcd = b & 7, j = b >> 3;
    grp = xcd + 8 * (j >> 1);
    h = j & 1;
  } else {
    grp = b >> 1;
    h = b & 1;
  }
  const int f = grp % F;
  const int s = grp / F;

  // DFT operand registers: the same contents serve as the B operand of
  // Y^T = X^T W^T (passes 1-3) and as the A operand of Y = W X (pass 4).
  half8 Wf_hi, Wf_lo;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = 8 * hh + i, j = k & 7;
    const float2 w = tw16[((col & 15) * j) & 15];
    const float v = 0.125f * embed(w, col >= 16, k >= 8);
    const _Float16 hi = (_Float16)v;
    Wf_hi[i] = hi;
    Wf_lo[i] = (_Float16)(v - (float)hi);
  }

  float acc[CPL];
#pragma unroll
  for (int i = 0; i < CPL; ++i) acc[i] = 0.f;
  const floatx16 zero = {};

  // wave w = 2 i0 + tt.  P1 tile: lines r = col -> (i0, i1, i2) = (w / 2, 4 tt + r / 8, r % 8)
  const int i0w = wave >> 1, tw = wave & 1;
  const int p1_off = ((i0w * 8 + 4 * tw + (col >> 3)) * 8 + (col & 7)) * 8;
  const int64_t t0 = (int64_t)s * t_per_slice;
  const int64_t t1 = min(T, t0 + t_per_slice);
  Raw<FMT> raw;
  if (t0 < t1) raw.load(src, (t0 * F + f) * 4096 + p1_off);
  const bool keep = (col & 1) == h;

  // ---- P1: axis 3 from the prefetched sample, then the next sample's prefetch (the last sample
  //      re-reads its own: an unconditional load into the consumed registers needs no second copy)
  auto pass1 = [&](int64_t t_next) {
    const half8 a = raw.to_half(hh);
    floatx16 d = mfma(a, Wf_hi, zero);
    d = mfma(a, Wf_lo, d);
    // column: kappa_3 = col % 16 (re / im halves); keep kappa_3 = 2q + h.  rows: i1 = 4 tt + i, i2 = 4 hh + j
    const int comp = col >> 4, q = (col & 15) >> 1;
    if (keep) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        store4(&L2[l2_row(comp, i0w, q, 4 * tw + i) * 8 + 4 * hh], d[4 * i], d[4 * i + 1], d[4 * i + 2],
               d[4 * i + 3]);
    }
    // the prefetch goes out after everything above, so that no wait for another memory access (a
    // register reload, say) can stall on it before its data are needed
    __builtin_amdgcn_sched_barrier(0);
    raw.load(src, (t_next * F + f) * 4096 + p1_off);
  };
  // ---- P2: axis 2; lines (i0, q, i1) = (w / 2, 4 tt + r / 8, r % 8)
  auto pass2_mfma = [&]() {
    const half8 a = *reinterpret_cast<const half8*>(&L2[l2_row(hh, i0w, 4 * tw + (col >> 3), col & 7) * 8]);
    const floatx16 d = mfma(a, Wf_hi, zero);
    return mfma(a, Wf_lo, d);
  };
  auto pass2_store = [&](const floatx16& d) {
    // column -> (comp, k2); rows -> q = 4 tt + i, i1 = 4 hh + j
    const int comp = col >> 4, k2 = col & 15;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      store4(&L3[l3_row(comp, 4 * tw + i, k2, i0w) * 8 + 4 * (hh ^ (k2 >> 3))], d[4 * i], d[4 * i + 1],
             d[4 * i + 2], d[4 * i + 3]);
  };
  // ---- P3 (axis 1) for kappa_2 half cc into L4[cc]: lines (idx2, i0) = (4 w + r / 8, r % 8) with
  //      idx2 = 8 q + k2c, kappa_2 = 8 cc + k2c
  auto pass3_mfma = [&](int cc) {
    const int idx2 = 4 * wave + (col >> 3);
    half8 a = *reinterpret_cast<const half8*>(&L3[l3_row(hh, idx2 >> 3, 8 * cc + (idx2 & 7), col & 7) * 8]);
    if (cc) a = __builtin_shufflevector(a, a, 4, 5, 6, 7, 0, 1, 2, 3);  // units stored swapped for k2 >= 8
    const floatx16 d = mfma(a, Wf_hi, zero);
    return mfma(a, Wf_lo, d);
  };
  auto pass3_store = [&](int cc, const floatx16& d) {
    const int comp = col >> 4, k1 = col & 15;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      store4(&L4[cc][l4_row(comp, k1, 4 * wave + i) * 8 + 4 * hh], d[4 * i], d[4 * i + 1], d[4 * i + 2],
             d[4 * i + 3]);
  };
  // ---- P4 (axis 0) on lines (k1, idx2) = (w, 32 tt + r): W x data, rows of d: 4hh + j (re),
  //      8 + 4hh + j (re), 16 + 4hh + j (im), 24 + 4hh + j (im); square and accumulate
  auto pass4_mfma = [&](int cc, int tt) {
    const half8 bop = *reinterpret_cast<const half8*>(&L4[cc][l4_row(hh, wave, 32 * tt + col) * 8]);
    const floatx16 d = mfma(Wf_hi, bop, zero);
    return mfma(Wf_lo, bop, d);
  };
  auto pass4_square = [&](int cc, int tt, const floatx16& d) {
    const int base = cc * 16 + tt * 8;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[base + j] = fmaf(d[j], d[j], fmaf(d[8 + j], d[8 + j], acc[base + j]));
      acc[base + 4 + j] = fmaf(d[4 + j], d[4 + j], fmaf(d[12 + j], d[12 + j], acc[base + 4 + j]));
    }
  };

  // Two phases per sample, software-pipelined over samples: phase A runs P1 of sample t + 1 and P3 of
  // sample t, phase B runs P2 of t + 1 and P4 of t.  Each buffer is written in one phase and read in the
  // other (L2: P1 -> P2, L3: P2 -> P3, L4: P3 -> P4), so one barrier after each phase suffices.
  if (t0 < t1) {
    pass1(min(t0 + 1, t1 - 1));
    __syncthreads();
    pass2_store(pass2_mfma());
    __syncthreads();
  }
  // float32 blocks of time_block samples are added into the float64 partial sums of this work-group
  // (the first block stores; |X|^2 carried 8^-8 = 2^-24 from the four scaled stages)
  double* const out = partial + ((int64_t)grp * 2 + h) * 32768;
  bool flushed = false;
  auto flush = [&]() {
    // addresses formed here (the empty asm keeps them out of the time loop); loads in groups of 4
    double* o = out + tid;
    asm volatile("" : "+v"(o));
    if (flushed) {
#pragma unroll
      for (int i0 = 0; i0 < CPL; i0 += 4) {
        double prev[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) prev[k] = o[(i0 + k) * NT];
#pragma unroll
        for (int k = 0; k < 4; ++k) o[(i0 + k) * NT] = prev[k] + (double)acc[i0 + k] * 16777216.0;
      }
    } else {
#pragma unroll
      for (int i = 0; i < CPL; ++i) o[i * NT] = (double)acc[i] * 16777216.0;
    }
#pragma unroll
    for (int i = 0; i < CPL; ++i) acc[i] = 0.f;
    flushed = true;
  };
  int blk = 0;
  for (int64_t t = t0; t < t1; ++t) {
    const bool more = t + 1 < t1;  // uniform
    {
      const floatx16 d0 = pass3_mfma(0);
      const floatx16 d1 = pass3_mfma(1);
      if (more) pass1(min(t + 2, t1 - 1));
      pass3_store(0, d0);
      pass3_store(1, d1);
    }
    __syncthreads();
    {
      const floatx16 d0 = pass4_mfma(0, 0);
      const floatx16 d1 = pass4_mfma(0, 1);
      if (more) pass2_store(pass2_mfma());
      pass4_square(0, 0, d0);
      const floatx16 d2 = pass4_mfma(1, 0);
      pass4_square(0, 1, d1);
      const floatx16 d3 = pass4_mfma(1, 1);
      pass4_square(1, 0, d2);
      pass4_square(1, 1, d3);
    }
    __syncthreads();
    if (++blk == time_block) {
      blk = 0;
      flush();
    }
  }
  if (blk > 0 || !flushed) flush();
}

hipError_t launch_fused8x4_mixed(int fmt, const void* src, int64_t T, int64_t tps, const float2* tw16,
                                 double* partial, int F, int n_slices, int time_block, hipStream_t st) {
  const int groups = n_slices * F;
  const int xcd = (groups % 8 == 0) ? 1 : 0;
  const dim3 grid(groups * 2), block(f8m::NT);
  if (fmt == 1)
    hipLaunchKernelGGL(fused8x4_mixed_kernel<1>, grid, block, 0, st, src, T, tps, tw16, partial, F, xcd,
                       time_block);
  else if (fmt == 2)
    hipLaunchKernelGGL(fused8x4_mixed_kernel<2>, grid, block, 0, st, src, T, tps, tw16, partial, F, xcd,
                       time_block);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace omni
