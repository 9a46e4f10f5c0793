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
// Work-group = (time slice, channel f, residue h of kappa_3 mod 2), 512 threads
// (8 waves).  It owns the 32768 cells with kappa_3 = h (mod 2); each lane keeps
// 64 of them in float32 registers for the whole slice.  Per time sample:
//   P1 axis 3 (i3) straight from HBM; of its 16 outputs the 8 with
//      kappa_3 = 2q + h are kept -> LDS L2
//   P2 axis 2, 16 outputs -> L3
//   P3 axis 1 and P4 axis 0 in four chunks of kappa_2: P3 -> L4, then P4 squares
//   the modulus (real and imaginary rows of an output land in the same lane)
//   and accumulates.
// In every pass the 32 lines of a tile are ordered with the next pass'
// contracted axis fastest, so each lane stores 4 consecutive values of it with
// one 8-byte LDS write and the next pass reads an operand with one 16-byte read.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace omni {

namespace f8m {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int NT = 512;
constexpr int CPL = 64;  // cells per lane

__device__ __forceinline__ floatx16 mfma(half8 a, half8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// Real-embedded DFT operand entry for lane column `col` and row k (0..15) of
// the K dimension: output o = col % 16 (real part for col < 16, imaginary part
// otherwise), input j = k % 8 (real part for k < 8, imaginary otherwise).
__device__ __forceinline__ float embed(float2 w, bool im_out, bool im_in) {
  return !im_out ? (!im_in ? w.x : -w.y) : (!im_in ? w.y : w.x);
}

// 8 samples of one component (0 = re, 1 = im) along i3, from the sample format.
template <int FMT>
__device__ __forceinline__ half8 load_line(const void* __restrict__ base, int64_t sample, int comp);

template <>
__device__ __forceinline__ half8 load_line<1>(const void* __restrict__ base, int64_t sample, int comp) {
  const uint4 v = *reinterpret_cast<const uint4*>(reinterpret_cast<const int8_t*>(base) + 2 * sample);
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  half8 r;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const uint32_t word = w[i >> 1];
    const int sh = 16 * (i & 1) + 8 * comp;
    r[i] = (_Float16)(float)(int8_t)(word >> sh);
  }
  return r;
}

template <>
__device__ __forceinline__ half8 load_line<2>(const void* __restrict__ base, int64_t sample, int comp) {
  const uint2 v = *reinterpret_cast<const uint2*>(reinterpret_cast<const int8_t*>(base) + sample);
  const uint32_t w[2] = {v.x, v.y};
  half8 r;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int8_t byte = (int8_t)(w[i >> 2] >> (8 * (i & 3)));
    const int val = comp == 0 ? (byte >> 4) : ((int8_t)(byte << 4) >> 4);
    r[i] = (_Float16)(float)val;
  }
  return r;
}

__device__ __forceinline__ void store4(_Float16* p, float a, float b, float c, float d) {
  half4 v;
  v[0] = (_Float16)a;
  v[1] = (_Float16)b;
  v[2] = (_Float16)c;
  v[3] = (_Float16)d;
  *reinterpret_cast<half4*>(p) = v;
}

}  // namespace f8m

template <int FMT>
__global__ __launch_bounds__(f8m::NT, 4) void fused8x4_mixed_kernel(const void* __restrict__ src, int64_t T,
                                                                 int64_t t_per_slice,
                                                                 const float2* __restrict__ tw16,
                                                                 double* __restrict__ partial, int F,
                                                                 int xcd_groups) {
  using namespace f8m;
  __shared__ _Float16 L2[2 * 8 * 8 * 8 * 8];   // [comp][i0][i1][q][i2]
  __shared__ _Float16 L3[2 * 8 * 8 * 16 * 8];  // [comp][i0][q][k2][i1]
  __shared__ _Float16 L4[2 * 16 * 8 * 4 * 8];  // [comp][k1][q][k2c][i0]

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
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

  // DFT operands (identical register contents serve as the B operand of
  // Y^T = X^T W^T and as the A operand of Y = W X).
  half8 Wf_hi, Wf_lo;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = 8 * hh + i, j = k & 7;
    const int o = col & 15;
    const float2 w = tw16[(o * j) & 15];
    const float v = 0.125f * embed(w, col >= 16, k >= 8);
    const _Float16 hi = (_Float16)v;
    Wf_hi[i] = hi;
    Wf_lo[i] = (_Float16)(v - (float)hi);
  }

  float acc[CPL];
#pragma unroll
  for (int i = 0; i < CPL; ++i) acc[i] = 0.f;
  const floatx16 zero = {};

  const int64_t t0 = (int64_t)s * t_per_slice;
  const int64_t t1 = min(T, t0 + t_per_slice);
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t tile = (t * F + f) * 4096;
    // ---- P1: axis 3, tiles 2 wave + tt (of 16): line r -> (i0, i1, i2) = (T1/2, 4(T1%2) + r/8, r%8)
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
      const int T1 = 2 * wave + tt;
      const int i0 = T1 >> 1, i1 = 4 * (T1 & 1) + (col >> 3), i2 = col & 7;
      const half8 a = load_line<FMT>(src, tile + ((i0 * 8 + i1) * 8 + i2) * 8, hh);
      floatx16 d = mfma(a, Wf_hi, zero);
      d = mfma(a, Wf_lo, d);
      // column col: kappa_3 = col % 16 (re for col < 16, im otherwise); only kappa_3 = 2q + h is kept.
      // rows -> i1 = 4(T1%2) + i, i2 = 4hh + j
      if (((col & 15) & 1) == h) {
        const int comp = col >> 4, q = (col & 15) >> 1;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int ii1 = 4 * (T1 & 1) + i;
          store4(&L2[(((comp * 8 + i0) * 8 + ii1) * 8 + q) * 8 + 4 * hh], d[4 * i], d[4 * i + 1], d[4 * i + 2],
                 d[4 * i + 3]);
        }
      }
    }
    __syncthreads();
    // ---- P2: axis 2, lines (i0, q, i1), i1 fastest; tiles 2 wave + tt: i0 = T2/2, q = 4(T2%2) + r/8, i1 = r%8
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
      const int T2 = 2 * wave + tt;
      const int i0 = T2 >> 1, q = 4 * (T2 & 1) + (col >> 3), i1 = col & 7;
      const half8 a = *reinterpret_cast<const half8*>(&L2[(((hh * 8 + i0) * 8 + i1) * 8 + q) * 8]);
      floatx16 d = mfma(a, Wf_hi, zero);
      d = mfma(a, Wf_lo, d);
      // column col -> (comp, k2); rows -> q = 4(T2%2) + i, i1 = 4hh + j
      const int comp = col >> 4, k2 = col & 15;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int qq = 4 * (T2 & 1) + i;
        store4(&L3[(((comp * 8 + i0) * 8 + qq) * 16 + k2) * 8 + 4 * hh], d[4 * i], d[4 * i + 1], d[4 * i + 2],
               d[4 * i + 3]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      // ---- P3: axis 1 for kappa_2 in [4cc, 4cc+4): lines (i0, q, k2c), i0 fastest; tile = wave:
      //      (q, k2c) index = 4 wave + r/8, i0 = r%8
      {
        const int idx = 4 * wave + (col >> 3);
        const int q = idx >> 2, k2c = idx & 3, i0 = col & 7;
        const half8 a =
            *reinterpret_cast<const half8*>(&L3[(((hh * 8 + i0) * 8 + q) * 16 + 4 * cc + k2c) * 8]);
        floatx16 d = mfma(a, Wf_hi, zero);
        d = mfma(a, Wf_lo, d);
        // column -> (comp, k1); rows -> (q, k2c) index = 4 wave + i, i0 = 4hh + j
        const int comp = col >> 4, k1 = col & 15;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int id2 = 4 * wave + i;
          store4(&L4[(((comp * 16 + k1) * 8 + (id2 >> 2)) * 4 + (id2 & 3)) * 8 + 4 * hh], d[4 * i], d[4 * i + 1],
                 d[4 * i + 2], d[4 * i + 3]);
        }
      }
      __syncthreads();
      // ---- P4: axis 0 on lines (k1, q, k2c); tile T4 = 2 wave + tt: k1 = T4, q = r/4, k2c = r%4
#pragma unroll
      for (int tt = 0; tt < 2; ++tt) {
        const int k1 = 2 * wave + tt, q = col >> 2, k2c = col & 3;
        const half8 bop = *reinterpret_cast<const half8*>(&L4[(((hh * 16 + k1) * 8 + q) * 4 + k2c) * 8]);
        floatx16 d = mfma(Wf_hi, bop, zero);
        d = mfma(Wf_lo, bop, d);
        // rows: 4hh + j (re), 8 + 4hh + j (re), 16 + 4hh + j (im), 24 + 4hh + j (im)
        const int base = (cc * 2 + tt) * 8;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[base + j] = fmaf(d[j], d[j], fmaf(d[8 + j], d[8 + j], acc[base + j]));
          acc[base + 4 + j] = fmaf(d[4 + j], d[4 + j], fmaf(d[12 + j], d[12 + j], acc[base + 4 + j]));
        }
      }
      __syncthreads();
    }
  }
  // |X|^2 carried 8^-8 = 2^-24 from the four scaled stages
  double* out = partial + ((int64_t)grp * 2 + h) * 32768;
#pragma unroll
  for (int i = 0; i < CPL; ++i) out[i * NT + tid] = (double)acc[i] * 16777216.0;
}

hipError_t launch_fused8x4_mixed(int fmt, const void* src, int64_t T, int64_t tps, const float2* tw16,
                                 double* partial, int F, int n_slices, hipStream_t st) {
  const int groups = n_slices * F;
  const int xcd = (groups % 8 == 0) ? 1 : 0;
  const dim3 grid(groups * 2), block(f8m::NT);
  switch (fmt) {
    case 1:
      hipLaunchKernelGGL(fused8x4_mixed_kernel<1>, grid, block, 0, st, src, T, tps, tw16, partial, F, xcd);
      break;
    case 2:
      hipLaunchKernelGGL(fused8x4_mixed_kernel<2>, grid, block, 0, st, src, T, tps, tw16, partial, F, xcd);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace omni
