// Fused float32 correlator for the two-level 8x8-of-8x8 hierarchy (four axes of
// 8 antennas, padded to 16; M = 65536 Fourier cells per channel), gfx950.
//
// Work-group = (time slice, channel f, residue c of axis 0 mod 8), 256 threads.
// It owns the 8192 Fourier cells with kappa_0 in {c, c+8} and, for every time
// sample of its slice:
//   A  loads the channel's 4096 samples (coalesced) and folds axis 0:
//      X0[k] = sum_{i0} x[i0] w16^{(c + 8k) i0}, k in {0,1}  (the fold + 2-point
//      DFT of the residue-c outputs of the zero-padded length-16 DFT)
//   B  axis 3: half-line jobs (one residue mod 2 of the 16 outputs each),
//   C  axis 2: full pruned 16-point DFT per thread,
//   D  axis 1: two lines per thread, |X|^2 into 32 float32 registers that are
//      flushed into float64 registers every time_block samples.
// Every short transform is an 8-point radix-2 FFT of the 8 antennas, preceded
// for odd outputs by the twiddles w16^j (the zero-padded 16-point DFT split
// into its even and odd outputs, Sec. II.C "zero-padded FFT").  Twiddles come
// from the float64-generated table w16^q.  LDS: 48 KiB.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace omni {

namespace f8 {

constexpr int NT = 256;
constexpr int CPT = 32;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }
// multiply by w8 = (1 - i)/sqrt2 and by w8^3 = (-1 - i)/sqrt2 ; h = sqrt2/2
__device__ __forceinline__ float2 mul_w8(float2 a, float h) { return make_float2((a.x + a.y) * h, (a.y - a.x) * h); }
__device__ __forceinline__ float2 mul_w83(float2 a, float h) { return make_float2((a.y - a.x) * h, -(a.x + a.y) * h); }

// 8-point DFT, natural order in and out: X[k] = sum_j a[j] w8^{jk}.
__device__ __forceinline__ void fft8(float2 (&a)[8], float h) {
  // radix-2 decimation in time on the bit-reversed order 0 4 2 6 1 5 3 7
  float2 b0 = add(a[0], a[4]), b1 = sub(a[0], a[4]);
  float2 b2 = add(a[2], a[6]), b3 = sub(a[2], a[6]);
  float2 b4 = add(a[1], a[5]), b5 = sub(a[1], a[5]);
  float2 b6 = add(a[3], a[7]), b7 = sub(a[3], a[7]);
  float2 c0 = add(b0, b2), c2 = sub(b0, b2);
  float2 t3 = mul_mi(b3);
  float2 c1 = add(b1, t3), c3 = sub(b1, t3);
  float2 c4 = add(b4, b6), c6 = sub(b4, b6);
  float2 t7 = mul_mi(b7);
  float2 c5 = add(b5, t7), c7 = sub(b5, t7);
  a[0] = add(c0, c4);
  a[4] = sub(c0, c4);
  float2 t5 = mul_w8(c5, h);
  a[1] = add(c1, t5);
  a[5] = sub(c1, t5);
  float2 t6 = mul_mi(c6);
  a[2] = add(c2, t6);
  a[6] = sub(c2, t6);
  float2 t7b = mul_w83(c7, h);
  a[3] = add(c3, t7b);
  a[7] = sub(c3, t7b);
}

// a[j] *= w16^j (odd outputs of the zero-padded 16-point DFT).
__device__ __forceinline__ void twiddle16(float2 (&a)[8], const float2 (&w)[8], float h) {
  a[1] = cmul(a[1], w[1]);
  a[2] = mul_w8(a[2], h);
  a[3] = cmul(a[3], w[3]);
  a[4] = mul_mi(a[4]);
  a[5] = cmul(a[5], w[5]);
  a[6] = mul_w83(a[6], h);
  a[7] = cmul(a[7], w[7]);
}

// Two consecutive samples.
template <int FMT>
__device__ __forceinline__ void load2(const void* __restrict__ base, int64_t i, float2& s0, float2& s1);
template <>
__device__ __forceinline__ void load2<0>(const void* __restrict__ base, int64_t i, float2& s0, float2& s1) {
  const float4 v = *reinterpret_cast<const float4*>(reinterpret_cast<const float2*>(base) + i);
  s0 = make_float2(v.x, v.y);
  s1 = make_float2(v.z, v.w);
}
template <>
__device__ __forceinline__ void load2<1>(const void* __restrict__ base, int64_t i, float2& s0, float2& s1) {
  const char4 v = *reinterpret_cast<const char4*>(reinterpret_cast<const char2*>(base) + i);
  s0 = make_float2((float)v.x, (float)v.y);
  s1 = make_float2((float)v.z, (float)v.w);
}
template <>
__device__ __forceinline__ void load2<2>(const void* __restrict__ base, int64_t i, float2& s0, float2& s1) {
  const char2 v = *reinterpret_cast<const char2*>(reinterpret_cast<const int8_t*>(base) + i);
  const int8_t a = v.x, b = v.y;
  s0 = make_float2((float)(a >> 4), (float)((int8_t)(a << 4) >> 4));
  s1 = make_float2((float)(b >> 4), (float)((int8_t)(b << 4) >> 4));
}

}  // namespace f8

template <int FMT>
__global__ __launch_bounds__(f8::NT) void fused8x4_fp32_kernel(const void* __restrict__ src, int64_t T,
                                                               int64_t t_per_slice,
                                                               const float2* __restrict__ tw16,
                                                               double* __restrict__ partial, int F, int xcd_groups,
                                                               int time_block) {
  using namespace f8;
  __shared__ float2 B0[2 * 8 * 16 * 16];  // stage A output [k][i1][i2][i3], stage C output [k][i1][p2][p3]
  __shared__ float2 B1[2 * 8 * 8 * 16];   // stage B output [k][i1][i2][p3]
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  int grp, c;
  if (xcd_groups) {
    const int xcd = b & 7, j = b >> 3;
    grp = xcd + 8 * (j >> 3);
    c = j & 7;
  } else {
    grp = b >> 3;
    c = b & 7;
  }
  const int f = grp % F;
  const int s = grp / F;

  float2 w[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) w[q] = tw16[q];
  const float h = tw16[2].x;  // sqrt2 / 2
  float2 u[8];                // fold twiddles w16^{c p}
#pragma unroll
  for (int p = 0; p < 8; ++p) u[p] = tw16[(c * p) & 15];

  const int64_t t0 = (int64_t)s * t_per_slice;
  const int64_t t1 = min(T, t0 + t_per_slice);
  float acc32[CPT];
  double acc64[CPT];
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    acc32[i] = 0.f;
    acc64[i] = 0.0;
  }
  int blk = 0;

  // stage B mapping: line L = (k, i1, i2) = tid >> 1, half hb = tid & 1
  const int LB = tid >> 1, hb = tid & 1;
  // stage C mapping: line (k, i1, p3)
  const int p3c = tid & 15, i1c = (tid >> 4) & 7, kc = tid >> 7;

  for (int64_t t = t0; t < t1; ++t) {
    // ---- A: load 2 lines (q = 2 tid, 2 tid + 1 over (i1, i2, i3)) x 8 values of i0
    const int64_t tile = (t * F + f) * 4096;
    float2 x0[8], x1[8];
#pragma unroll
    for (int i0 = 0; i0 < 8; ++i0) load2<FMT>(src, tile + i0 * 512 + 2 * tid, x0[i0], x1[i0]);
    float2 X00, X01, X10, X11;  // [line][k]
    {
      float2 z0 = make_float2(0.f, 0.f), z1 = z0, y0 = z0, y1 = z0;
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        z0 = add(z0, cmul(x0[2 * l], u[2 * l]));
        z1 = add(z1, cmul(x0[2 * l + 1], u[2 * l + 1]));
        y0 = add(y0, cmul(x1[2 * l], u[2 * l]));
        y1 = add(y1, cmul(x1[2 * l + 1], u[2 * l + 1]));
      }
      X00 = add(z0, z1);
      X01 = sub(z0, z1);
      X10 = add(y0, y1);
      X11 = sub(y0, y1);
    }
    __syncthreads();  // previous sample's stage D has finished reading B0
    *reinterpret_cast<float4*>(&B0[2 * tid]) = make_float4(X00.x, X00.y, X10.x, X10.y);
    *reinterpret_cast<float4*>(&B0[512 + 2 * tid]) = make_float4(X01.x, X01.y, X11.x, X11.y);
    __syncthreads();

    // ---- B: axis 3 (contiguous), one half (residue hb mod 2) of line LB
    {
      float2 a[8];
#pragma unroll
      for (int j = 0; j < 8; j += 2) {
        const float4 v = *reinterpret_cast<const float4*>(&B0[LB * 8 + j]);
        a[j] = make_float2(v.x, v.y);
        a[j + 1] = make_float2(v.z, v.w);
      }
      if (hb) twiddle16(a, w, h);
      fft8(a, h);
#pragma unroll
      for (int j = 0; j < 8; j += 2)
        *reinterpret_cast<float4*>(&B1[LB * 16 + hb * 8 + j]) = make_float4(a[j].x, a[j].y, a[j + 1].x, a[j + 1].y);
    }
    __syncthreads();

    // ---- C: axis 2, full pruned 16-point DFT of line (kc, i1c, p3c)
    {
      float2 a[8], e[8];
#pragma unroll
      for (int i2 = 0; i2 < 8; ++i2) a[i2] = B1[((kc * 8 + i1c) * 8 + i2) * 16 + p3c];
#pragma unroll
      for (int j = 0; j < 8; ++j) e[j] = a[j];
      twiddle16(e, w, h);
      fft8(a, h);
      fft8(e, h);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        B0[((kc * 8 + i1c) * 16 + j) * 16 + p3c] = a[j];
        B0[((kc * 8 + i1c) * 16 + 8 + j) * 16 + p3c] = e[j];
      }
    }
    __syncthreads();

    // ---- D: axis 1 (last), lines l = tid and tid + 256 over (k, p2, p3); square and accumulate
#pragma unroll
    for (int ls = 0; ls < 2; ++ls) {
      const int l = tid + ls * NT;
      const int k = l >> 8, p2 = (l >> 4) & 15, p3 = l & 15;
      float2 a[8], e[8];
#pragma unroll
      for (int i1 = 0; i1 < 8; ++i1) a[i1] = B0[((k * 8 + i1) * 16 + p2) * 16 + p3];
#pragma unroll
      for (int j = 0; j < 8; ++j) e[j] = a[j];
      twiddle16(e, w, h);
      fft8(a, h);
      fft8(e, h);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        acc32[ls * 16 + j] = fmaf(a[j].x, a[j].x, fmaf(a[j].y, a[j].y, acc32[ls * 16 + j]));
        acc32[ls * 16 + 8 + j] = fmaf(e[j].x, e[j].x, fmaf(e[j].y, e[j].y, acc32[ls * 16 + 8 + j]));
      }
    }
    if (++blk == time_block) {
      blk = 0;
#pragma unroll
      for (int i = 0; i < CPT; ++i) {
        acc64[i] += (double)acc32[i];
        acc32[i] = 0.f;
      }
    }
  }
  // cell i of thread tid sits at i * 256 + tid
  double* out = partial + ((int64_t)grp * 8 + c) * 8192;
#pragma unroll
  for (int i = 0; i < CPT; ++i) out[i * NT + tid] = acc64[i] + (double)acc32[i];
}

hipError_t launch_fused8x4_fp32(int fmt, const void* src, int64_t T, int64_t tps, const float2* tw16, double* partial,
                                int F, int n_slices, int time_block, hipStream_t st) {
  const int groups = n_slices * F;
  const int xcd = (groups % 8 == 0) ? 1 : 0;
  const dim3 grid(groups * 8), block(f8::NT);
  switch (fmt) {
    case 0:
      hipLaunchKernelGGL(fused8x4_fp32_kernel<0>, grid, block, 0, st, src, T, tps, tw16, partial, F, xcd, time_block);
      break;
    case 1:
      hipLaunchKernelGGL(fused8x4_fp32_kernel<1>, grid, block, 0, st, src, T, tps, tw16, partial, F, xcd, time_block);
      break;
    case 2:
      hipLaunchKernelGGL(fused8x4_fp32_kernel<2>, grid, block, 0, st, src, T, tps, tw16, partial, F, xcd, time_block);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace omni
