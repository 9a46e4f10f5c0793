// Short radix-2 DFTs with compile-time twiddles, shared by the float32 kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

namespace omni {
namespace sd {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// w_32^q = exp(-2 pi i q / 32), q < 16, as float32 constants: cos from the
// first octant table (correctly rounded), sin by symmetry.
constexpr float kCos32[9] = {0x1p+0f,         0x1.f6297cp-1f, 0x1.d906bcp-1f, 0x1.a9b662p-1f, 0x1.6a09e6p-1f,
                             0x1.1c73b4p-1f, 0x1.87de2ap-2f, 0x1.8f8b84p-3f, 0.0f};
constexpr float cos32(int q) { return q <= 8 ? kCos32[q] : -kCos32[16 - q]; }
constexpr float msin32(int q) { return q <= 8 ? -kCos32[8 - q] : -kCos32[q - 8]; }

// v * w_32^Q with Q a compile-time constant (Q = 0 and Q = 8 (-i) cost nothing)
template <int Q>
__device__ __forceinline__ float2 rot32(float2 v) {
  if constexpr (Q == 0) return v;
  if constexpr (Q == 8) return make_float2(v.y, -v.x);
  constexpr float c = cos32(Q), sn = msin32(Q);
  return make_float2(fmaf(v.x, c, -v.y * sn), fmaf(v.x, sn, v.y * c));
}

template <int L, int S, int K, int J>
__device__ __forceinline__ void butterfly(float2 (&z)[L]) {
  const float2 v = rot32<J * (32 / (2 * S))>(z[K + J + S]);
  const float2 u = z[K + J];
  z[K + J] = cadd(u, v);
  z[K + J + S] = csub(u, v);
}

template <int L, int S, int K, int... J>
__device__ __forceinline__ void butterflies(float2 (&z)[L], std::integer_sequence<int, J...>) {
  (butterfly<L, S, K, J>(z), ...);
}

template <int L, int S, int... K>
__device__ __forceinline__ void stage(float2 (&z)[L], std::integer_sequence<int, K...>) {
  (butterflies<L, S, K * 2 * S>(z, std::make_integer_sequence<int, S>{}), ...);
}

// Radix-2 DIT DFT of length L <= 32 (power of two), natural order, compile-time twiddles.
template <int L>
__device__ __forceinline__ void dft(float2 (&z)[L]) {
#pragma unroll
  for (int i = 0; i < L; ++i) {
    int j = 0;
#pragma unroll
    for (int b = 1, rb = L >> 1; b < L; b <<= 1, rb >>= 1)
      if (i & b) j |= rb;
    if (j > i) {
      const float2 t = z[i];
      z[i] = z[j];
      z[j] = t;
    }
  }
  if constexpr (L >= 2) stage<L, 1>(z, std::make_integer_sequence<int, L / 2>{});
  if constexpr (L >= 4) stage<L, 2>(z, std::make_integer_sequence<int, L / 4>{});
  if constexpr (L >= 8) stage<L, 4>(z, std::make_integer_sequence<int, L / 8>{});
  if constexpr (L >= 16) stage<L, 8>(z, std::make_integer_sequence<int, L / 16>{});
  if constexpr (L >= 32) stage<L, 16>(z, std::make_integer_sequence<int, L / 32>{});
}

}  // namespace sd
}  // namespace omni
