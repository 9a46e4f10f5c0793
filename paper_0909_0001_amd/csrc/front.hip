// Front passes for arrays whose per-channel Fourier grid is too large for one
// fused kernel (gfx950, float32).
//
// One pass transforms a single axis k of every (time, channel) tile, reading
// [outer][n_k][inner] and writing [outer][m_k][inner] to HBM: the zero-padded
// DFT of Sec. II.A/II.C along that axis, X[kappa] = sum_{j<n} x_j w_m^{kappa j},
// kappa in [0, m), in natural frequency order.  It is done as the fold + short
// DFT of the residue classes rho (mod r): for each rho the thread forms
// z_j = sum_l x[j + l L] w_m^{rho (j + l L)} and a length-L DFT gives
// X[r q + rho].  Consecutive threads take consecutive inner indices, so every
// global load and store is coalesced.  After the front passes over the
// outermost axes, each outer Fourier index is an independent "channel" of the
// remaining axes for the fused kernel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <stdint.h>

#include "shortdft.hpp"

namespace omni {

namespace fr {

using sd::cadd;
using sd::cmul;

template <int FMT>
__device__ __forceinline__ float2 load(const void* __restrict__ base, int64_t i) {
  if (FMT == 0) return reinterpret_cast<const float2*>(base)[i];
  if (FMT == 1) {
    const char2 v = reinterpret_cast<const char2*>(base)[i];
    return make_float2((float)v.x, (float)v.y);
  }
  const int8_t v = reinterpret_cast<const int8_t*>(base)[i];
  return make_float2((float)(v >> 4), (float)((int8_t)(v << 4) >> 4));
}

// V samples at consecutive inner indices, the first at byte address q (ES bytes per sample)
template <int FMT, int V>
__device__ __forceinline__ void load_v(const char* __restrict__ q, float2 (&x)[V]) {
  if constexpr (V == 1) {
    x[0] = load<FMT>(q, 0);
  } else if constexpr (FMT == 2) {  // V packed 4-bit samples in one 2- or 4-byte word
    const uint32_t u = V == 4 ? *reinterpret_cast<const uint32_t*>(q) : (uint32_t)*reinterpret_cast<const uint16_t*>(q);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int8_t b = (int8_t)(u >> (8 * v));
      x[v] = make_float2((float)(b >> 4), (float)((int8_t)(b << 4) >> 4));
    }
  } else {  // FMT 1: V int8 pairs in 2 V bytes
    uint2 u;
    if constexpr (V == 4) {
      u = *reinterpret_cast<const uint2*>(q);
    } else {
      u.x = *reinterpret_cast<const uint32_t*>(q);
      u.y = 0;
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const uint32_t h = v < 2 ? u.x : u.y;
      const int s = 16 * (v & 1);
      x[v] = make_float2((float)(int8_t)(h >> s), (float)(int8_t)(h >> (s + 8)));
    }
  }
}

// bytes per sample of the formats load_v reads
template <int FMT>
constexpr int sample_bytes() {
  return FMT == 0 ? 8 : FMT == 1 ? 2 : 1;
}

}  // namespace fr

// Grid: x over (tile, outer, inner / V) flattened with inner fastest, y over residues.
// tiles = time samples x channels of this call; tile stride in the source is
// src_tile (elements), in the destination dst_tile.  Each thread transforms V
// consecutive inner indices, so that 1- and 2-byte samples are read as 4- or
// 8-byte words (V = 4) and the outputs leave as 32-byte runs.  R = m / L is
// the fold modulus, a compile-time constant so that all n loads of a thread
// are issued before the arithmetic that consumes them: n = L R / 2 inputs, one
// block of L per l < R / 2 (for R = 1, the first L / 2 of one block).
//
// H16: the output is float16, scaled by `scale`, in planar blocks: for every
// (tile, outer index, Fourier index) the inner run of real parts, then that of
// imaginary parts (the operand layout of the float16 matrix-core kernel).
//
// A launch covers tiles tile0 .. tile0 + total / (outer * inner_v) - 1; its item
// index is 32-bit (the launcher splits larger calls), and each item forms its
// two 64-bit base addresses once: rows and Fourier indices are offsets that are
// the same for every lane.
template <int FMT, int L, int V, int R, bool H16>
__global__ __launch_bounds__(256) void front_axis_kernel(const void* __restrict__ src, void* __restrict__ dst_,
                                                          const float2* __restrict__ twm, uint32_t total,
                                                          uint32_t outer, uint32_t inner_v, int64_t tile0,
                                                          int64_t inner, int64_t src_tile, int64_t dst_tile,
                                                          float scale) {
  using namespace fr;
  constexpr int M = L * R, N = M / 2;
  constexpr int NB = R >= 2 ? R / 2 : 1;
  const uint32_t per_tile = outer * inner_v;
  const int rho = blockIdx.y;
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    const uint32_t tl = idx / per_tile;
    const uint32_t rem = idx - tl * per_tile;
    const uint32_t o = rem / inner_v, in = (rem - o * inner_v) * V;
    const int64_t tile = tile0 + tl;
    const int64_t sbase = tile * src_tile + (int64_t)o * N * inner + in;
    // V inputs of row p; FMT 3 reads float16 planar blocks of (tile, o): N * inner real parts, then as many
    // imaginary parts (the H16 output of a previous front pass)
    const char* const sp = static_cast<const char*>(src) + (FMT == 3 ? 0 : sbase * sample_bytes<FMT>());
    const _Float16* const hp = static_cast<const _Float16*>(src) + (FMT == 3 ? 2 * (sbase - in) + in : 0);
    auto ld = [&](int p, float2(&xv)[V]) {
      if constexpr (FMT == 3) {
        const _Float16* h = hp + (int64_t)p * inner;
        const int64_t plane = (int64_t)N * inner;
#pragma unroll
        for (int v = 0; v < V; ++v) xv[v] = make_float2((float)h[v], (float)h[plane + v]);
      } else {
        load_v<FMT, V>(sp + (int64_t)p * inner * sample_bytes<FMT>(), xv);
      }
    };
    _Float16* const dh = static_cast<_Float16*>(dst_) + ((tile * outer + o) * M) * 2 * inner + in;
    float2* const dp = static_cast<float2*>(dst_) + tile * dst_tile + (int64_t)o * M * inner + in;
    auto store = [&](const float2(&zz)[V][L], int res) {
      if constexpr (H16) {
#pragma unroll
        for (int q = 0; q < L; ++q) {
          // planar block of (tile, o, kappa): 2 * inner halves
          _Float16* d = dh + (int64_t)(R * q + res) * 2 * inner;
          if constexpr (V == 2) {  // one 4-byte store per plane
            typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
            half2_t re, im;
            re[0] = (_Float16)(zz[0][q].x * scale);
            re[1] = (_Float16)(zz[1][q].x * scale);
            im[0] = (_Float16)(zz[0][q].y * scale);
            im[1] = (_Float16)(zz[1][q].y * scale);
            *reinterpret_cast<half2_t*>(d) = re;
            *reinterpret_cast<half2_t*>(d + inner) = im;
          } else {
#pragma unroll
            for (int v = 0; v < V; ++v) {
              d[v] = (_Float16)(zz[v][q].x * scale);
              d[inner + v] = (_Float16)(zz[v][q].y * scale);
            }
          }
        }
        return;
      }
#pragma unroll
      for (int q = 0; q < L; ++q) {
        float2* d = dp + (int64_t)(R * q + res) * inner;
        if constexpr (V == 4) {
          reinterpret_cast<float4*>(d)[0] = make_float4(zz[0][q].x, zz[0][q].y, zz[1][q].x, zz[1][q].y);
          reinterpret_cast<float4*>(d)[1] = make_float4(zz[2][q].x, zz[2][q].y, zz[3][q].x, zz[3][q].y);
        } else if constexpr (V == 2) {
          reinterpret_cast<float4*>(d)[0] = make_float4(zz[0][q].x, zz[0][q].y, zz[1][q].x, zz[1][q].y);
        } else {
          d[0] = zz[0][q];
        }
      }
    };
    if constexpr (R == 2) {
      // n = L: both residues use the same inputs, z_j = w_m^{rho j} x_j; one thread does both.  The inputs are
      // loaded again for the second residue (from the cache) rather than kept: holding them cost 4 V L registers
      // and a wave per SIMD of this memory-bound pass.
      float2 z[V][L];
#pragma unroll
      for (int j = 0; j < L; ++j) {
        float2 xv[V];
        ld(j, xv);
#pragma unroll
        for (int v = 0; v < V; ++v) z[v][j] = xv[v];
      }
#pragma unroll
      for (int v = 0; v < V; ++v) sd::dft<L>(z[v]);
      store(z, 0);
#pragma unroll
      for (int j = 0; j < L; ++j) {
        float2 xv[V];
        ld(j, xv);
        const float2 w = twm[j];  // w_m^j
#pragma unroll
        for (int v = 0; v < V; ++v) z[v][j] = j ? cmul(xv[v], w) : xv[v];
      }
#pragma unroll
      for (int v = 0; v < V; ++v) sd::dft<L>(z[v]);
      store(z, 1);
      continue;
    }
    float2 z[V][L];
#pragma unroll
    for (int blk = 0; blk < NB; ++blk) {
#pragma unroll
      for (int j = 0; j < L; ++j) {
        const int p = j + blk * L;
        if (p >= N) {
#pragma unroll
          for (int v = 0; v < V; ++v) z[v][j] = make_float2(0.f, 0.f);
          continue;
        }
        float2 x[V];
        ld(p, x);
        const float2 w = twm[(rho * p) & (M - 1)];  // w_m^{rho p}, uniform across the block
#pragma unroll
        for (int v = 0; v < V; ++v) z[v][j] = blk == 0 ? cmul(x[v], w) : cadd(z[v][j], cmul(x[v], w));
      }
    }
#pragma unroll
    for (int v = 0; v < V; ++v) sd::dft<L>(z[v]);
    store(z, rho);
  }
}

// Both front passes of a 16 x 16 outer level in one kernel, float16 planar
// output (for the three-level matrix-core kernel).  Work-group = (tile, block
// of RB = 32 consecutive rest indices), 256 threads: the 16 x 16 x RB raw
// samples are copied to LDS (one row of RB samples per thread); then for each
// half h of kappa_0 (kappa_0 = 2q + h): axis 0 (z_j = x_j w_32^{h j}, 16-point
// DFT, scaled by 1/16) into an LDS block of float16 [q][i1][r], then axis 1
// (the two residues of kappa_1 from the same 16 inputs, scaled by 1/16)
// straight to HBM.  The output is the one the two separate passes write,
// without their float16 intermediate in HBM: for (tile, kappa_0, kappa_1) the
// rest-many real parts, then the imaginary parts.
template <int FMT>
__global__ __launch_bounds__(256, 4) void front2_16x16_kernel(const void* __restrict__ src, _Float16* __restrict__ dst,
                                                               const float2* __restrict__ tw32, int64_t rest,
                                                               float scale) {
  using namespace fr;
  constexpr int RB = 32, SB = FMT == 1 ? 2 : 1;  // rest block; bytes per sample
  constexpr int ROW = RB * SB;                     // bytes of one (i0, i1) row in LDS
  __shared__ __attribute__((aligned(16))) uint8_t raw[256 * ROW];
  __shared__ __attribute__((aligned(16))) _Float16 mid[2][16 * 16 * RB];  // [re | im][q][i1][r]
  const int tid = threadIdx.x;
  const int64_t nrb = rest / RB;
  // consecutive work-groups go to the 8 XCDs in turn; remap so that the blocks of one XCD take consecutive
  // rest blocks, which share 128-byte lines of the raw rows (in that XCD's L2)
  int64_t b = blockIdx.x;
  if ((gridDim.x & 7) == 0) b = (b & 7) * (gridDim.x >> 3) + (b >> 3);
  const int64_t tile = b / nrb;
  const int64_t rb = b - tile * nrb;
  {
    const uint4* g = reinterpret_cast<const uint4*>(static_cast<const uint8_t*>(src) +
                                                    ((tile * 256 + tid) * rest + rb * RB) * SB);
    uint4* l = reinterpret_cast<uint4*>(raw + tid * ROW);
#pragma unroll
    for (int k = 0; k < ROW / 16; ++k) l[k] = g[k];
  }
  __syncthreads();
  auto sample = [&](int row, int r) -> float2 {
    if constexpr (FMT == 1) {
      const int8_t* b = reinterpret_cast<const int8_t*>(raw + row * ROW + 2 * r);
      return make_float2((float)b[0], (float)b[1]);
    } else {
      const int8_t b = (int8_t)raw[row * ROW + r];
      return make_float2((float)(b >> 4), (float)((int8_t)(b << 4) >> 4));
    }
  };
  _Float16* const out_tile = dst + tile * (32 * 32 * 2 * rest) + rb * RB;
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    // ---- axis 0 for kappa_0 = 2q + h: jobs (i1, r), r fastest
#pragma unroll 1
    for (int jj = 0; jj < 2; ++jj) {
      const int job = jj * 256 + tid, i1 = job / RB, r = job % RB;
      float2 z[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const float2 x = sample(j * 16 + i1, r);
        z[j] = (h && j) ? cmul(x, tw32[j]) : x;
      }
      sd::dft<16>(z);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        mid[0][(q * 16 + i1) * RB + r] = (_Float16)(z[q].x * 0.0625f);
        mid[1][(q * 16 + i1) * RB + r] = (_Float16)(z[q].y * 0.0625f);
      }
    }
    __syncthreads();
    // ---- axis 1 on (q, r): both residues of kappa_1 from the same 16 inputs (read twice), r fastest
#pragma unroll 1
    for (int jj = 0; jj < 2; ++jj) {
      const int job = jj * 256 + tid, q = job / RB, r = job % RB;
      _Float16* const o = out_tile + (int64_t)(2 * q + h) * 32 * 2 * rest + r;  // (kappa_0, kappa_1 = 0)
#pragma unroll 1
      for (int res = 0; res < 2; ++res) {
        float2 z[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const float2 y = make_float2((float)mid[0][(q * 16 + j) * RB + r], (float)mid[1][(q * 16 + j) * RB + r]);
          z[j] = (res && j) ? cmul(y, tw32[j]) : y;
        }
        sd::dft<16>(z);
#pragma unroll
        for (int k = 0; k < 16; ++k) {  // kappa_1 = 2k + res
          o[(2 * k + res) * 2 * rest] = (_Float16)(z[k].x * scale);
          o[(2 * k + res) * 2 * rest + rest] = (_Float16)(z[k].y * scale);
        }
      }
    }
    __syncthreads();  // the next half overwrites mid
  }
}

// Both front passes of a 16 x 16 outer level (fmt 1 ci8 or 2 ci4) into float16 planar blocks, each pass
// scaled by 1/16 (the second by `scale`); tw32: w_32^q.  rest % 32 == 0, 16-byte aligned rows.
hipError_t launch_front2_16x16(int fmt, const void* src, void* dst, const float2* tw32, int64_t tiles, int64_t rest,
                               float scale, hipStream_t st) {
  const int sb = fmt == 1 ? 2 : 1;
  if ((fmt != 1 && fmt != 2) || rest % 32 != 0 || (reinterpret_cast<uintptr_t>(src) & 15) != 0 ||
      ((rest * sb) & 15) != 0)
    return hipErrorInvalidValue;
  const int64_t blocks = tiles * (rest / 32);
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  if (fmt == 1)
    hipLaunchKernelGGL(front2_16x16_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, st, src,
                       static_cast<_Float16*>(dst), tw32, rest, scale);
  else
    hipLaunchKernelGGL(front2_16x16_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, st, src,
                       static_cast<_Float16*>(dst), tw32, rest, scale);
  return hipGetLastError();
}

// fmt: 0 float32 complex, 1 ci8, 2 ci4, 3 float16 planar blocks (the H16 output of a front pass).
// half16: float16 planar output scaled by `scale` (see H16 above); else float32 complex.
hipError_t launch_front_axis(int fmt, const void* src, void* dst, const float2* twm, int64_t tiles, int64_t outer,
                             int n, int m, int r, int64_t inner, int64_t src_tile, int64_t dst_tile, hipStream_t st,
                             bool half16, float scale) {
  const int L = m / r;
  if (m != 2 * n || L * r != m) return hipErrorInvalidValue;
  // packed integer samples: four inner indices per thread when the word loads stay aligned
  const int V = (fmt != 0 && L <= 16 && inner % 2 == 0 && src_tile % 2 == 0 &&
                 (reinterpret_cast<uintptr_t>(src) & 3) == 0)
                    ? 2
                    : 1;  // fmt 3 (float16 planar) reads its halves one by one, two inner indices per thread
  // items of one tile; a launch takes as many whole tiles as keep its item index below 2^31
  const int64_t per_tile = outer * (inner / V);
  if (tiles < 0 || per_tile <= 0 || per_tile > INT32_MAX) return tiles == 0 ? hipSuccess : hipErrorInvalidValue;
  const int64_t tiles_per_launch = INT32_MAX / per_tile;
  // r = 2: one thread computes both residue classes from the same inputs
  const dim3 block(256);
#define OMNI_FRONT(F_, L_, V_, R_)                                                                               \
  do {                                                                                                            \
    for (int64_t t0 = 0; t0 < tiles; t0 += tiles_per_launch) {                                                    \
      const int64_t total = std::min(tiles_per_launch, tiles - t0) * per_tile;                                    \
      const dim3 grid((unsigned)std::min<int64_t>((total + 255) / 256, 65536), (unsigned)(r == 2 ? 1 : r));      \
      if (half16)                                                                                                 \
        hipLaunchKernelGGL((front_axis_kernel<F_, L_, V_, R_, true>), grid, block, 0, st, src, dst, twm,          \
                           (uint32_t)total, (uint32_t)outer, (uint32_t)(inner / V), t0, inner, src_tile,          \
                           dst_tile, scale);                                                                      \
      else                                                                                                        \
        hipLaunchKernelGGL((front_axis_kernel<F_, L_, V_, R_, false>), grid, block, 0, st, src, dst, twm,         \
                           (uint32_t)total, (uint32_t)outer, (uint32_t)(inner / V), t0, inner, src_tile,          \
                           dst_tile, scale);                                                                      \
    }                                                                                                             \
  } while (0)
  // the planner's fold moduli: L = 16 for m >= 16 (r = m / 16), else r = 1 and L = m
#define OMNI_FRONT_LR(F_, V_)                              \
  if (r == 1 && L == 2) OMNI_FRONT(F_, 2, V_, 1);          \
  else if (r == 1 && L == 4) OMNI_FRONT(F_, 4, V_, 1);     \
  else if (r == 1 && L == 8) OMNI_FRONT(F_, 8, V_, 1);     \
  else if (r == 1 && L == 16) OMNI_FRONT(F_, 16, V_, 1);   \
  else if (r == 2 && L == 16) OMNI_FRONT(F_, 16, V_, 2);   \
  else if (r == 4 && L == 16) OMNI_FRONT(F_, 16, V_, 4);   \
  else return hipErrorInvalidValue;
  if (fmt == 0) {
    OMNI_FRONT_LR(0, 1)
  } else if (fmt == 1 && V == 2) {
    OMNI_FRONT_LR(1, 2)
  } else if (fmt == 1) {
    OMNI_FRONT_LR(1, 1)
  } else if (fmt == 3 && V == 2) {
    OMNI_FRONT_LR(3, 2)
  } else if (fmt == 3) {
    OMNI_FRONT_LR(3, 1)
  } else if (fmt == 2 && V == 2) {
    OMNI_FRONT_LR(2, 2)
  } else if (fmt == 2) {
    OMNI_FRONT_LR(2, 1)
  } else {
    return hipErrorInvalidValue;
  }
#undef OMNI_FRONT_LR
#undef OMNI_FRONT
  return hipGetLastError();
}

}  // namespace omni
