// Direct N^2 correlator: the pairwise product x_a conj(x_b) of every antenna
// pair, summed over time and binned by index difference Delta = idx(a) - idx(b)
// (the definition of the visibility hypercube, Sec. II.D, Eq. ProofEq2, and the
// generic correlator whose N^2 cost the paper's method replaces, Sec. I).  It
// is the comparison baseline for the FFT forms on the same device; its result
// is exact (integer products and sums) until the final conversion to float.
//
// Integer samples only (ci8, ci4).  Per channel, C = sum_t x_t x_t^H is a
// Hermitian N x N product with the time samples as the contracted axis.  Each
// antenna's samples stay interleaved, u_a = (xr_a(t), xi_a(t))_t, and with
// w_b = (~xi_b(t), xr_b(t))_t (~x = -x - 1: no int8 negation, which -128 lacks)
//     Re C[a,b] = u_a . u_b,    Im C[a,b] = u_a . w_b + sum_t xr_a(t),
// two int8 matrix-core products (v_mfma_i32_32x32x32_i8, int32 sums).
//
// Work-group = (block pair I <= J of 128 consecutive antennas, channel), 8
// waves of 64 x 32 pairs.  Each step stages 32 time samples of both blocks in
// LDS, one row of 64 bytes (32 interleaved (re, im) pairs, padded to 80:
// conflict-free 16-byte reads) per antenna, in two buffers: while one step's
// matrix products read one buffer, the next step is written into the other and
// the step after is loaded into registers (one barrier per step).  After the
// last step every pair (a in I, b in J, a <= b) adds its sums into LDS bins
// covering the box of Delta values the two blocks can form (64-bit integer LDS
// atomics), and the box is added into the channel's int64 half-sum G (global
// 64-bit atomics, one per nonzero bin).  Pairs a > b are the conjugates of
// pairs a < b at -Delta, so the finalize step forms
//     V[Delta] = G[Delta] + conj G[-Delta]  (Delta != 0),   V[0] = G[0].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "direct.hpp"

namespace omni {
namespace dc {

constexpr int NT = 512;     // 8 waves, each a 64 x 32 block of the 128 x 128 pair tile; two work-groups per CU
constexpr int KS = 32;      // time samples per step (two matrix-core products of contracted length 32 bytes)
constexpr int QS = KS / 32; // quads of 4 samples per thread and block per step
constexpr int RS = 2 * KS + 16; // LDS bytes per antenna row (KS interleaved samples, padded: conflict-free
                                // 16-byte reads)
// LDS row of antenna a of a block: (a mod 4) 36 + a / 4.  A staging store (antennas 4 ag + j of lanes
// ag = 0..31) then covers consecutive rows (2-way bank conflicts instead of 8-way for rows 4 apart), and the
// 16 rows an operand read serves at once stay on distinct banks (row mod 16 distinct).
constexpr int NROWS = 3 * 36 + kDirectTile / 4;
__device__ __forceinline__ int lds_row(int a) { return (a & 3) * 36 + (a >> 2); }
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

__device__ __forceinline__ v16i mfma(v4i a, v4i b, v16i c) {
  return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

// 4 consecutive antennas of one sample, raw: ci8 (re, im) byte pairs in 8 bytes, ci4 one byte each in .x
template <int FMT>
__device__ __forceinline__ uint2 load_raw4(const uint8_t* p) {
  if constexpr (FMT == 1) return *reinterpret_cast<const uint2*>(p);
  return make_uint2(*reinterpret_cast<const uint32_t*>(p), 0u);
}

// antenna j of a raw word -> its (re, im) int8 pair in the low 16 bits (re in the low byte)
template <int FMT>
__device__ __forceinline__ uint32_t pair_of(uint2 raw, int j) {
  if constexpr (FMT == 1) {
    return ((j < 2 ? raw.x : raw.y) >> (16 * (j & 1))) & 0xffffu;
  } else {  // ci4: re = high nibble, im = low nibble, two's complement
    const int b = (int)(int8_t)(raw.x >> (8 * j));
    return (uint32_t)((b >> 4) & 0xff) | ((uint32_t)(((int)(int8_t)(b << 4) >> 4) & 0xff) << 8);
  }
}

// (re, im) byte pairs -> (~im, re) byte pairs, for each pair of a 32-bit word
__device__ __forceinline__ int swap_not(int u) {
  const uint32_t v = (uint32_t)u;
  return (int)((((v >> 8) & 0x00ff00ffu) | ((v << 8) & 0xff00ff00u)) ^ 0x00ff00ffu);
}

template <int FMT>
__global__ __launch_bounds__(NT) void direct_tile_kernel(const uint8_t* __restrict__ src, int64_t T, int64_t N,
                                                        int F, const int32_t* __restrict__ pairs,
                                                        const int32_t* __restrict__ blk, DirectGeom g,
                                                        unsigned long long* __restrict__ G) {
  constexpr int SB = FMT == 1 ? 2 : 1;  // bytes per sample
  // two buffers of the staging planes of blocks I and J ([antenna][interleaved samples]): step s is read from
  // buffer s mod 2 while step s + 1 is written into the other
  __shared__ __attribute__((aligned(16))) uint8_t pl[2][2][NROWS * RS];
  __shared__ unsigned long long bins[kDirectMaxBins][2];
  __shared__ int alpha[kDirectTile], beta[kDirectTile];
  __shared__ int srow[kDirectTile];  // sum_t xr_a(t) over this launch, a in block I
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int f = blockIdx.y;
  const int I = pairs[2 * blockIdx.x], J = pairs[2 * blockIdx.x + 1];
  const int64_t aI = (int64_t)I * kDirectTile, aJ = (int64_t)J * kDirectTile;

  // ---- the Delta box of this block pair: Delta_k = c_k(a) - c_k(b) in [minI - maxJ, maxI - minJ]
  int size[kDirectMaxD], stride[kDirectMaxD];
  int nb = 1;
  for (int k = g.d - 1; k >= 0; --k) {
    const int* bi = blk + ((int64_t)I * kDirectMaxD + k) * 2;
    const int* bj = blk + ((int64_t)J * kDirectMaxD + k) * 2;
    size[k] = (bi[1] - bi[0]) + (bj[1] - bj[0]) + 1;
    stride[k] = nb;
    nb *= size[k];
  }
  if (nb > kDirectMaxBins) return;  // the planner never launches such a pair
  // bin(a, b) = alpha[a - aI] + beta[b - aJ], alpha = sum_k (c_k(a) - minI_k) stride_k,
  // beta = sum_k (maxJ_k - c_k(b)) stride_k
  if (tid < 2 * kDirectTile) {
    const bool isA = tid < kDirectTile;
    const int r = isA ? tid : tid - kDirectTile;
    int64_t a = (isA ? aI : aJ) + r;
    const int B = isA ? I : J;
    int acc = 0;
    for (int k = g.d - 1; k >= 0; --k) {
      const int c = (int)(a % g.n[k]);
      a /= g.n[k];
      const int* bb = blk + ((int64_t)B * kDirectMaxD + k) * 2;
      acc += (isA ? c - bb[0] : bb[1] - c) * stride[k];
    }
    (isA ? alpha : beta)[r] = acc;
  }
  for (int q = tid; q < nb; q += NT) bins[q][0] = bins[q][1] = 0ull;
  if (tid < kDirectTile) srow[tid] = 0;

  // ---- staging items: threads 0..255 stage block I, 256..511 block J; samples 4 tq .. 4 tq + 3 of the
  // step (tq = (tid mod 256) / 32 + 8 u, u < QS), antennas 4 ag .. 4 ag + 3 of the block
  const int half = (tid >> 8) & 1, tg = (tid & 255) >> 5, ag = tid & 31;
  const int64_t row_stride = (int64_t)F * N;  // samples between consecutive times
  const uint8_t* const pX = src + ((int64_t)f * N + (half ? aJ : aI) + 4 * ag) * SB;
  uint2 raw[QS][4];
  int sre[4] = {0, 0, 0, 0};  // block I stagers: sum of the real parts of antennas 4 ag + j
  auto load = [&](int64_t t0) {
#pragma unroll
    for (int u = 0; u < QS; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t t = t0 + 4 * (tg + 8 * u) + s;
        raw[u][s] = t < T ? load_raw4<FMT>(pX + t * row_stride * SB) : make_uint2(0u, 0u);
      }
  };

  constexpr int WJ = 1;  // 32-column blocks per wave
  constexpr int IW = 2;
  v16i cre[IW][WJ], cim[IW][WJ];
#pragma unroll
  for (int i = 0; i < IW; ++i)
#pragma unroll
    for (int j = 0; j < WJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) cre[i][j][r] = cim[i][j][r] = 0;

  const int mw = (w & 1) * 64, nw = (w >> 1) * 32;
  const int orow = lane & 31, ok = 16 * (lane >> 5);
  auto stage = [&](int buf) {
#pragma unroll
    for (int u = 0; u < QS; ++u)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        uint32_t p[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          p[s] = pair_of<FMT>(raw[u][s], j);
          if (half == 0) sre[j] += (int)(int8_t)(p[s] & 0xffu);
        }
        const int o = lds_row(4 * ag + j) * RS + 8 * (tg + 8 * u);
        *reinterpret_cast<uint2*>(&pl[buf][half][o]) = make_uint2(p[0] | (p[1] << 16), p[2] | (p[3] << 16));
      }
  };
  // one barrier per step: step s + 1 is staged (and step s + 2 loaded) while step s's products run
  load(0);
  stage(0);
  if (KS < T) load(KS);
  __syncthreads();
  int cur = 0;
  for (int64_t t0 = 0; t0 < T; t0 += KS) {
    if (t0 + KS < T) {
      stage(cur ^ 1);
      if (t0 + 2 * KS < T) load(t0 + 2 * KS);
    }
    const uint8_t(*const P)[NROWS * RS] = pl[cur];
#pragma unroll
    for (int kk = 0; kk < 2 * KS / 32; ++kk) {
      v4i ua[IW], ub[WJ], wb[WJ];
#pragma unroll
      for (int i = 0; i < IW; ++i)
        ua[i] = *reinterpret_cast<const v4i*>(&P[0][lds_row(mw + 32 * i + orow) * RS + 32 * kk + ok]);
#pragma unroll
      for (int j = 0; j < WJ; ++j) {
        ub[j] = *reinterpret_cast<const v4i*>(&P[1][lds_row(nw + 32 * j + orow) * RS + 32 * kk + ok]);
#pragma unroll
        for (int e = 0; e < 4; ++e) wb[j][e] = swap_not(ub[j][e]);
      }
#pragma unroll
      for (int i = 0; i < IW; ++i)
#pragma unroll
        for (int j = 0; j < WJ; ++j) {
          cre[i][j] = mfma(ua[i], ub[j], cre[i][j]);
          cim[i][j] = mfma(ua[i], wb[j], cim[i][j]);
        }
    }
    __syncthreads();
    cur ^= 1;
  }
  if (half == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) atomicAdd(&srow[4 * ag + j], sre[j]);
  }
  __syncthreads();

  // ---- bin: accumulator r of lane l holds pair (row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32)
#pragma unroll
  for (int i = 0; i < IW; ++i)
#pragma unroll
    for (int j = 0; j < WJ; ++j) {
      const int n = nw + 32 * j + (lane & 31);
      const int bn = beta[n];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = mw + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (I == J && m > n) continue;  // a > b: the conjugate of (b, a)
        const int q = alpha[m] + bn;
        const long long re = (long long)cre[i][j][r];
        const long long im = (long long)cim[i][j][r] + (long long)srow[m];
        if (re) atomicAdd(&bins[q][0], (unsigned long long)re);
        if (im) atomicAdd(&bins[q][1], (unsigned long long)im);
      }
    }
  __syncthreads();

  // ---- box -> the channel's half-sum G (centred layout of the visibility hypercube)
  unsigned long long* const Gf = G + (int64_t)f * g.n_out * 2;
  for (int q = tid; q < nb; q += NT) {
    const unsigned long long re = bins[q][0], im = bins[q][1];
    if (!re && !im) continue;
    int rem = q;
    int64_t gi = 0;
    for (int k = g.d - 1; k >= 0; --k) {
      const int c = rem % size[k];
      rem /= size[k];
      const int* bi = blk + ((int64_t)I * kDirectMaxD + k) * 2;
      const int* bj = blk + ((int64_t)J * kDirectMaxD + k) * 2;
      const int delta = bi[0] - bj[1] + c;
      gi += (int64_t)(delta + g.n[k] - 1) * g.gstride[k];
    }
    if (re) atomicAdd(&Gf[2 * gi], re);
    if (im) atomicAdd(&Gf[2 * gi + 1], im);
  }
}

// V[Delta] = G[Delta] + conj G[-Delta] (Delta != 0), V[0] = G[0]; the centred layout is symmetric, so
// -Delta is the mirrored linear index.
__global__ void direct_finalize_kernel(const long long* __restrict__ G, float2* __restrict__ vis, int64_t n_out,
                                       int64_t total) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = i / n_out, k = i - f * n_out, km = n_out - 1 - k;
    const long long* gf = G + f * n_out * 2;
    long long re = gf[2 * k], im = gf[2 * k + 1];
    if (km != k) {
      re += gf[2 * km];
      im -= gf[2 * km + 1];
    }
    vis[i] = make_float2((float)re, (float)im);
  }
}

__global__ void direct_zero_kernel(unsigned long long* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// Block boxes and block pairs of the no-allocation entry point, built on the device: blk[B][k] = (min, max)
// of axis k's index over the kDirectTile consecutive antennas of block B; pairs = every (I, J), I <= J, in the
// order I-major (the same list the planner builds on the host).
__global__ void direct_setup_kernel(DirectGeom g, int64_t nbk, int32_t* __restrict__ blk, int32_t* __restrict__ pairs) {
  const int64_t n_pairs = nbk * (nbk + 1) / 2;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nbk + n_pairs;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < nbk) {
      int lo[kDirectMaxD], hi[kDirectMaxD];
      for (int r = 0; r < kDirectTile; ++r) {
        int64_t a = i * kDirectTile + r;
        for (int k = g.d - 1; k >= 0; --k) {
          const int c = (int)(a % g.n[k]);
          a /= g.n[k];
          lo[k] = r == 0 ? c : min(lo[k], c);
          hi[k] = r == 0 ? c : max(hi[k], c);
        }
      }
      for (int k = 0; k < kDirectMaxD; ++k) {
        blk[(i * kDirectMaxD + k) * 2] = k < g.d ? lo[k] : 0;
        blk[(i * kDirectMaxD + k) * 2 + 1] = k < g.d ? hi[k] : 0;
      }
    } else {
      // pair q -> (I, J): the rows before row I hold S(I) = I nbk - I (I - 1) / 2 pairs, and
      // q = S(I) + (J - I); I is the largest row with S(I) <= q (a float64 root, then corrected)
      const int64_t q = i - nbk;
      auto S = [&](int64_t r) { return r * nbk - r * (r - 1) / 2; };
      const double b = 2.0 * (double)nbk + 1.0;
      int64_t I = (int64_t)((b - sqrt(b * b - 8.0 * (double)q)) / 2.0);
      I = max<int64_t>(0, min<int64_t>(I, nbk - 1));
      while (I > 0 && S(I) > q) --I;
      while (I + 1 < nbk && S(I + 1) <= q) ++I;
      pairs[2 * q] = (int32_t)I;
      pairs[2 * q + 1] = (int32_t)(I + (q - S(I)));
    }
  }
}

}  // namespace dc

// ---------------------------------------------------------------------------
// Fixed device scratch of the no-allocation entry point (omni_direct_correlate_noalloc): the int64 half-sums,
// the block pairs and the block boxes live in this array instead of buffers the library allocates.  Every
// call on a device shares that device's copy, which keeps the last call's contents; calls that overlap on
// one device race.  Host code uses the address resolved per device by direct_noalloc_scratch, never the
// array's name.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

size_t direct_noalloc_capacity() { return kNoAllocScratchBytes; }

// The device address of `scratch` on the current device, resolved once per device (the first call on a
// device, with that device current).  Returns hipSuccess and sets *ptr, or the HIP error of the lookup.
hipError_t direct_noalloc_scratch(void** ptr) {
  constexpr int kMaxDevices = 64;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t launch_direct_setup(const DirectGeom& g, int64_t nbk, int32_t* blk, int32_t* pairs, hipStream_t st) {
  const int64_t items = nbk + nbk * (nbk + 1) / 2;
  if (items <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((items + 255) / 256, 4096);
  dc::direct_setup_kernel<<<(unsigned)blocks, 256, 0, st>>>(g, nbk, blk, pairs);
  return hipGetLastError();
}

hipError_t launch_direct_zero(unsigned long long* G, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  dc::direct_zero_kernel<<<(unsigned)blocks, 256, 0, st>>>(G, n);
  return hipGetLastError();
}

hipError_t launch_direct_tiles(int fmt, const void* src, int64_t T, int64_t N, int F, const int32_t* pairs,
                               int64_t n_pairs, const int32_t* blk, const DirectGeom& g, unsigned long long* G,
                               hipStream_t st) {
  if (T <= 0) return hipSuccess;
  if (T > kDirectMaxT || N % kDirectTile != 0 || n_pairs <= 0 || n_pairs * dc::NT >= (int64_t(1) << 32) || F <= 0 || F > 65535 ||
      g.d < 1 || g.d > kDirectMaxD)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)n_pairs, (unsigned)F);
  if (fmt == 1)
    dc::direct_tile_kernel<1><<<grid, dc::NT, 0, st>>>(static_cast<const uint8_t*>(src), T, N, F, pairs, blk, g, G);
  else if (fmt == 2)
    dc::direct_tile_kernel<2><<<grid, dc::NT, 0, st>>>(static_cast<const uint8_t*>(src), T, N, F, pairs, blk, g, G);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_direct_finalize(const unsigned long long* G, void* vis, int64_t n_out, int F, hipStream_t st) {
  const int64_t total = n_out * F;
  if (total <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
  dc::direct_finalize_kernel<<<(unsigned)blocks, 256, 0, st>>>(reinterpret_cast<const long long*>(G),
                                                              static_cast<float2*>(vis), n_out, total);
  return hipGetLastError();
}

}  // namespace omni
