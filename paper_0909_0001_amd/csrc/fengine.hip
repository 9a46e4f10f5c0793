// F-engine ahead of the correlator (Appendix A, steps 2-3): each antenna's
// real time series is cut into blocks of 2F samples, each block is Fourier
// transformed (bins k = 0 .. F-1, no window, the Nyquist bin dropped),
// multiplied by a complex per-antenna, per-channel gain (calibration and
// requantisation scale), rounded half to even and clipped to the 4- or 8-bit
// format, and written in the correlator's [t][k][n] layout (the corner turn:
// antenna-major streams in, channel-major hypercube input out).
//
// The per-block transform is a dense contraction, X = W x with W[k][j] =
// exp(-2 pi i j k / 2F), batched over antennas and blocks, so it runs on the
// matrix cores: one real-embedded product per block on
// v_mfma_f32_32x32x16_f16 with W on the A side (rows = Re and Im of 16 bins,
// so an output's two parts land in one lane) and 32 antennas' samples on the
// B side (columns), float16 operands (int8 samples are exact in float16; W is
// split into float16 hi + lo parts) and float32 accumulation.  A vector-ALU FFT
// of the same blocks would need about 20 ALU operations per sample and be
// ALU-bound at well under the HBM rate; the product needs about
// 4 x 2F flops a sample on the matrix cores, about level with the HBM time of
// the 1 + 0.5 (or 1) bytes each sample moves.
//
// Work-group: 256 threads, 4 waves; a wave owns 16 bins (output tile) of 64
// antennas (two 32-column tiles) for every block of its time range.  Waves
// split the F / 16 output tiles, the rest of the factor 4 goes to more antennas
// (F = 64: 64 antennas a work-group; F = 16: 256).  The W fragments and the
// lane's gains stay in registers and the W fragments in LDS for the whole time
// range; samples go straight from HBM to registers (16-byte loads, the next
// block's while the current one is transformed; each lane half reads alternate
// 16-byte pieces of the block, and the W fragments follow the same sample
// order).

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace omni {
namespace {

typedef _Float16 fe_half8 __attribute__((ext_vector_type(8)));
typedef _Float16 fe_half2 __attribute__((ext_vector_type(2)));
typedef float fe_floatx16 __attribute__((ext_vector_type(16)));

constexpr int kFeThreads = 256;

// Sample order of the B operand: K-step s (16 samples), lane half h, element e -> sample j of the block.
__device__ __forceinline__ int fe_sample(int s, int h, int e) { return 32 * (s >> 1) + 16 * h + 8 * (s & 1) + e; }

// Two signed bytes of `w` (bytes b, b + 1) as exact float16: (1024 + (x + 128)) - 1152.
__device__ __forceinline__ fe_half2 fe_bytes2(uint32_t x_flipped, uint32_t sel) {
  const uint32_t p = __builtin_amdgcn_perm(0u, x_flipped, sel) | 0x64006400u;
  const _Float16 b = (_Float16)1152.f;
  const fe_half2 bias = {b, b};
  return __builtin_bit_cast(fe_half2, p) - bias;
}

__device__ __forceinline__ void fe_unpack16(uint4 raw, fe_half8& a, fe_half8& b) {
  const uint32_t w[4] = {raw.x ^ 0x80808080u, raw.y ^ 0x80808080u, raw.z ^ 0x80808080u, raw.w ^ 0x80808080u};
  fe_half8 v[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const fe_half2 lo = fe_bytes2(w[2 * q + p], 0x0c010c00u);
      const fe_half2 hi = fe_bytes2(w[2 * q + p], 0x0c030c02u);
      v[q][4 * p + 0] = lo[0];
      v[q][4 * p + 1] = lo[1];
      v[q][4 * p + 2] = hi[0];
      v[q][4 * p + 3] = hi[1];
    }
  }
  a = v[0];
  b = v[1];
}

template <int F, bool CI8>
__global__ __launch_bounds__(kFeThreads) void fengine_kernel(const int8_t* __restrict__ raw, int64_t N, int64_t T,
                                                             int64_t t_per_chunk, const float2* __restrict__ gains,
                                                             uint8_t* __restrict__ out) {
  constexpr int KS = F / 8;          // K-steps of 16 samples (2F samples a block)
  constexpr int TILES = F / 16;      // output tiles of 16 bins
  constexpr int CG = 4 / TILES;      // column groups of 64 antennas per work-group
  constexpr int ANT = 64 * CG;       // antennas per work-group
  constexpr int L = 2 * F;           // samples per block
  __shared__ float2 tw[L];
  // W fragments of every output tile: [tile][K-step][hi, lo][lane] (16 bytes each, conflict-free reads)
  __shared__ fe_half8 wf[TILES * KS * 2 * 64];

  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int tile = w % TILES, cg = w / TILES;
  const int col = l & 31, h = l >> 5;
  const int64_t t0 = (int64_t)blockIdx.y * t_per_chunk;
  const int64_t t1 = min(T, t0 + t_per_chunk);

  // exp(-2 pi i q / 2F), q < 2F, from float64
  for (int q = tid; q < L; q += kFeThreads) {
    double s, c;
    sincospi(-2.0 * (double)q / (double)L, &s, &c);
    tw[q] = make_float2((float)c, (float)s);
  }
  __syncthreads();

  // W fragments (A operand): row col = 2 kk + comp (bin k = 16 tile + kk, comp 0 = Re, 1 = Im), samples of
  // K-step s in the B operand's order; hi and lo parts.  Waves of column group 0 build their tile's.
  if (cg == 0) {
    const int kk = col >> 1, comp = col & 1, k = 16 * tile + kk;
    for (int s = 0; s < KS; ++s) {
      fe_half8 vh, vl;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int j = fe_sample(s, h, e);
        const float2 z = tw[(j * k) % L];
        const float v = comp ? z.y : z.x;
        const _Float16 hi = (_Float16)v;
        vh[e] = hi;
        vl[e] = (_Float16)(v - (float)hi);
      }
      wf[((tile * KS + s) * 2 + 0) * 64 + l] = vh;
      wf[((tile * KS + s) * 2 + 1) * 64 + l] = vl;
    }
  }
  __syncthreads();
  const fe_half8* wt = wf + tile * KS * 2 * 64 + l;

  // antennas of the lane's two column tiles, and their gains for the lane's 8 bins (j4, p):
  // rows 8 j4 + 4 h + 2 p + {0, 1} -> bin kk = 4 j4 + 2 h + p
  const int64_t n_base = (int64_t)blockIdx.x * ANT + 64 * cg;
  int64_t n[2];
  bool ok[2];
  float2 g[2][8];
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    n[ct] = n_base + 32 * ct + col;
    ok[ct] = n[ct] < N;
#pragma unroll
    for (int j4 = 0; j4 < 4; ++j4)
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int k = 16 * tile + 4 * j4 + 2 * h + p;
        g[ct][2 * j4 + p] = ok[ct] ? gains[n[ct] * F + k] : make_float2(0.f, 0.f);
      }
  }

  const float qmax = CI8 ? 127.f : 7.f;
  // raw samples of the lane for one block: KS / 2 16-byte pieces per column tile; the next block's pieces are
  // loaded while the current block is transformed
  uint4 cur[2][KS / 2], nxt[2][KS / 2];
  auto load = [&](int64_t t, uint4 (&dst)[2][KS / 2]) {
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int sp = 0; sp < KS / 2; ++sp)
        dst[ct][sp] = ok[ct] && t < t1
                          ? *reinterpret_cast<const uint4*>(raw + n[ct] * (T * L) + t * L + 16 * h + 32 * sp)
                          : make_uint4(0u, 0u, 0u, 0u);
  };
  load(t0, cur);
  for (int64_t t = t0; t < t1; ++t) {
    load(t + 1, nxt);
    // one accumulation chain per column tile (hi and lo parts of W in turn)
    fe_floatx16 acc[2] = {};
#pragma unroll
    for (int sp = 0; sp < KS / 2; ++sp) {
      const fe_half8 wh0 = wt[(4 * sp + 0) * 64], wl0 = wt[(4 * sp + 1) * 64];
      const fe_half8 wh1 = wt[(4 * sp + 2) * 64], wl1 = wt[(4 * sp + 3) * 64];
      fe_half8 a[2], b[2];
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) fe_unpack16(cur[ct][sp], a[ct], b[ct]);
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_f16(wh0, a[ct], acc[ct], 0, 0, 0);
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_f16(wl0, a[ct], acc[ct], 0, 0, 0);
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
        acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_f16(wh1, b[ct], acc[ct], 0, 0, 0);
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
        acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_f16(wl1, b[ct], acc[ct], 0, 0, 0);
    }
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
#pragma unroll
      for (int sp = 0; sp < KS / 2; ++sp) cur[ct][sp] = nxt[ct][sp];
      if (!ok[ct]) continue;
#pragma unroll
      for (int j4 = 0; j4 < 4; ++j4) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const int i = 4 * j4 + 2 * p;
          const float xr = acc[ct][i], xi = acc[ct][i + 1];
          const float2 gg = g[ct][2 * j4 + p];
          const float yr = gg.x * xr - gg.y * xi;
          const float yi = gg.x * xi + gg.y * xr;
          const int cr = (int)fminf(qmax, fmaxf(-qmax, rintf(yr)));
          const int ci = (int)fminf(qmax, fmaxf(-qmax, rintf(yi)));
          const int k = 16 * tile + 4 * j4 + 2 * h + p;
          const int64_t o = (t * F + k) * N + n[ct];
          if (CI8) {
            const uint16_t v = (uint16_t)((uint8_t)(int8_t)cr | ((uint16_t)(uint8_t)(int8_t)ci << 8));
            *reinterpret_cast<uint16_t*>(out + 2 * o) = v;
          } else {
            out[o] = (uint8_t)(((cr & 0xF) << 4) | (ci & 0xF));
          }
        }
      }
    }
  }
}

template <int F, bool CI8>
hipError_t launch_fe(const int8_t* raw, int64_t N, int64_t T, const float2* gains, uint8_t* out, hipStream_t st) {
  constexpr int ANT = 64 * (4 / (F / 16));
  const int64_t groups = (N + ANT - 1) / ANT;
  // about 2048 work-groups (8 a CU), at least 4 blocks each
  int64_t chunks = std::max<int64_t>(1, std::min<int64_t>((2048 + groups - 1) / groups, (T + 3) / 4));
  const int64_t tpc = (T + chunks - 1) / chunks;
  chunks = (T + tpc - 1) / tpc;
  if (groups > INT32_MAX || chunks > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL((fengine_kernel<F, CI8>), dim3((unsigned)groups, (unsigned)chunks), dim3(kFeThreads), 0, st,
                     raw, N, T, tpc, gains, out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fengine(const void* raw, int64_t N, int64_t T, int F, const void* gains, bool ci8, void* out,
                          hipStream_t st) {
  const int8_t* r = static_cast<const int8_t*>(raw);
  const float2* g = static_cast<const float2*>(gains);
  uint8_t* o = static_cast<uint8_t*>(out);
  if (N < 1 || T < 1) return hipSuccess;
  switch (F) {
    case 16: return ci8 ? launch_fe<16, true>(r, N, T, g, o, st) : launch_fe<16, false>(r, N, T, g, o, st);
    case 32: return ci8 ? launch_fe<32, true>(r, N, T, g, o, st) : launch_fe<32, false>(r, N, T, g, o, st);
    case 64: return ci8 ? launch_fe<64, true>(r, N, T, g, o, st) : launch_fe<64, false>(r, N, T, g, o, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace omni
