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
// matrix cores, and in integers: the samples are int8 already, so they are the
// B operand of v_mfma_i32_32x32x32_i8 exactly as they sit in memory (no decode
// at all), and W is split into three int8 parts,
//   W ~= (h + (m + l / 254) / 254) / 127,  h = rint(127 W), m, l in [-127, 127],
// each part's products summed exactly in int32 (|sum| <= 127 * 128 * 2F).  The
// parts are combined once per output, X * 127 * 254^2 = 254^2 acc_h +
// (254 acc_m + acc_l), with one float32 rounding; the split's own error is at
// most 0.5 / (127 * 254^2) ~= 6e-8 per coefficient.  A wave's A fragments (W
// rows = Re and Im of 16 bins, so an output's two parts land in one lane) stay
// in registers for the whole time range.  An int8 product does the work of two
// float16 ones per instruction, so the three parts cost 3/4 of the matrix-core
// time of a float16 hi + lo split, and the samples skip the int8 -> float16
// conversion that a float16 product needs (about 1.75 vector instructions a
// sample, done once per wave, so four times per sample).
//
// Rounding and clipping use the float32 "magic number" form: adding
// 1.5 * 2^23 rounds a value below 2^22 in magnitude to an integer, ties to
// even, and leaves that integer in the low mantissa bits; the clip to
// [-qmax, qmax] is a median of three in the same shifted domain (rounding is
// monotone, so clipping after it is the same as clipping the rounded value).
// The low 4 or 8 bits of the result are the code.  A ci4 byte is then one
// shift-and-add of the two parts' bits (the imaginary part's magic offset by
// 8 so that nothing borrows), fixed up four bytes at a time before the store.
//
// Work-group: 256 threads, 4 waves; a wave owns 16 bins (output tile) of 64
// antennas (two 32-column tiles, done one after the other) for every block of
// its time range.  Waves split the F / 16 output tiles, the rest of the factor
// 4 goes to more antennas (F = 64: 64 antennas a work-group; F = 16: 256).
// A work-group's samples of a block (64 to 256 antennas, 8 KB) travel once
// from HBM (16-byte loads, eight consecutive threads covering 128 contiguous
// bytes, the next block's while the current one is transformed) into a
// double-buffered LDS array laid out [16-byte chunk][antenna] with a pad that
// keeps both the writes and the B-fragment reads free of bank conflicts; the
// waves' output tiles all read it there.  Antennas past N read antenna N - 1,
// whose columns are never stored.  Codes go through a per-wave LDS tile of 16 bins x 64
// antennas so that each lane stores 16 contiguous bytes (rows of 64 antennas,
// 64 or 128 bytes) when N is a multiple of 16 (ci4) or 8 (ci8) and the output
// is 16-byte aligned; otherwise each lane stores its codes one by one.

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace omni {
namespace {

typedef int fe_int4 __attribute__((ext_vector_type(4)));
typedef int fe_int16 __attribute__((ext_vector_type(16)));

constexpr int kFeThreads = 256;
constexpr int kFeColTiles = 2;                   // 32-antenna column tiles per wave
constexpr float kFeMagic = 12582912.0f;          // 1.5 * 2^23
constexpr float kFeScale = 1.0f / 8193532.0f;    // 1 / (127 * 254^2)

// Ordering barrier for a wave reading LDS that other lanes of the same wave wrote (the LDS executes one
// wave's accesses in order; this keeps the compiler from moving them across).
__device__ __forceinline__ void fe_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Bit pattern of (magic + bias) + rint(v) clipped to [-qmax, qmax]: its low bits are bias plus the code, in
// two's complement (bias 0 or 8; magic + bias is even, so ties still round to even).
template <int BIAS>
__device__ __forceinline__ uint32_t fe_code(float v, float qmax) {
  constexpr float m = kFeMagic + (float)BIAS;
  return __builtin_bit_cast(uint32_t, __builtin_amdgcn_fmed3f(v + m, m - qmax, m + qmax));
}

// One ci4 byte from the real part's bits (bias 0) and the imaginary part's (bias 8): the low byte of
// (re << 4) + im is (re & 15) << 4 | (8 + im), 8 + im in [1, 15] so nothing carries; XOR with 8 then gives
// (re & 15) << 4 | (im & 15).  The XOR is left to the caller (four bytes at a time on the staged path).
__device__ __forceinline__ uint32_t fe_ci4_biased(uint32_t re_bits, uint32_t im_bits) { return (re_bits << 4) + im_bits; }

// One ci8 pair: low byte of the real part's bits, then the imaginary part's.
__device__ __forceinline__ uint32_t fe_ci8(uint32_t re_bits, uint32_t im_bits) {
  return __builtin_amdgcn_perm(im_bits, re_bits, 0x0c0c0400u);
}

template <int F, bool CI8, bool VEC>
__global__ __launch_bounds__(kFeThreads) void fengine_kernel(const int8_t* __restrict__ raw, int64_t N, int64_t T,
                                                             int64_t t_per_chunk, const float2* __restrict__ gains,
                                                             uint8_t* __restrict__ out) {
  constexpr int KS = F / 16;         // K-steps of 32 samples (2F samples a block)
  constexpr int TILES = F / 16;      // output tiles of 16 bins
  constexpr int CG = 4 / TILES;      // column groups per work-group
  constexpr int CT = kFeColTiles;    // 32-antenna column tiles per wave
  constexpr int WA = 32 * CT;        // antennas per wave
  constexpr int ANT = WA * CG;       // antennas per work-group
  constexpr int L = 2 * F;           // samples per block
  constexpr int CH = L / 16;         // 16-byte chunks per block
  constexpr int SP = ANT + 8 / CH;   // LDS chunk stride in 16-byte slots (padded: conflict-free writes and reads)
  constexpr int OB = CI8 ? 2 : 1;    // output bytes per code pair
  constexpr int PPT = ANT * CH / kFeThreads;  // 16-byte pieces a thread moves per block
  constexpr int SPC = 32 * CT * OB;  // 16-byte pieces of a wave's code tile
  static_assert(PPT * kFeThreads == ANT * CH && SPC % 64 == 0, "work-group geometry");
  __shared__ double tw[L][2];
  // the work-group's samples of one block, [chunk][antenna] (chunk c = bytes 16 c .. 16 c + 15), double-buffered
  __shared__ fe_int4 xin[2][CH * SP];
  // per wave: codes of 16 bins x WA antennas, row-major (a row is WA consecutive antennas of one bin)
  __shared__ uint4 stage[4][SPC];

  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int tile = w % TILES, cg = w / TILES;
  const int col = l & 31, h = l >> 5;
  const int64_t t0 = (int64_t)blockIdx.y * t_per_chunk;
  const int64_t t1 = min(T, t0 + t_per_chunk);

  // exp(-2 pi i q / 2F), q < 2F, in float64
  for (int q = tid; q < L; q += kFeThreads) sincospi(-2.0 * (double)q / (double)L, &tw[q][1], &tw[q][0]);
  __syncthreads();

  // A fragments, three int8 parts: row col = 2 kk + comp (bin k = 16 tile + kk, comp 0 = Re, 1 = Im); within
  // K-step s, lane half h, byte e -> sample 32 s + 16 h + e of the block (the B operand reads the same bytes).
  fe_int4 wa[3][KS];
  {
    const int kk = col >> 1, comp = col & 1, k = 16 * tile + kk;
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        uint32_t ph = 0, pm = 0, pl = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int j = 32 * s + 16 * h + 4 * d + b;
          const double a = 127.0 * tw[(j * k) % L][comp];
          const double hv = rint(a);
          const double r = (a - hv) * 254.0;
          const double mv = rint(r);
          const double lv = rint((r - mv) * 254.0);
          ph |= (uint32_t)((int)hv & 0xFF) << (8 * b);
          pm |= (uint32_t)((int)mv & 0xFF) << (8 * b);
          pl |= (uint32_t)((int)lv & 0xFF) << (8 * b);
        }
        wa[0][s][d] = (int)ph;
        wa[1][s][d] = (int)pm;
        wa[2][s][d] = (int)pl;
      }
  }

  // the PPT 16-byte pieces this thread moves from HBM to LDS each block: piece q * 256 + tid = (antenna a,
  // chunk c), eight consecutive threads covering one antenna's block (or two or four antennas) in full;
  // antennas past N read antenna N - 1 (their columns are never stored)
  const int64_t n_wg = (int64_t)blockIdx.x * ANT;
  const int8_t* gsrc[PPT];
  int lds_at[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int piece = q * kFeThreads + tid, a = piece / CH, c = piece % CH;
    gsrc[q] = raw + min(n_wg + a, N - 1) * (T * L) + 16 * c;
    lds_at[q] = c * SP + a;
  }

  // antennas of the lane's CT column tiles and their gains for the lane's 8 bins (j4, p), scaled by
  // 1 / (127 * 254^2): rows 8 j4 + 4 h + 2 p + {0, 1} -> bin kk = 4 j4 + 2 h + p
  const int64_t n_base = n_wg + WA * cg;
  int64_t n[CT];
  bool ok[CT];
  float2 g[CT][8];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    n[ct] = n_base + 32 * ct + col;
    ok[ct] = n[ct] < N;
#pragma unroll
    for (int j4 = 0; j4 < 4; ++j4)
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int k = 16 * tile + 4 * j4 + 2 * h + p;
        const float2 gg = ok[ct] ? gains[n[ct] * F + k] : make_float2(0.f, 0.f);
        g[ct][2 * j4 + p] = make_float2(gg.x * kFeScale, gg.y * kFeScale);
      }
  }

  const float qmax = CI8 ? 127.f : 7.f;
  uint8_t* const st_bytes = reinterpret_cast<uint8_t*>(stage[w]);

  auto block = [&](int64_t t, const fe_int4* xb) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      // one column tile's three accumulators live at a time (keeps the kernel at two waves a SIMD)
      if (ct) __builtin_amdgcn_sched_barrier(0);
      fe_int4 b[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s)
        b[s] = xb[(2 * s + h) * SP + WA * cg + 32 * ct + col];
      fe_int16 acc[3] = {};
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(wa[q][s], b[s], acc[q], 0, 0, 0);
#pragma unroll
      for (int j4 = 0; j4 < 4; ++j4)
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const int i = 4 * j4 + 2 * p;
          const float xr = fmaf((float)acc[0][i], 64516.f, (float)(__mul24(acc[1][i], 254) + acc[2][i]));
          const float xi = fmaf((float)acc[0][i + 1], 64516.f, (float)(__mul24(acc[1][i + 1], 254) + acc[2][i + 1]));
          const float2 gg = g[ct][2 * j4 + p];
          const uint32_t cr = fe_code<0>(gg.x * xr - gg.y * xi, qmax);
          const uint32_t ci = fe_code<CI8 ? 0 : 8>(gg.x * xi + gg.y * xr, qmax);
          const uint32_t v = CI8 ? fe_ci8(cr, ci) : fe_ci4_biased(cr, ci);
          const int kk = 4 * j4 + 2 * h + p;
          if (VEC) {
            if (CI8)
              reinterpret_cast<uint16_t*>(st_bytes)[kk * WA + 32 * ct + col] = (uint16_t)v;
            else
              st_bytes[kk * WA + 32 * ct + col] = (uint8_t)v;
          } else if (ok[ct]) {
            const int64_t o = (t * F + 16 * tile + kk) * N + n[ct];
            if (CI8)
              *reinterpret_cast<uint16_t*>(out + 2 * o) = (uint16_t)v;
            else
              out[o] = (uint8_t)(v ^ 8u);
          }
        }
    }
    if (VEC) {
      fe_wave_sync();
#pragma unroll
      for (int c0 = 0; c0 < SPC / 64; ++c0) {
        // 16-byte piece c of the tile: row c / (2 CT OB), antennas 16 / OB * (c % (2 CT OB)) ..
        const int c = 64 * c0 + l;
        const int row = c / (2 * CT * OB), seg = c % (2 * CT * OB);
        const int64_t n0 = n_base + (16 / OB) * seg;
        uint4 v = stage[w][c];
        if (!CI8) v = make_uint4(v.x ^ 0x08080808u, v.y ^ 0x08080808u, v.z ^ 0x08080808u, v.w ^ 0x08080808u);
        if (n0 < N) *reinterpret_cast<uint4*>(out + OB * ((t * F + 16 * tile + row) * N + n0)) = v;
      }
      fe_wave_sync();
    }
  };

  // block t + 1 travels HBM -> registers while block t is transformed, then registers -> LDS; one barrier a block
  auto gload = [&](int64_t t, int q) { return *reinterpret_cast<const fe_int4*>(gsrc[q] + t * L); };
  fe_int4 r[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) r[q] = gload(t0, q);
#pragma unroll
  for (int q = 0; q < PPT; ++q) xin[0][lds_at[q]] = r[q];
  __syncthreads();
  for (int64_t t = t0; t < t1; ++t) {
    const int buf = (int)((t - t0) & 1);
    const bool more = t + 1 < t1;
    if (more) {
#pragma unroll
      for (int q = 0; q < PPT; ++q) r[q] = gload(t + 1, q);
    }
    block(t, xin[buf]);
    if (more) {
#pragma unroll
      for (int q = 0; q < PPT; ++q) xin[buf ^ 1][lds_at[q]] = r[q];
    }
    __syncthreads();
  }
}

template <int F, bool CI8>
hipError_t launch_fe(const int8_t* raw, int64_t N, int64_t T, const float2* gains, uint8_t* out, hipStream_t st) {
  // 16-byte row pieces need rows that start on 16 bytes: N a multiple of 16 / (bytes a code pair), aligned output
  const bool vec = N % (CI8 ? 8 : 16) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0;
  constexpr int ANT = 32 * kFeColTiles * (4 / (F / 16));
  const int64_t groups = (N + ANT - 1) / ANT;
  // about 2048 work-groups (8 a CU), at least 4 blocks each
  int64_t chunks = std::max<int64_t>(1, std::min<int64_t>((2048 + groups - 1) / groups, (T + 3) / 4));
  const int64_t tpc = (T + chunks - 1) / chunks;
  chunks = (T + tpc - 1) / tpc;
  if (groups > INT32_MAX || chunks > 65535) return hipErrorInvalidValue;
  if (vec)
    hipLaunchKernelGGL((fengine_kernel<F, CI8, true>), dim3((unsigned)groups, (unsigned)chunks), dim3(kFeThreads), 0,
                       st, raw, N, T, tpc, gains, out);
  else
    hipLaunchKernelGGL((fengine_kernel<F, CI8, false>), dim3((unsigned)groups, (unsigned)chunks), dim3(kFeThreads), 0,
                       st, raw, N, T, tpc, gains, out);
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
