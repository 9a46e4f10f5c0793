// Hybrid tiles (Sec. III): P rectangular n_x x n_y tiles at arbitrary
// translations.  Inside a tile the FFT method applies; between tiles the
// tiles' transforms ("synthesized beams") are correlated pair by pair.
//
// Per time sample each tile's zero-padded 2-D transform Y_p[kappa] (m = 2n per
// axis) comes from two front passes (front.hip).  The pair stage here is the
// X-engine over Fourier cells: for every channel f and cell kappa,
//   S_pq[kappa] += sum_t Y_p[t][kappa] conj(Y_q[t][kappa]),   all ordered (p, q),
// which the inverse transform (finalize.hip) turns into the cross-correlation
// of tiles p and q over index differences (C_pp is tile p's own hypercube).
//
// xengine_kernel: a thread owns one cell kappa and a block of RB tiles p
// (rows) against all P tiles q (columns), RB x P complex float32 sums over the
// chunk's samples, then one float64 read-modify-write of S.  The row-block
// threads of one cell are adjacent lanes, so the P loads of a cell and sample
// are shared through the cache; consecutive cells are consecutive addresses.

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace omni {
namespace {

constexpr int kXeThreads = 256;

template <int P, int RB>
__global__ __launch_bounds__(kXeThreads) void xengine_kernel(const float2* __restrict__ Y, int64_t Tc, int F,
                                                             int64_t Mp, double2* __restrict__ S, int accumulate) {
  constexpr int NRB = P / RB;           // row blocks per cell
  constexpr int CELLS = kXeThreads / NRB;  // cells per work-group
  const int tid = threadIdx.x;
  const int rb = tid % NRB;
  const int64_t kappa = (int64_t)blockIdx.x * CELLS + tid / NRB;
  const int f = blockIdx.y;
  if (kappa >= Mp) return;
  float2 acc[RB][P];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int q = 0; q < P; ++q) acc[r][q] = make_float2(0.f, 0.f);
  for (int64_t t = 0; t < Tc; ++t) {
    const float2* y = Y + ((t * F + f) * (int64_t)P) * Mp + kappa;
    float2 v[P];
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] = y[(int64_t)q * Mp];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const float2 a = v[rb * RB + r];
#pragma unroll
      for (int q = 0; q < P; ++q) {
        // a conj(v_q)
        acc[r][q].x = fmaf(a.x, v[q].x, fmaf(a.y, v[q].y, acc[r][q].x));
        acc[r][q].y = fmaf(a.y, v[q].x, fmaf(-a.x, v[q].y, acc[r][q].y));
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int p = rb * RB + r;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      double2* s = S + (((int64_t)f * P + p) * P + q) * Mp + kappa;
      double2 o = make_double2((double)acc[r][q].x, (double)acc[r][q].y);
      if (accumulate) {
        const double2 old = *s;
        o.x += old.x;
        o.y += old.y;
      }
      *s = o;
    }
  }
}

__global__ void narrow_kernel(const double2* __restrict__ src, float2* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = make_float2((float)src[i].x, (float)src[i].y);
}

template <int P>
hipError_t launch_xe(const float2* Y, int64_t Tc, int F, int64_t Mp, double2* S, int accumulate, hipStream_t st) {
  constexpr int RB = P >= 2 ? 2 : 1;
  constexpr int CELLS = kXeThreads / (P / RB);
  const int64_t blocks = (Mp + CELLS - 1) / CELLS;
  if (blocks > INT32_MAX || F < 1 || F > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL((xengine_kernel<P, RB>), dim3((unsigned)blocks, (unsigned)F), dim3(kXeThreads), 0, st, Y, Tc,
                     F, Mp, S, accumulate);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_xengine(const float2* Y, int64_t Tc, int F, int P, int64_t Mp, double2* S, int accumulate,
                          hipStream_t st) {
  switch (P) {
    case 2: return launch_xe<2>(Y, Tc, F, Mp, S, accumulate, st);
    case 4: return launch_xe<4>(Y, Tc, F, Mp, S, accumulate, st);
    case 8: return launch_xe<8>(Y, Tc, F, Mp, S, accumulate, st);
    case 16: return launch_xe<16>(Y, Tc, F, Mp, S, accumulate, st);
    case 32: return launch_xe<32>(Y, Tc, F, Mp, S, accumulate, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_narrow(const double2* src, float2* dst, int64_t n, hipStream_t st) {
  const int64_t g = std::max<int64_t>(1, std::min<int64_t>(65536, (n + 255) / 256));
  hipLaunchKernelGGL(narrow_kernel, dim3((unsigned)g), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

}  // namespace omni
