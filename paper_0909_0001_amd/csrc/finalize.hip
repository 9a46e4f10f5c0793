// Integration state, inverse transform and twiddle tables (gfx950).
//
// After the forward kernels have produced per-slice float64 partial sums of
// |X_t[kappa]|^2, the accumulator A_f[kappa] = sum_t |X_t[kappa]|^2 (time
// integration, Sec. II.A) is formed in natural frequency order, and once per
// integration the visibilities follow from one pruned inverse DFT per axis
// (Sec. II.A "inverse FFT"; Sec. II.C "inverse transforming"):
//
//   V_f[Delta] = (1/M) sum_kappa A_f[kappa] exp(+2 pi i sum_k kappa_k Delta_k / m_k),
//   Delta_k in [-(n_k-1), n_k-1]  (Sec. II.D, index range after Eq. ProofEq2).
//
// Only the 2n_k-1 valid lags of each axis are produced; since every pair
// separation along axis k lies in that range and m_k = 2 n_k, no lag wraps.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>

namespace omni {

// A[f][kmap[c][cell]] (+)= sum_s partial[s][f][c][cell], float64, fixed summation order.
__global__ void reduce_scatter_kernel(const double* __restrict__ partial, const int32_t* __restrict__ kmap,
                                      double* __restrict__ A, int n_slices, int F, int n_split, int cells_wg,
                                      int64_t M, int accumulate) {
  const int64_t per_f = (int64_t)n_split * cells_wg;  // == M
  const int64_t total = (int64_t)F * per_f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = i / per_f;
    const int64_t cc = i - f * per_f;  // c * cells_wg + cell
    double s = 0.0;
    for (int sl = 0; sl < n_slices; ++sl) s += partial[((int64_t)sl * F + f) * per_f + cc];
    double* dst = A + f * M + kmap[cc];
    *dst = accumulate ? *dst + s : s;
  }
}

__global__ void fill_f64_kernel(double* __restrict__ p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// One axis of the inverse transform.  Source [outer][m][inner] (the real
// float64 accumulator if REAL_IN, else complex float32 from the previous axis),
// destination [outer][2n-1][inner] complex float32 (scaled by `scale` if LAST).
// Each lag is summed in float64; only the stored intermediates are float32.
// twi[q] = exp(+2 pi i q / m).  Output lag index o corresponds to Delta = o - (n-1).
template <bool REAL_IN, bool LAST>
__global__ void inverse_axis_kernel(const void* __restrict__ src, void* __restrict__ dst,
                                    const double2* __restrict__ twi, int64_t outer, int m, int n, int64_t inner,
                                    double scale) {
  const int nout = 2 * n - 1;
  const int64_t total = outer * nout * inner;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t in_i = i % inner;
    const int64_t rest = i / inner;
    const int o = (int)(rest % nout);
    const int64_t ou = rest / nout;
    const int delta = o - (n - 1);
    const int dm = ((delta % m) + m) % m;  // Delta mod m
    double re = 0.0, im = 0.0;
    const int64_t base = ou * m * inner + in_i;
    int e = 0;  // kappa * Delta mod m, stepped incrementally
    for (int k = 0; k < m; ++k) {
      const double2 w = twi[e];
      if (REAL_IN) {
        const double a = reinterpret_cast<const double*>(src)[base + (int64_t)k * inner];
        re = fma(a, w.x, re);
        im = fma(a, w.y, im);
      } else {
        const float2 af = reinterpret_cast<const float2*>(src)[base + (int64_t)k * inner];
        const double ax = af.x, ay = af.y;
        re = fma(ax, w.x, fma(-ay, w.y, re));
        im = fma(ax, w.y, fma(ay, w.x, im));
      }
      e += dm;
      if (e >= m) e -= m;
    }
    const double sc = LAST ? scale : 1.0;
    reinterpret_cast<float2*>(dst)[i] = make_float2((float)(re * sc), (float)(im * sc));
  }
}

// The same axis transform with the m inputs of TC columns staged in LDS, so
// that each input is read from HBM once instead of once per output lag.
// Columns are the flattened (outer, inner) index pairs; a work-group takes TC
// consecutive columns and produces their (2n - 1) lags.  m <= 256.
template <bool REAL_IN, bool LAST, int TC>
__global__ __launch_bounds__(256) void inverse_axis_tiled_kernel(const void* __restrict__ src, void* __restrict__ dst,
                                                                 const double2* __restrict__ twi, int64_t outer,
                                                                 int m, int n, int64_t inner, double scale) {
  using Elem = typename std::conditional<REAL_IN, double, float2>::type;
  __shared__ Elem a[TC == 32 ? 2048 : 4096];  // m * TC: m <= 64 for TC = 32, m <= 256 for TC = 16
  __shared__ double2 w[256];
  const int nout = 2 * n - 1;
  const int64_t cols = outer * inner;
  const int64_t col0 = (int64_t)blockIdx.x * TC;
  const int tid = threadIdx.x;
  for (int q = tid; q < m; q += 256) w[q] = twi[q];
  const Elem* s = static_cast<const Elem*>(src);
  // load order: consecutive threads take consecutive inner indices where the tile has them
  const int in_run = inner >= TC ? TC : (TC % inner == 0 ? (int)inner : 1);
  for (int l = tid; l < m * TC; l += 256) {
    const int r = l % in_run, rest = l / in_run;
    const int k = rest % m;
    const int c = (rest / m) * in_run + r;
    const int64_t col = col0 + c;
    if (col < cols) {
      const int64_t ou = col / inner, in = col - ou * inner;
      a[k * TC + c] = s[(ou * m + k) * inner + in];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < nout * TC; idx += 256) {
    const int c = idx % TC, o = idx / TC;
    const int64_t col = col0 + c;
    if (col >= cols) continue;
    const int delta = o - (n - 1);
    const int dm = ((delta % m) + m) % m;
    double re = 0.0, im = 0.0;
    int e = 0;
    for (int k = 0; k < m; ++k) {
      const double2 wk = w[e];
      if constexpr (REAL_IN) {
        const double v = a[k * TC + c];
        re = fma(v, wk.x, re);
        im = fma(v, wk.y, im);
      } else {
        const float2 v = a[k * TC + c];
        const double vx = v.x, vy = v.y;
        re = fma(vx, wk.x, fma(-vy, wk.y, re));
        im = fma(vx, wk.y, fma(vy, wk.x, im));
      }
      e += dm;
      if (e >= m) e -= m;
    }
    const int64_t ou = col / inner, in = col - ou * inner;
    const int64_t oi = (ou * nout + o) * inner + in;
    const double sc = LAST ? scale : 1.0;
    reinterpret_cast<float2*>(dst)[oi] = make_float2((float)(re * sc), (float)(im * sc));
  }
}

// Twiddle generator, float64 on the device: for each table entry (m, q, sign)
// w = exp(sign * 2 pi i q / m), evaluated with sincospi on the exact reduced
// ratio 2q/m.  Writes float32 copies for the forward kernels and float64
// copies for the inverse.
__global__ void twiddle_kernel(const int32_t* __restrict__ desc, int n_tables, float2* __restrict__ tw32,
                               double2* __restrict__ tw64) {
  // desc: per table {m, sign, offset}
  for (int t = 0; t < n_tables; ++t) {
    const int m = desc[3 * t], sign = desc[3 * t + 1], off = desc[3 * t + 2];
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < m; q += gridDim.x * blockDim.x) {
      double s, c;
      sincospi(2.0 * (double)q / (double)m, &s, &c);
      const double im = sign * s;
      if (tw32) tw32[off + q] = make_float2((float)c, (float)im);
      if (tw64) tw64[off + q] = make_double2(c, im);
    }
  }
}

static inline int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_reduce_scatter(const double* partial, const int32_t* kmap, double* A, int n_slices, int F,
                                 int n_split, int cells_wg, int64_t M, int accumulate, hipStream_t st) {
  const int64_t total = (int64_t)F * M;
  hipLaunchKernelGGL(reduce_scatter_kernel, dim3(grid_for(total, 256)), dim3(256), 0, st, partial, kmap, A, n_slices,
                     F, n_split, cells_wg, M, accumulate);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t st) {
  hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_inverse_axis(bool real_in, bool last, const void* src, void* dst, const double2* twi,
                               int64_t outer, int m, int n, int64_t inner, double scale, hipStream_t st) {
  const int64_t cols = outer * inner;
  if (m <= 256 && cols >= (m <= 64 ? 32 : 16) * 256) {
    // TC columns per work-group (m * TC <= 2048 or 4096 elements of LDS), at least 256 work-groups
    const dim3 b(256);
#define OMNI_INV_TILED(TC_)                                                                                          \
  do {                                                                                                               \
    const int64_t nb = (cols + TC_ - 1) / TC_;                                                                       \
    if (nb > INT32_MAX) return hipErrorInvalidValue;                                                                 \
    const dim3 g((unsigned)nb);                                                                                      \
    if (real_in && last)                                                                                             \
      hipLaunchKernelGGL((inverse_axis_tiled_kernel<true, true, TC_>), g, b, 0, st, src, dst, twi, outer, m, n,     \
                         inner, scale);                                                                              \
    else if (real_in)                                                                                                \
      hipLaunchKernelGGL((inverse_axis_tiled_kernel<true, false, TC_>), g, b, 0, st, src, dst, twi, outer, m, n,    \
                         inner, scale);                                                                              \
    else if (last)                                                                                                   \
      hipLaunchKernelGGL((inverse_axis_tiled_kernel<false, true, TC_>), g, b, 0, st, src, dst, twi, outer, m, n,    \
                         inner, scale);                                                                              \
    else                                                                                                             \
      hipLaunchKernelGGL((inverse_axis_tiled_kernel<false, false, TC_>), g, b, 0, st, src, dst, twi, outer, m, n,   \
                         inner, scale);                                                                              \
  } while (0)
    if (m <= 64)
      OMNI_INV_TILED(32);
    else
      OMNI_INV_TILED(16);
#undef OMNI_INV_TILED
    return hipGetLastError();
  }
  const int64_t total = outer * (2 * n - 1) * inner;
  const dim3 g(grid_for(total, 256)), b(256);
  if (real_in && last)
    hipLaunchKernelGGL((inverse_axis_kernel<true, true>), g, b, 0, st, src, dst, twi, outer, m, n, inner, scale);
  else if (real_in)
    hipLaunchKernelGGL((inverse_axis_kernel<true, false>), g, b, 0, st, src, dst, twi, outer, m, n, inner, scale);
  else if (last)
    hipLaunchKernelGGL((inverse_axis_kernel<false, true>), g, b, 0, st, src, dst, twi, outer, m, n, inner, scale);
  else
    hipLaunchKernelGGL((inverse_axis_kernel<false, false>), g, b, 0, st, src, dst, twi, outer, m, n, inner, scale);
  return hipGetLastError();
}

hipError_t launch_twiddles(const int32_t* desc_dev, int n_tables, float2* tw32, double2* tw64, hipStream_t st) {
  hipLaunchKernelGGL(twiddle_kernel, dim3(4), dim3(256), 0, st, desc_dev, n_tables, tw32, tw64);
  return hipGetLastError();
}

}  // namespace omni
