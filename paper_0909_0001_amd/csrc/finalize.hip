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

// The same axis transform for a power-of-two m <= 32 as a radix-2 FFT in
// registers: one thread per column (consecutive threads take consecutive inner
// indices), all m outputs y_j = sum_k a_k exp(+2 pi i k j / m) in float64, of
// which the 2n - 1 = m - 1 lags Delta = j (j < n) and Delta = j - m (j > n) are
// stored.  O(m log m) work per column instead of O(m^2).
template <int M>
constexpr int bitrev(int k) {
  int r = 0;
  for (int b = 1; b < M; b <<= 1) r = (r << 1) | ((k / b) & 1);
  return r;
}

template <int M, bool REAL_IN, bool LAST>
__global__ __launch_bounds__(256) void inverse_axis_fft_kernel(const void* __restrict__ src, void* __restrict__ dst,
                                                               const double2* __restrict__ twi, int64_t outer,
                                                               int64_t inner, double scale) {
  constexpr int NOUT = M - 1, NH = M / 2;
  __shared__ double2 w[NH];  // exp(+2 pi i q / M), q < M / 2
  for (int q = threadIdx.x; q < NH; q += blockDim.x) w[q] = twi[q];
  __syncthreads();
  const int64_t cols = outer * inner;
  const double sc = LAST ? scale : 1.0;
  for (int64_t col = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; col < cols;
       col += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ou = col / inner, in = col - ou * inner;
    double2 x[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int64_t at = (ou * M + k) * inner + in;
      if constexpr (REAL_IN) {
        x[bitrev<M>(k)] = make_double2(static_cast<const double*>(src)[at], 0.0);
      } else {
        const float2 v = static_cast<const float2*>(src)[at];
        x[bitrev<M>(k)] = make_double2(v.x, v.y);
      }
    }
#pragma unroll
    for (int len = 2; len <= M; len <<= 1) {
#pragma unroll
      for (int i = 0; i < M; i += len) {
#pragma unroll
        for (int j = 0; j < len / 2; ++j) {
          const double2 u = x[i + j];
          double2 v = x[i + j + len / 2];
          if (j > 0) {
            const double2 wj = w[j * (M / len)];  // exp(+2 pi i j / len)
            v = make_double2(fma(v.x, wj.x, -v.y * wj.y), fma(v.x, wj.y, v.y * wj.x));
          }
          x[i + j] = make_double2(u.x + v.x, u.y + v.y);
          x[i + j + len / 2] = make_double2(u.x - v.x, u.y - v.y);
        }
      }
    }
    float2* d = static_cast<float2*>(dst);
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      const int delta = o - (NH - 1);
      const double2 y = x[delta >= 0 ? delta : delta + M];
      d[(ou * NOUT + o) * inner + in] = make_float2((float)(y.x * sc), (float)(y.y * sc));
    }
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

template <int M>
static hipError_t launch_inverse_fft(bool real_in, bool last, const void* src, void* dst, const double2* twi,
                                     int64_t outer, int64_t inner, double scale, hipStream_t st) {
  const dim3 g(grid_for(outer * inner, 256)), b(256);
  if (real_in && last)
    hipLaunchKernelGGL((inverse_axis_fft_kernel<M, true, true>), g, b, 0, st, src, dst, twi, outer, inner, scale);
  else if (real_in)
    hipLaunchKernelGGL((inverse_axis_fft_kernel<M, true, false>), g, b, 0, st, src, dst, twi, outer, inner, scale);
  else if (last)
    hipLaunchKernelGGL((inverse_axis_fft_kernel<M, false, true>), g, b, 0, st, src, dst, twi, outer, inner, scale);
  else
    hipLaunchKernelGGL((inverse_axis_fft_kernel<M, false, false>), g, b, 0, st, src, dst, twi, outer, inner, scale);
  return hipGetLastError();
}

hipError_t launch_inverse_axis(bool real_in, bool last, const void* src, void* dst, const double2* twi,
                               int64_t outer, int m, int n, int64_t inner, double scale, hipStream_t st) {
  const int64_t cols = outer * inner;
  if (m == 2 * n) {
    if (m == 4) return launch_inverse_fft<4>(real_in, last, src, dst, twi, outer, inner, scale, st);
    if (m == 8) return launch_inverse_fft<8>(real_in, last, src, dst, twi, outer, inner, scale, st);
    if (m == 16) return launch_inverse_fft<16>(real_in, last, src, dst, twi, outer, inner, scale, st);
    if (m == 32) return launch_inverse_fft<32>(real_in, last, src, dst, twi, outer, inner, scale, st);
  }
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


// The even Fourier cells of the last `axes` (1 or 2) axes of a real float64 array: rows of (2 na) x (2 nb)
// values in, na x nb out (nb = 1 for one axis).  With m = 2n, the cell 2b of the zero-padded transform is
// the unpadded transform's cell b.
__global__ void even_cells_kernel(const double* __restrict__ A, double* __restrict__ E, int64_t rows, int na,
                                  int nb, int axes) {
  const int64_t per = (int64_t)na * nb;
  const int64_t total = rows * per;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / per;
    const int c = (int)(i - r * per);
    const int bx = c / nb, by = c - bx * nb;
    E[i] = axes == 2 ? A[(r * 2 * na + 2 * bx) * (2 * nb) + 2 * by] : A[r * 2 * na + 2 * bx];
  }
}

hipError_t launch_even_cells(const double* A, double* E, int64_t rows, int na, int nb, int axes, hipStream_t st) {
  if ((axes != 1 && axes != 2) || na < 1 || nb < 1 || (axes == 1 && nb != 1)) return hipErrorInvalidValue;
  const int64_t total = rows * na * nb;
  const int64_t g = std::max<int64_t>(1, std::min<int64_t>(65536, (total + 255) / 256));
  hipLaunchKernelGGL(even_cells_kernel, dim3((unsigned)g), dim3(256), 0, st, A, E, rows, na, nb, axes);
  return hipGetLastError();
}

}  // namespace omni
