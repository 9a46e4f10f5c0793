// Physical-baseline fold of the visibility hypercube and the baseline-distribution
// products of Sec. III.
//
// Sec. II.D: the hypercube cell Delta collects every antenna pair whose index
// tuples differ by Delta; its physical separation is b(Delta) = sum_k Delta_k a_k
// (Eq. GridEq).  When distinct cells share one separation (the 3-level layout
// of Fig. 1 does this) the physical correlation at b is the sum of those cells.
// The fold sums the cells into pixels of a (u, v) grid: cell Delta lands in
// pixel (rint(b_x / du), rint(b_y / dv)) relative to the image centre, which
// is the exact fold for integer lattice vectors and du = dv = 1, and
// nearest-pixel gridding otherwise.
//
// Layout of the work.  The cell -> pixel map depends only on the geometry, so
// the plan computes every cell's pixel on the device once, sorts the cells by
// pixel (stable radix sort, so cells of one pixel stay in ascending order) and
// keeps the sorted cell list with per-pixel offsets (CSR).  A fold call is then
// a gather: one thread per pixel and group of eight channels sums the pixel's
// cells in that fixed order in float64, so the result is deterministic.  The radial distribution uses
// the same scheme over pixels grouped by radial bin, one wave per (bin,
// channel) with a fixed-order reduction.
//
// The baseline and radius arithmetic is done with fused multiply-add
// contraction off, in the order the method's definitions state it, so that the
// integer decisions it feeds (pixel, radial bin) follow from correctly rounded
// float64 operations alone.

#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>

#include "fold.hpp"

namespace omni {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double cell_coord_sum(double acc, double a0, double d0, double a1, double d1) {
#pragma clang fp contract(off)
  const double t = a0 * d0;
  const double u = a1 * d1;
  const double s = t + u;
  return acc + s;
}

__global__ void fold_keys_kernel(FoldGeom g, uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
#pragma clang fp contract(off)
  const int d = 2 * g.levels;
  const int64_t npix = g.nx * g.ny;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < g.cells;
       c += (int64_t)gridDim.x * blockDim.x) {
    int delta[2 * kFoldMaxLevels];
    int64_t rem = c;
    for (int k = d - 1; k >= 0; --k) {
      const int e = 2 * g.n[k] - 1;
      delta[k] = (int)(rem % e) - (g.n[k] - 1);
      rem /= e;
    }
    double bx = 0.0, by = 0.0;
    for (int l = 0; l < g.levels; ++l) {
      const double dx = (double)delta[2 * l], dy = (double)delta[2 * l + 1];
      bx = cell_coord_sum(bx, g.A[l][0], dx, g.A[l][1], dy);
      by = cell_coord_sum(by, g.A[l][2], dx, g.A[l][3], dy);
    }
    const int64_t px = (int64_t)rint(bx / g.du) + g.cx;
    const int64_t py = (int64_t)rint(by / g.dv) + g.cy;
    const bool in = px >= 0 && px < g.nx && py >= 0 && py < g.ny;
    // a cell outside the image would sort behind every pixel and be caught by the plan's count check
    key[c] = in ? (uint32_t)(py * g.nx + px) : (uint32_t)npix;
    val[c] = (uint32_t)c;
  }
}

__global__ void radial_keys_kernel(RadialGeom g, uint32_t* __restrict__ key, uint32_t* __restrict__ val,
                                   uint32_t* __restrict__ max_bin) {
#pragma clang fp contract(off)
  const int64_t npix = g.nx * g.ny;
  uint32_t mx = 0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t iy = p / g.nx, ix = p - iy * g.nx;
    const double bx = (double)(ix - g.cx) * g.du;
    const double by = (double)(iy - g.cy) * g.dv;
    const double r2 = bx * bx + by * by;
    const double r = __builtin_sqrt(r2);
    const double q = r * g.scale / g.dr;
    const uint32_t k = (uint32_t)floor(q);
    key[p] = k;
    val[p] = (uint32_t)p;
    mx = k > mx ? k : mx;
  }
  atomicMax(max_bin, mx);
}

__global__ void group_offsets_kernel(const uint32_t* __restrict__ keys, int64_t n, uint32_t* __restrict__ off,
                                     int64_t n_groups) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n_groups) return;
  // first position whose key is >= i
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)keys[mid] < i)
      lo = mid + 1;
    else
      hi = mid;
  }
  off[i] = (uint32_t)lo;
}

// One thread per pixel and group of kFoldCh channels: the pixel's cell list is read once and its channels'
// loads are independent of each other.
constexpr int kFoldCh = 8;

__global__ void fold_gather_kernel(const float2* __restrict__ vis, int64_t cells, const uint32_t* __restrict__ cell,
                                   const uint32_t* __restrict__ off, int64_t npix, int F, int64_t origin,
                                   double2* __restrict__ image) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int f0 = blockIdx.y * kFoldCh;
  if (p >= npix) return;
  const int nf = min(kFoldCh, F - f0);
  double re[kFoldCh], im[kFoldCh];
#pragma unroll
  for (int j = 0; j < kFoldCh; ++j) re[j] = im[j] = 0.0;
  if (p != origin) {
    const uint32_t e = off[p + 1];
    for (uint32_t i = off[p]; i < e; ++i) {
      const float2* v = vis + (int64_t)f0 * cells + cell[i];
      float2 x[kFoldCh];
#pragma unroll
      for (int j = 0; j < kFoldCh; ++j) x[j] = j < nf ? v[(int64_t)j * cells] : make_float2(0.f, 0.f);
#pragma unroll
      for (int j = 0; j < kFoldCh; ++j) {
        re[j] += (double)x[j].x;
        im[j] += (double)x[j].y;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kFoldCh; ++j)
    if (j < nf) image[(int64_t)(f0 + j) * npix + p] = make_double2(re[j], im[j]);
}

__global__ void channel_max_kernel(const double2* __restrict__ image, int64_t npix, double* __restrict__ dmax) {
  __shared__ double red[kThreads];
  const int f = blockIdx.x;
  const double2* im = image + (int64_t)f * npix;
  double m = -__builtin_inf();
  for (int64_t p = threadIdx.x; p < npix; p += kThreads) m = fmax(m, im[p].x);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) dmax[f] = red[0];
}

__global__ void asinh_map_kernel(const double2* __restrict__ image, int64_t npix, const double* __restrict__ dmax,
                                 double* __restrict__ map) {
#pragma clang fp contract(off)
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (p >= npix) return;
  const double m = dmax[f] > 0.0 ? dmax[f] : 1.0;
  const double x = 4.0 * image[(int64_t)f * npix + p].x / m;
  map[(int64_t)f * npix + p] = asinh(x);
}

// One wave per (bin, channel): lane l adds pixels l, l + 64, ... of the bin, then a fixed butterfly.
__global__ void radial_sum_kernel(const double2* __restrict__ image, int64_t npix, const uint32_t* __restrict__ pix,
                                  const uint32_t* __restrict__ boff, int64_t nbins, double* __restrict__ hist) {
  const int64_t k = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  const int f = blockIdx.y;
  if (k >= nbins) return;
  const double2* im = image + (int64_t)f * npix;
  double s = 0.0;
  for (uint32_t i = boff[k] + l; i < boff[k + 1]; i += 64) s += im[pix[i]].x;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (l == 0) hist[(int64_t)f * nbins + k] = s;
}

__global__ void boxcar_kernel(const double* __restrict__ hist, int64_t nbins, int width, double* __restrict__ smooth) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (k >= nbins) return;
  const double* h = hist + (int64_t)f * nbins;
  const int half = width / 2;
  double s = 0.0;
  for (int j = -half; j <= half; ++j) {
    const int64_t q = k + j;
    s += (q >= 0 && q < nbins) ? h[q] : 0.0;
  }
  smooth[(int64_t)f * nbins + k] = s / (double)width;
}

unsigned grid_for(int64_t n, int64_t cap = 65536) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cap, (n + kThreads - 1) / kThreads));
}

}  // namespace

hipError_t launch_fold_keys(const FoldGeom& g, uint32_t* key, uint32_t* val, hipStream_t st) {
  if (g.cells <= 0) return hipSuccess;
  hipLaunchKernelGGL(fold_keys_kernel, dim3(grid_for(g.cells)), dim3(kThreads), 0, st, g, key, val);
  return hipGetLastError();
}

hipError_t launch_radial_keys(const RadialGeom& g, uint32_t* key, uint32_t* val, uint32_t* max_bin, hipStream_t st) {
  hipLaunchKernelGGL(radial_keys_kernel, dim3(grid_for(g.nx * g.ny)), dim3(kThreads), 0, st, g, key, val, max_bin);
  return hipGetLastError();
}

hipError_t launch_group_offsets(const uint32_t* sorted_keys, int64_t n, uint32_t* off, int64_t n_groups,
                                hipStream_t st) {
  const int64_t blocks = (n_groups + 1 + kThreads - 1) / kThreads;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(group_offsets_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, st, sorted_keys, n, off,
                     n_groups);
  return hipGetLastError();
}

hipError_t sort_pairs(void* tmp, size_t* tmp_bytes, const uint32_t* key_in, uint32_t* key_out, const uint32_t* val_in,
                      uint32_t* val_out, int64_t n, int key_bits, hipStream_t st) {
  return rocprim::radix_sort_pairs(tmp, *tmp_bytes, key_in, key_out, val_in, val_out, (size_t)n, 0u,
                                   (unsigned)key_bits, st);
}

hipError_t launch_fold_gather(const float2* vis, int64_t cells, const uint32_t* cell, const uint32_t* off,
                              int64_t npix, int F, int64_t origin, double2* image, hipStream_t st) {
  const int64_t blocks = (npix + kThreads - 1) / kThreads;
  if (F < 1 || F > 65535 || blocks > INT32_MAX) return hipErrorInvalidValue;
  const unsigned groups = (unsigned)((F + kFoldCh - 1) / kFoldCh);
  hipLaunchKernelGGL(fold_gather_kernel, dim3((unsigned)blocks, groups), dim3(kThreads), 0, st, vis, cells, cell, off,
                     npix, F, origin, image);
  return hipGetLastError();
}

hipError_t launch_channel_max(const double2* image, int64_t npix, int F, double* dmax, hipStream_t st) {
  if (F < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(channel_max_kernel, dim3((unsigned)F), dim3(kThreads), 0, st, image, npix, dmax);
  return hipGetLastError();
}

hipError_t launch_asinh_map(const double2* image, int64_t npix, int F, const double* dmax, double* map,
                            hipStream_t st) {
  const int64_t blocks = (npix + kThreads - 1) / kThreads;
  if (F < 1 || F > 65535 || blocks > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(asinh_map_kernel, dim3((unsigned)blocks, (unsigned)F), dim3(kThreads), 0, st, image, npix, dmax,
                     map);
  return hipGetLastError();
}

hipError_t launch_radial_sum(const double2* image, int64_t npix, int F, const uint32_t* pix, const uint32_t* boff,
                             int64_t nbins, double* hist, hipStream_t st) {
  const int64_t blocks = (nbins + kThreads / 64 - 1) / (kThreads / 64);
  if (F < 1 || F > 65535 || blocks > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(radial_sum_kernel, dim3((unsigned)blocks, (unsigned)F), dim3(kThreads), 0, st, image, npix, pix,
                     boff, nbins, hist);
  return hipGetLastError();
}

hipError_t launch_boxcar(const double* hist, int64_t nbins, int F, int width, double* smooth, hipStream_t st) {
  const int64_t blocks = (nbins + kThreads - 1) / kThreads;
  if (F < 1 || F > 65535 || blocks > INT32_MAX || width < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(boxcar_kernel, dim3((unsigned)blocks, (unsigned)F), dim3(kThreads), 0, st, hist, nbins, width,
                     smooth);
  return hipGetLastError();
}

}  // namespace omni
