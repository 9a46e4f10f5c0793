// Physical-baseline fold of the visibility hypercube and the baseline-distribution
// products of Sec. III (fold.hip), shared with the host entry points.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace omni {

constexpr int kFoldMaxLevels = 4;

// Geometry of one array as the fold sees it: the hypercube axes (2 per level, all of them, size-1 axes
// included, as in the visibility layout [F][2 n_1 - 1]...[2 n_d - 1]) and the lattice matrices.
struct FoldGeom {
  int levels = 0;
  int n[2 * kFoldMaxLevels] = {};       // antennas per axis
  double A[kFoldMaxLevels][4] = {};     // per level, row-major [[a_xx, a_yx], [a_xy, a_yy]] (columns = vectors)
  int64_t cells = 0;                    // prod (2 n_k - 1)
  double du = 1.0, dv = 1.0;            // pixel size
  int64_t cx = 0, cy = 0, nx = 1, ny = 1;  // zero baseline pixel, image extent
};

// Radial binning of the image pixels: bin k = floor(|b| * scale / dr).
struct RadialGeom {
  int64_t cx = 0, cy = 0, nx = 1, ny = 1;
  double du = 1.0, dv = 1.0, dr = 1.0, scale = 1.0;
};

// key[c] = pixel of cell c, val[c] = c.
hipError_t launch_fold_keys(const FoldGeom& g, uint32_t* key, uint32_t* val, hipStream_t st);
// key[p] = radial bin of pixel p, val[p] = p; *max_bin (device) receives the largest bin (must start at 0).
hipError_t launch_radial_keys(const RadialGeom& g, uint32_t* key, uint32_t* val, uint32_t* max_bin, hipStream_t st);
// off[i] = first position of sorted_keys holding a key >= i, i in [0, n_groups]  (CSR offsets).
hipError_t launch_group_offsets(const uint32_t* sorted_keys, int64_t n, uint32_t* off, int64_t n_groups,
                                hipStream_t st);
// Stable sort of (key, value) pairs by key (n elements, keys below 2^key_bits); `tmp` of `*tmp_bytes`
// (query with tmp == nullptr).
hipError_t sort_pairs(void* tmp, size_t* tmp_bytes, const uint32_t* key_in, uint32_t* key_out,
                      const uint32_t* val_in, uint32_t* val_out, int64_t n, int key_bits, hipStream_t st);
// image[f][p] = sum over the cells of pixel p (ascending cell order) of vis[f][cell], float64 complex.
hipError_t launch_fold_gather(const float2* vis, int64_t cells, const uint32_t* cell, const uint32_t* off,
                              int64_t npix, int F, int64_t origin, double2* image, hipStream_t st);
// Per channel: dmax[f] = max_p Re image[f][p]; map (may be null) = asinh(4 Re image / dmax);
// hist (may be null) [F][nbins] = radial sums; smooth (may be null) = centred boxcar of hist over `width` bins.
hipError_t launch_channel_max(const double2* image, int64_t npix, int F, double* dmax, hipStream_t st);
hipError_t launch_asinh_map(const double2* image, int64_t npix, int F, const double* dmax, double* map,
                            hipStream_t st);
hipError_t launch_radial_sum(const double2* image, int64_t npix, int F, const uint32_t* pix, const uint32_t* boff,
                             int64_t nbins, double* hist, hipStream_t st);
hipError_t launch_boxcar(const double* hist, int64_t nbins, int F, int width, double* smooth, hipStream_t st);

}  // namespace omni
