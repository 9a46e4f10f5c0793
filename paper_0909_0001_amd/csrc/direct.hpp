// Shapes and launchers of the direct N^2 correlator (direct.hip), shared with the host planner.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace omni {

constexpr int kDirectTile = 128;       // antennas per block of the pair tile
constexpr int kDirectMaxD = 8;         // axes
constexpr int kDirectMaxBins = 2048;   // Delta box of one block pair, held in LDS
constexpr int64_t kDirectMaxT = 32768; // samples per launch: int32 pair sums cannot overflow (2 * 128^2 * 2^15 = 2^30)

struct DirectGeom {
  int d = 0;                       // axes (row-major antenna index over n[0..d-1])
  int n[kDirectMaxD] = {};         // antennas per axis
  int64_t gstride[kDirectMaxD] = {};  // strides of the centred output hypercube, extents 2 n_k - 1
  int64_t n_out = 0;               // cells of the output hypercube
};

hipError_t launch_direct_zero(unsigned long long* G, int64_t n, hipStream_t st);
hipError_t launch_direct_tiles(int fmt, const void* src, int64_t T, int64_t N, int F, const int32_t* pairs,
                               int64_t n_pairs, const int32_t* blk, const DirectGeom& g, unsigned long long* G,
                               hipStream_t st);
hipError_t launch_direct_finalize(const unsigned long long* G, void* vis, int64_t n_out, int F, hipStream_t st);
// The no-allocation entry point's fixed device scratch (direct.hip): its size, its address on the current device
// (resolved once per device), and the kernel that builds the block boxes and block pairs in it.
size_t direct_noalloc_capacity();
hipError_t direct_noalloc_scratch(void** ptr);
hipError_t launch_direct_setup(const DirectGeom& g, int64_t nbk, int32_t* blk, int32_t* pairs, hipStream_t st);

}  // namespace omni
