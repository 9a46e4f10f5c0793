// Fused float32 correlator with a compile-time shape (gfx950).
//
// The schedule is the general fused kernel's (fold + short DFT per axis,
// Fourier cells divided among work-groups by residue classes of axis 0, cells
// in the same layout), but every extent and stride is a compile-time power of
// two, so job and address arithmetic reduce to shifts and masks, intermediate
// arrays ping-pong between two LDS buffers (one barrier per pass), the short
// DFTs' twiddles live in registers, and the last pass adds |X|^2 straight into
// the thread's registers.
//
// Per axis k: n_k antennas, padded length m_k = 2 n_k, fold modulus r_k,
// short-DFT length L_k = m_k / r_k; the outputs with frequency = rho (mod r_k)
// are X[r_k q + rho] = DFT_L(z)[q], z_j = sum_l x[j + l L] w_m^{rho (j + l L)}
// (the zero-padded DFT of Sec. II.A/II.C split by residue class).  A
// work-group holds R_k = r_k / S_k residue classes of axis k (S_0 = the split,
// S_k = 1 otherwise), so its extent along k is E_k = R_k L_k.  Passes run over
// axis 0 (from HBM), then axes d-1 ... 2 (LDS), then axis 1 (squared).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>
#include <utility>

#include "plan.hpp"
#include "shortdft.hpp"

namespace omni {

namespace ct {

using sd::cadd;
using sd::cmul;
using sd::csub;
using sd::dft;

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

template <int D_, int N0, int N1, int N2, int N3, int R0, int R1, int R2, int R3, int S0_>
struct Shape {
  static constexpr int D = D_;
  static constexpr int S0 = S0_;
  static constexpr int n(int k) { return k == 0 ? N0 : k == 1 ? N1 : k == 2 ? N2 : N3; }
  static constexpr int r(int k) { return k == 0 ? R0 : k == 1 ? R1 : k == 2 ? R2 : R3; }
  static constexpr int m(int k) { return 2 * n(k); }
  static constexpr int L(int k) { return m(k) / r(k); }
  static constexpr int Rw(int k) { return k == 0 ? r(0) / S0 : r(k); }
  static constexpr int E(int k) { return Rw(k) * L(k); }
  static constexpr int step(int k) { return k == 0 ? S0 : 1; }
  // processing order: 0, D-1, D-2, ..., 1
  static constexpr int axis_of(int p) { return p == 0 ? 0 : D - p; }
  static constexpr bool done_before(int p, int j) {
    for (int q = 0; q < p; ++q)
      if (axis_of(q) == j) return true;
    return false;
  }
  static constexpr int ext(int p, int j) { return done_before(p, j) ? E(j) : n(j); }
  static constexpr int inner(int p, int k) {
    int s = 1;
    for (int j = k + 1; j < D; ++j) s *= ext(p, j);
    return s;
  }
  static constexpr int lines(int p, int k) {
    int s = 1;
    for (int j = 0; j < D; ++j)
      if (j != k) s *= ext(p, j);
    return s;
  }
  static constexpr int size_after(int p) {  // elements of the array after pass p
    int s = 1;
    for (int j = 0; j < D; ++j) s *= done_before(p + 1, j) ? E(j) : n(j);
    return s;
  }
  static constexpr int N() {
    int s = 1;
    for (int j = 0; j < D; ++j) s *= n(j);
    return s;
  }
  static constexpr int cells() {
    int s = 1;
    for (int j = 0; j < D; ++j) s *= E(j);
    return s;
  }
};

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

// Fold of one job: z_j = sum_l x[j + l L] w_m^{rho (j + l L)}, j < L, with
// m = M the padded length and n = N = M / 2 inputs, i.e. l < r / 2 non-zero
// blocks (r = M / L).  Factored as z_j = w_m^{rho j} sum_l x[j + l L] w_r^{rho l},
// so that the inner twiddles sit in registers and each input costs four FMAs;
// the L outer twiddles come from the axis table.
//   r = 1: rho = 0 and z_j = x_j (j < n), zero above.
//   r = 2: one block, z_j = w_m^{rho j} x_j.
template <int N, int M, int L, class Get>
__device__ __forceinline__ void fold(float2 (&z)[L], int rho, const float2* __restrict__ twm, Get get) {
  constexpr int R = M / L;
  static_assert(M == 2 * N && R * L == M, "padded axis");
  if constexpr (R == 1) {
#pragma unroll
    for (int j = 0; j < L; ++j) z[j] = j < N ? get(j) : make_float2(0.f, 0.f);
    return;
  } else {
    constexpr int NB = N / L;  // = r / 2 non-zero blocks
    float2 u[NB];
#pragma unroll
    for (int l = 0; l < NB; ++l) u[l] = twm[(rho * l * L) & (M - 1)];  // w_r^{rho l}
#pragma unroll
    for (int j = 0; j < L; ++j) z[j] = get(j);  // l = 0: u_0 = 1
#pragma unroll
    for (int l = 1; l < NB; ++l) {
#pragma unroll
      for (int j = 0; j < L; ++j) {
        const float2 v = get(j + l * L);
        const float2 w = u[l];
        z[j].x = fmaf(v.x, w.x, fmaf(-v.y, w.y, z[j].x));
        z[j].y = fmaf(v.x, w.y, fmaf(v.y, w.x, z[j].y));
      }
    }
#pragma unroll
    for (int j = 1; j < L; ++j) z[j] = cmul(z[j], twm[(rho * j) & (M - 1)]);  // w_m^{rho j}
  }
}

}  // namespace ct

// LDS arrays of intermediate values carry one float2 of padding after every
// 32 (one sweep of the 64 four-byte banks): element e lives at e + e / 32.
// Rows at power-of-two strides then start on distinct banks, and within a
// job the offsets stay compile-time constants.
__device__ __forceinline__ int swz(int e) { return e + (e >> 5); }

template <int FMT>
struct Sample;
template <>
struct Sample<0> {
  static constexpr int bytes = 8;
  __device__ static float2 get(const unsigned char* p, int e) { return reinterpret_cast<const float2*>(p)[e]; }
};
template <>
struct Sample<1> {
  static constexpr int bytes = 2;
  __device__ static float2 get(const unsigned char* p, int e) {
    const char2 v = reinterpret_cast<const char2*>(p)[e];
    return make_float2((float)v.x, (float)v.y);
  }
};
template <>
struct Sample<2> {
  static constexpr int bytes = 1;
  __device__ static float2 get(const unsigned char* p, int e) {
    const int8_t v = reinterpret_cast<const int8_t*>(p)[e];
    return make_float2((float)(v >> 4), (float)((int8_t)(v << 4) >> 4));
  }
};

// STAGE: the work-group copies each (time, channel) tile into LDS with
// asynchronous direct-to-LDS loads (global_load_lds_dwordx4), one sample ahead
// of the transform, so that pass 0 reads LDS and the HBM latency overlaps the
// later passes.  Requires a 16-byte aligned source (checked by the host).
template <int FMT, class SH, int NT, bool STAGE>
__global__ __launch_bounds__(NT) void fused_ct_fp32_kernel(const void* __restrict__ src, int64_t T,
                                                           int64_t t_per_slice, const float2* __restrict__ tw_glob,
                                                           double* __restrict__ partial, int F, int xcd_groups,
                                                           int time_block, int accumulate) {
  using namespace ct;
  constexpr int D = SH::D;
  static_assert(D >= 2 && D <= 4, "compile-time shapes have 2 to 4 axes");
  constexpr int S0 = SH::S0;
  constexpr int CELLS = SH::cells();
  constexpr int N = SH::N();
  constexpr int SB = Sample<FMT>::bytes;
  // intermediate arrays: passes 0 and 2 write bufA, pass 1 writes bufB
  constexpr int BA = SH::size_after(0) > (D > 3 ? SH::size_after(2) : 0) ? SH::size_after(0) : SH::size_after(2);
  constexpr int BB = D > 2 ? SH::size_after(1) : 32;
  static_assert(BA % 32 == 0 && BB % 32 == 0, "padding blocks");
  constexpr int TWN = [] {
    int s = 0;
    for (int k = 0; k < SH::D; ++k) s += SH::m(k);
    return s;
  }();
  constexpr int RAWB = STAGE ? N * SB : 16;
  static_assert(!STAGE || RAWB % 1024 == 0, "a staged tile is whole 1 KiB wave loads");
  // INPLACE (three axes, float32 tile, one job per thread and column in pass 0): pass 0 writes its
  // output over the consumed tile instead of bufA, and the next tile is fetched after pass 1.  This
  // keeps two work-groups per CU for the (16,16,16) grid behind a front pass.
  constexpr bool INPLACE = STAGE && FMT == 0 && D == 3 && SH::Rw(0) == 1 &&
                           SH::lines(0, 0) == NT && (BA + BA / 32) * 8 <= RAWB;
  __shared__ __attribute__((aligned(16))) unsigned char raw[RAWB];
  __shared__ float2 bufA[INPLACE ? 32 : BA + BA / 32];
  float2* const rawf = reinterpret_cast<float2*>(raw);
  __shared__ float2 bufB[BB + BB / 32];
  __shared__ float2 tw[TWN];

  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  int grp, c;
  if (xcd_groups) {
    const int xcd = b & 7, j = b >> 3;
    grp = xcd + 8 * (j / S0);
    c = j % S0;
  } else {
    grp = b / S0;
    c = b % S0;
  }
  const int f = grp % F;
  const int s = grp / F;
  const int64_t t0 = (int64_t)s * t_per_slice;
  const int64_t t1 = min(T, t0 + t_per_slice);

  // asynchronous copy of tile (t, f) into raw: wave w moves 1 KiB pieces w, w + NT/64, ...
  auto stage = [&](int64_t t) {
    if constexpr (STAGE) {
      const unsigned char* g = static_cast<const unsigned char*>(src) + (t * F + f) * (int64_t)N * SB;
      const int w = tid >> 6, lane = tid & 63;
#pragma unroll
      for (int k = 0; k < (RAWB / 1024 + NT / 64 - 1) / (NT / 64); ++k) {
        const int piece = w + k * (NT / 64);
        if (piece < RAWB / 1024)
          __builtin_amdgcn_global_load_lds(g + piece * 1024 + lane * 16,
                                           (__attribute__((address_space(3))) void*)(raw + piece * 1024), 16, 0, 0);
      }
    }
  };
  if (t0 < t1) stage(t0);

  for (int i = tid; i < TWN; i += NT) tw[i] = tw_glob[i];
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  constexpr int KLAST = 1;
  constexpr int LLAST = SH::L(KLAST);
  constexpr int JOBS_LAST = SH::lines(D - 1, KLAST) * SH::Rw(KLAST);
  static_assert(JOBS_LAST % NT == 0, "last-pass jobs must fill the work-group evenly");
  constexpr int RL = JOBS_LAST / NT;
  constexpr int CPT = RL * LLAST;
  float acc32[CPT];
  double acc64[CPT];
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    acc32[i] = 0.f;
    acc64[i] = 0.0;
  }
  constexpr int TWO[4] = {0, SH::m(0), SH::m(0) + SH::m(1), SH::m(0) + SH::m(1) + SH::m(2)};

  // job -> (residue i, line (o, in)): the inner index is fastest, then the residue, then the outer index
  int blk = 0;
  for (int64_t t = t0; t < t1; ++t) {
    // ---- pass 0: axis 0 from the tile into bufA
    {
      constexpr int K = 0, P = 0;
      constexpr int n = SH::n(K), mm = SH::m(K), L = SH::L(K), RW = SH::Rw(K);
      constexpr int IN = SH::inner(P, K), LINES = SH::lines(P, K), JOBS = LINES * RW;
      constexpr int E = SH::E(K);
      const unsigned char* tile = STAGE ? raw
                                        : static_cast<const unsigned char*>(src) + (t * F + f) * (int64_t)N * SB;
#pragma unroll
      for (int jb = 0; jb < (JOBS + NT - 1) / NT; ++jb) {
        const int job = jb * NT + tid;
        if (JOBS % NT == 0 || job < JOBS) {
          const int in = job % IN, rest = job / IN;
          const int i = rest % RW, o = rest / RW;
          int rho = c + i * SH::step(K);
          if constexpr (IN % 64 == 0) rho = __builtin_amdgcn_readfirstlane(rho);
          float2 z[L];
          const int sb = o * n * IN + in;
          fold<n, mm, L>(z, rho, tw + TWO[K], [&](int p) { return Sample<FMT>::get(tile, sb + p * IN); });
          if constexpr (INPLACE) __syncthreads();  // every column has been read before any is overwritten
          dft<L>(z);
          float2* dst = INPLACE ? rawf : bufA;
#pragma unroll
          for (int q = 0; q < L; ++q) dst[swz((o * E + i * L + q) * IN + in)] = z[q];
        }
      }
    }
    __syncthreads();
    // the tile has been consumed: fetch the next one behind the later passes.  Every barrier after the
    // copy waits for it (the copy writes LDS), so it is issued ahead of the last pass that has no
    // barrier before the end of the sample: right here for D <= 3, after the middle passes for D = 4.
    if (!INPLACE && D <= 3 && t + 1 < t1) stage(t + 1);
    // ---- passes 1 .. D-2: axes D-1 ... 2, LDS -> LDS
    auto mid = [&](auto PC) {
      constexpr int P = decltype(PC)::value;
      constexpr int K = SH::axis_of(P);
      constexpr int n = SH::n(K), mm = SH::m(K), L = SH::L(K), RW = SH::Rw(K);
      constexpr int IN = SH::inner(P, K), LINES = SH::lines(P, K), JOBS = LINES * RW;
      constexpr int E = SH::E(K);
      const float2* sb_ = (P & 1) ? (INPLACE ? rawf : bufA) : bufB;
      float2* db_ = (P & 1) ? bufB : bufA;
#pragma unroll
      for (int jb = 0; jb < (JOBS + NT - 1) / NT; ++jb) {
        const int job = jb * NT + tid;
        if (JOBS % NT == 0 || job < JOBS) {
          const int in = job % IN, rest = job / IN;
          const int i = rest % RW, o = rest / RW;
          float2 z[L];
          const int sb = o * n * IN + in;
          fold<n, mm, L>(z, i, tw + TWO[K], [&](int p) { return sb_[swz(sb + p * IN)]; });
          dft<L>(z);
#pragma unroll
          for (int q = 0; q < L; ++q) db_[swz((o * E + i * L + q) * IN + in)] = z[q];
        }
      }
      __syncthreads();
    };
    if constexpr (D > 2) mid(std::integral_constant<int, 1>{});
    if (INPLACE && t + 1 < t1) stage(t + 1);  // pass 1 has read pass 0's output out of the tile's space
    if constexpr (D > 3) mid(std::integral_constant<int, 2>{});
    if (!INPLACE && D > 3 && t + 1 < t1) stage(t + 1);
    // ---- last pass: axis 1, squared into the registers
    {
      constexpr int P = D - 1, K = KLAST;
      constexpr int n = SH::n(K), mm = SH::m(K), L = SH::L(K), RW = SH::Rw(K);
      constexpr int IN = SH::inner(P, K);
      const float2* sb_ = ((P - 1) & 1) ? bufB : bufA;
#pragma unroll
      for (int jr = 0; jr < RL; ++jr) {
        const int job = jr * NT + tid;
        const int in = job % IN, rest = job / IN;
        const int i = rest % RW, o = rest / RW;
        float2 z[L];
        const int sb = o * n * IN + in;
        fold<n, mm, L>(z, i, tw + TWO[K], [&](int p) { return sb_[swz(sb + p * IN)]; });
        dft<L>(z);
#pragma unroll
        for (int q = 0; q < L; ++q) acc32[jr * L + q] = fmaf(z[q].x, z[q].x, fmaf(z[q].y, z[q].y, acc32[jr * L + q]));
      }
    }
    if constexpr (STAGE) __builtin_amdgcn_s_waitcnt(0);  // this wave's part of the next tile has landed
    __syncthreads();  // next pass 0 overwrites bufA and reads the staged tile
    if (++blk == time_block) {
      blk = 0;
#pragma unroll
      for (int i = 0; i < CPT; ++i) {
        acc64[i] += (double)acc32[i];
        acc32[i] = 0.f;
      }
    }
  }
  // cells in the layout [E_0][E_1]...[E_{D-1}] (row-major); job jr of this thread covers line (o, in) of
  // axis 1 and residue i, its outputs q at (o * E_1 + i L + q) * IN + in.  With `accumulate` the sums are
  // added to what the slot holds (successive launches over time chunks of the same slices).
  if (t0 >= t1 && accumulate) return;
  {
    constexpr int P = D - 1, K = KLAST;
    constexpr int L = SH::L(K), RW = SH::Rw(K), E = SH::E(K);
    constexpr int IN = SH::inner(P, K);
    double* out = partial + ((int64_t)grp * S0 + c) * CELLS;
#pragma unroll
    for (int jr = 0; jr < RL; ++jr) {
      const int job = jr * NT + tid;
      const int in = job % IN, rest = job / IN;
      const int i = rest % RW, o = rest / RW;
#pragma unroll
      for (int q = 0; q < L; ++q) {
        const int cell = (o * E + i * L + q) * IN + in;
        const double v = acc64[jr * L + q] + (double)acc32[jr * L + q];
        out[cell] = accumulate ? out[cell] + v : v;
      }
    }
  }
}

// Shapes with a compile-time kernel.  The planner (api.cpp) must choose the same
// fold moduli and split; launch_fused_ct returns hipErrorInvalidValue otherwise.
struct CtEntry {
  int d, n[4], r[4], s0;
};

template <int FMT, class SH>
static hipError_t launch_one(const void* src, int64_t T, int64_t tps, const float2* tw, double* partial, int F,
                             int n_slices, int time_block, int accumulate, hipStream_t st) {
  const int groups = n_slices * F;
  const int xcd = (groups % 8 == 0) ? 1 : 0;
  // stage tiles of at most 32 KiB through LDS when the source is 16-byte aligned
  constexpr int tile_bytes = SH::N() * Sample<FMT>::bytes;
  const bool aligned = (reinterpret_cast<uintptr_t>(src) & 15) == 0;
  if constexpr (tile_bytes <= 32768 && tile_bytes % 1024 == 0) {
    if (aligned) {
      hipLaunchKernelGGL((fused_ct_fp32_kernel<FMT, SH, 256, true>), dim3(groups * SH::S0), dim3(256), 0, st, src,
                         T, tps, tw, partial, F, xcd, time_block, accumulate);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((fused_ct_fp32_kernel<FMT, SH, 256, false>), dim3(groups * SH::S0), dim3(256), 0, st, src, T,
                     tps, tw, partial, F, xcd, time_block, accumulate);
  return hipGetLastError();
}

// (8,8,4,4): the three-level hierarchy after its 16x16 front; (16,16,16): the
// 16x16-of-16x16 array after one front axis; (4,4,4,4,4) does not fit d <= 4.
// Splits as measured: (8,8,4,4) is fastest at 4 (four work-groups per CU);
// the 64x64 and 128x128 grids lose with a larger split than listed.
using ShapeA = ct::Shape<4, 8, 8, 4, 4, 8, 2, 1, 1, 4>;      // cells 4096, split 4
using ShapeB = ct::Shape<3, 16, 16, 16, 0, 4, 2, 2, 1, 4>;   // cells 8192, split 4
using ShapeC = ct::Shape<2, 32, 32, 0, 0, 8, 8, 1, 1, 1>;    // 32x32: cells 4096
using ShapeD = ct::Shape<2, 64, 64, 0, 0, 8, 8, 1, 1, 2>;      // 64x64: cells 8192, split 2
using ShapeE = ct::Shape<2, 128, 128, 0, 0, 16, 16, 1, 1, 8>;  // 128x128: cells 8192, split 8

const CtEntry kCtShapes[] = {
    {4, {8, 8, 4, 4}, {8, 2, 1, 1}, 4},
    {3, {16, 16, 16, 0}, {4, 2, 2, 1}, 4},
    {2, {32, 32, 0, 0}, {8, 8, 1, 1}, 1},
    {2, {64, 64, 0, 0}, {8, 8, 1, 1}, 2},
    {2, {128, 128, 0, 0}, {16, 16, 1, 1}, 8},
};

int fused_ct_lookup(int d, const int* n) {
  for (int i = 0; i < (int)(sizeof(kCtShapes) / sizeof(kCtShapes[0])); ++i) {
    const CtEntry& e = kCtShapes[i];
    if (e.d != d) continue;
    bool ok = true;
    for (int k = 0; k < d; ++k) ok = ok && e.n[k] == n[k];
    if (ok) return i;
  }
  return -1;
}

void fused_ct_params(int idx, int* r, int* s0) {
  const CtEntry& e = kCtShapes[idx];
  for (int k = 0; k < e.d; ++k) r[k] = e.r[k];
  *s0 = e.s0;
}

hipError_t launch_fused_ct(int idx, int fmt, const void* src, int64_t T, int64_t tps, const float2* tw,
                           double* partial, int F, int n_slices, int time_block, int accumulate, hipStream_t st) {
#define OMNI_CT(SH_)                                                                                          \
  switch (fmt) {                                                                                              \
    case 0: return launch_one<0, SH_>(src, T, tps, tw, partial, F, n_slices, time_block, accumulate, st);                 \
    case 1: return launch_one<1, SH_>(src, T, tps, tw, partial, F, n_slices, time_block, accumulate, st);                 \
    case 2: return launch_one<2, SH_>(src, T, tps, tw, partial, F, n_slices, time_block, accumulate, st);                 \
    default: return hipErrorInvalidValue;                                                                     \
  }
  switch (idx) {
    case 0: OMNI_CT(ShapeA)
    case 1: OMNI_CT(ShapeB)
    case 2: OMNI_CT(ShapeC)
    case 3: OMNI_CT(ShapeD)
    case 4: OMNI_CT(ShapeE)
    default: return hipErrorInvalidValue;
  }
#undef OMNI_CT
}

}  // namespace omni
