// General fused correlator, float32 form, for gfx950 (kernel templates; the instantiations are spread over
// fused_fp32_*.hip so that the build compiles them in parallel).
//
// One work-group owns (time slice s, channel f, split residue c).  For every
// time sample of its slice it
//   1. reads the channel's voltage tile from HBM, decodes it and performs the
//      first axis' fold + short DFT (pass 0) into the LDS working array W,
//   2. transforms the remaining axes but the last in place in W,
//   3. transforms the last axis, squares the modulus (Sec. II.A: "square
//      modulus"; Sec. II.C: "squaring the result") into the LDS power array,
//   4. adds the power of each of its Fourier cells into float32 registers,
//      flushing into float64 registers every time_block samples
//      (time integration, Sec. II.A).
// At the end it writes its float64 partial sums to the partial buffer.  The
// cells a work-group owns never change, so nothing but the voltages and the
// final partial sums touches HBM.
//
// The per-axis transform is the fold + short-DFT form described in plan.hpp.
// Axis shapes are runtime values; only the short-DFT length class (a power of
// two up to 32) and the cells per thread are compile-time.
#pragma once

#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace omni {

enum { FMT_CF32 = 0, FMT_CI8 = 1, FMT_CI4 = 2 };

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c) {
  return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

template <int FMT>
__device__ __forceinline__ float2 load_sample(const void* __restrict__ base, int64_t i);

template <>
__device__ __forceinline__ float2 load_sample<FMT_CF32>(const void* __restrict__ base, int64_t i) {
  return reinterpret_cast<const float2*>(base)[i];
}
template <>
__device__ __forceinline__ float2 load_sample<FMT_CI8>(const void* __restrict__ base, int64_t i) {
  const char2 v = reinterpret_cast<const char2*>(base)[i];
  return make_float2((float)v.x, (float)v.y);
}
template <>
__device__ __forceinline__ float2 load_sample<FMT_CI4>(const void* __restrict__ base, int64_t i) {
  const int8_t v = reinterpret_cast<const int8_t*>(base)[i];
  // high nibble: arithmetic shift of the signed byte; low nibble: move it up first
  return make_float2((float)(v >> 4), (float)((int8_t)(v << 4) >> 4));
}

// Twiddle w_m^{e} for an exponent e >= 0 reduced mod m (mmask = m-1 when m is a power of two).
__device__ __forceinline__ float2 tw_at(const float2* __restrict__ twm, int e, int m, int mmask) {
  return twm[mmask >= 0 ? (e & mmask) : (e % m)];
}

// In-register DFT of length L (runtime, L <= LT) of z, natural output order.
// Powers of two use radix-2 decimation in time; other lengths a direct sum.
// w_L^q = w_m^{q r} is read from the axis' w_m table.
template <int LT>
__device__ __forceinline__ void short_dft(float2 (&z)[LT], int L, int r, int m, int mmask,
                                          const float2* __restrict__ twm) {
  if (L == LT) {
    // bit-reversal permutation (compile-time)
#pragma unroll
    for (int i = 0; i < LT; ++i) {
      int j = 0;
#pragma unroll
      for (int b = 1, rb = LT >> 1; b < LT; b <<= 1, rb >>= 1)
        if (i & b) j |= rb;
      if (j > i) {
        float2 t = z[i];
        z[i] = z[j];
        z[j] = t;
      }
    }
#pragma unroll
    for (int s = 1; s < LT; s <<= 1) {
#pragma unroll
      for (int k = 0; k < LT; k += 2 * s) {
#pragma unroll
        for (int j = 0; j < s; ++j) {
          float2 v = z[k + j + s];
          if (j != 0) v = cmul(v, twm[j * (LT / (2 * s)) * r]);
          const float2 u = z[k + j];
          z[k + j] = cadd(u, v);
          z[k + j + s] = csub(u, v);
        }
      }
    }
  } else {
    float2 out[LT];
#pragma unroll
    for (int q = 0; q < LT; ++q) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int j = 0; j < LT; ++j)
        if (q < L && j < L) acc = cfma(z[j], tw_at(twm, q * j * r, m, mmask), acc);
      out[q] = acc;
    }
#pragma unroll
    for (int q = 0; q < LT; ++q) z[q] = out[q];
  }
}

// One pass over one axis.  SRC: 0 = LDS working array, 1 = global voltage tile.
// SINK: 0 = LDS working array (in place), 1 = LDS power array (|X|^2).  Inlined: as calls, the schedule
// structs they take by reference and their register arrays went through per-lane scratch memory.
template <int LT, int SRC, int SINK, int FMT, int NT>
__device__ __forceinline__ void run_pass_t(const PassP& ps, const AxisP& a, int rho0, const void* __restrict__ src, int64_t tile,
                           float2* W, float* Pw, const float2* __restrict__ tw) {
  const float2* twm = tw + a.tw_off;
  const int m = a.m, mmask = (m & (m - 1)) == 0 ? m - 1 : -1;
  const int L = a.L, r = a.r, n = a.n;
  const int stride_src = SRC ? a.in_stride : a.w_stride;
  const bool inplace = (SRC == 0 && SINK == 0);
  for (int q0 = 0; q0 < ps.jobs; q0 += NT) {
    const int q = q0 + (int)threadIdx.x;
    const bool active = q < ps.jobs;
    float2 z[LT];
    int dst_off = 0;
    if (active) {
      const int line = q / a.R, i = q - line * a.R;
      int rem = line, src_off = 0;
      for (int o = 0; o < ps.n_other; ++o) {
        const int e = ps.ext[o];
        const int idx = rem % e;
        rem /= e;
        src_off += idx * ps.src_str[o];
        dst_off += idx * (SINK ? ps.p_str[o] : ps.w_str[o]);
      }
      const int rho = rho0 + i * a.rho_step;
      dst_off += i * L * (SINK ? a.p_stride : a.w_stride);
      // fold: z_j = sum_l x[j + l L] w_m^{rho (j + l L)}
#pragma unroll
      for (int j = 0; j < LT; ++j) {
        float2 acc = make_float2(0.f, 0.f);
        if (j < L) {
          for (int p = j; p < n; p += L) {
            float2 v;
            if (SRC)
              v = load_sample<FMT>(src, tile + src_off + (int64_t)p * stride_src);
            else
              v = W[src_off + p * stride_src];
            acc = rho ? cfma(v, tw_at(twm, rho * p, m, mmask), acc) : cadd(acc, v);
          }
        }
        z[j] = acc;
      }
      short_dft<LT>(z, L, r, m, mmask, twm);
    }
    if (inplace) __syncthreads();
    if (active) {
      if (SINK) {
#pragma unroll
        for (int k = 0; k < LT; ++k)
          if (k < L) Pw[dst_off + k * a.p_stride] = z[k].x * z[k].x + z[k].y * z[k].y;
      } else {
#pragma unroll
        for (int k = 0; k < LT; ++k)
          if (k < L) W[dst_off + k * a.w_stride] = z[k];
      }
    }
    if (inplace) __syncthreads();
  }
}

template <int SRC, int SINK, int FMT, int NT>
__device__ __forceinline__ void run_pass(const PassP& ps, const AxisP& a, int rho0, const void* __restrict__ src, int64_t tile,
                         float2* W, float* Pw, const float2* __restrict__ tw) {
  const int L = a.L;
  if (L <= 1)
    run_pass_t<1, SRC, SINK, FMT, NT>(ps, a, rho0, src, tile, W, Pw, tw);
  else if (L <= 2)
    run_pass_t<2, SRC, SINK, FMT, NT>(ps, a, rho0, src, tile, W, Pw, tw);
  else if (L <= 4)
    run_pass_t<4, SRC, SINK, FMT, NT>(ps, a, rho0, src, tile, W, Pw, tw);
  else if (L <= 8)
    run_pass_t<8, SRC, SINK, FMT, NT>(ps, a, rho0, src, tile, W, Pw, tw);
  else if (L <= 16)
    run_pass_t<16, SRC, SINK, FMT, NT>(ps, a, rho0, src, tile, W, Pw, tw);
  else
    run_pass_t<32, SRC, SINK, FMT, NT>(ps, a, rho0, src, tile, W, Pw, tw);
}

template <int FMT, int CPT, int NT>
__global__ __launch_bounds__(NT) void fused_fp32_kernel(const void* __restrict__ src, int64_t T, int64_t t_per_slice,
                                                        const float2* __restrict__ tw_glob,
                                                        double* __restrict__ partial, FusedP P) {
  extern __shared__ float2 smem[];
  float2* W = smem;
  float* Pw = reinterpret_cast<float*>(W + P.w_elems);
  float2* tw = reinterpret_cast<float2*>(Pw + CPT * NT);

  // Block -> (slice, channel, split residue).  With the XCD-aware mapping the
  // n_split work-groups of one (slice, channel) land on the same XCD (blocks
  // are dealt round-robin over the 8 XCDs), so the re-reads of the channel's
  // voltage tile are served by that XCD's L2.
  const int b = blockIdx.x;
  int grp, c;
  if (P.xcd_groups) {
    const int xcd = b & 7, j = b >> 3;
    grp = xcd + 8 * (j / P.n_split);
    c = j % P.n_split;
  } else {
    grp = b / P.n_split;
    c = b % P.n_split;
  }
  const int f = grp % P.F;
  const int s = grp / P.F;

  for (int i = threadIdx.x; i < P.n_tw; i += NT) tw[i] = tw_glob[i];

  const int64_t t0 = (int64_t)s * t_per_slice;
  const int64_t t1 = min(T, t0 + t_per_slice);

  float acc32[CPT];
  double acc64[CPT];
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    acc32[i] = 0.f;
    acc64[i] = 0.0;
  }
  int blk = 0;
  const int d = P.d;
  for (int64_t t = t0; t < t1; ++t) {
    __syncthreads();  // W / Pw free, twiddles visible
    const int64_t tile = (t * P.F + f) * (int64_t)P.N;
    const PassP& p0 = P.pass[0];
    const AxisP& a0 = P.ax[p0.axis];
    if (d == 1) {
      run_pass<1, 1, FMT, NT>(p0, a0, (c / a0.split_div) % a0.split, src, tile, W, Pw, tw);
    } else {
      run_pass<1, 0, FMT, NT>(p0, a0, (c / a0.split_div) % a0.split, src, tile, W, Pw, tw);
      __syncthreads();
      for (int p = 1; p < d - 1; ++p) {
        const PassP& pp = P.pass[p];
        const AxisP& ap = P.ax[pp.axis];
        run_pass<0, 0, FMT, NT>(pp, ap, (c / ap.split_div) % ap.split, src, tile, W, Pw, tw);
      }
      const PassP& pl = P.pass[d - 1];
      const AxisP& al = P.ax[pl.axis];
      run_pass<0, 1, FMT, NT>(pl, al, (c / al.split_div) % al.split, src, tile, W, Pw, tw);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int cell = (int)threadIdx.x + i * NT;
      if (cell < P.cells_wg) acc32[i] += Pw[cell];
    }
    if (++blk == P.time_block) {
      blk = 0;
#pragma unroll
      for (int i = 0; i < CPT; ++i) {
        acc64[i] += (double)acc32[i];
        acc32[i] = 0.f;
      }
    }
  }
  double* out = partial + ((int64_t)grp * P.n_split + c) * P.cells_wg;
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int cell = (int)threadIdx.x + i * NT;
    if (cell < P.cells_wg) out[cell] = acc64[i] + (double)acc32[i];
  }
}

// ---------------------------------------------------------------------------
// Launch of one instantiation (format, cells per thread).
// ---------------------------------------------------------------------------
constexpr int kFusedNT = 256;

template <int FMT, int CPT>
static hipError_t launch_fused_t(const void* src, int64_t T, int64_t tps, const float2* tw, double* partial,
                                 const FusedP& P, int grid, size_t lds, hipStream_t st) {
  auto k = fused_fp32_kernel<FMT, CPT, kFusedNT>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kFusedNT), lds, st, src, T, tps, tw, partial, P);
  return hipGetLastError();
}

// One translation unit per sample format and group of cells-per-thread values (each returns
// hipErrorInvalidValue for a value outside its group).
hipError_t launch_fused_fp32_cf32_lo(int cpt, const void* src, int64_t T, int64_t tps, const float2* tw,
                                     double* partial, const FusedP& P, int grid, size_t lds, hipStream_t st);
hipError_t launch_fused_fp32_cf32_hi(int cpt, const void* src, int64_t T, int64_t tps, const float2* tw,
                                     double* partial, const FusedP& P, int grid, size_t lds, hipStream_t st);
hipError_t launch_fused_fp32_ci8_lo(int cpt, const void* src, int64_t T, int64_t tps, const float2* tw,
                                    double* partial, const FusedP& P, int grid, size_t lds, hipStream_t st);
hipError_t launch_fused_fp32_ci8_hi(int cpt, const void* src, int64_t T, int64_t tps, const float2* tw,
                                    double* partial, const FusedP& P, int grid, size_t lds, hipStream_t st);
hipError_t launch_fused_fp32_ci4_lo(int cpt, const void* src, int64_t T, int64_t tps, const float2* tw,
                                    double* partial, const FusedP& P, int grid, size_t lds, hipStream_t st);
hipError_t launch_fused_fp32_ci4_hi(int cpt, const void* src, int64_t T, int64_t tps, const float2* tw,
                                    double* partial, const FusedP& P, int grid, size_t lds, hipStream_t st);

}  // namespace omni
