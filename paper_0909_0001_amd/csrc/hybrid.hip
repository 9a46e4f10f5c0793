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
// Only the Hermitian half of the pairs is summed: S_qp[kappa] =
// conj(S_pq[kappa]) at the same cell, so the other half is written as the
// conjugate.  A thread with row block rb (rows p = 2 rb + r, r = 0, 1) takes
// the pairs (p, (p + d) mod P) for d = 0 .. P/2: each unordered pair is then
// one thread's exactly once (offset d and P - d name the same pair, and only
// d <= P/2 is taken), except d = P/2, which rows p and p + P/2 would both take
// and only p < P/2 keeps.  Every thread does P + 2 pair sums (one of them
// dropped in half the threads) instead of 2 P, and touches the P/2 + 2 tiles
// q = 2 rb + e mod P, e = 0 .. P/2 + 1, so every register index is a
// compile-time constant.
//
// xengine_kernel: a thread owns one cell kappa and a row block, its P + 2
// complex float32 sums over the chunk's samples, then float64
// read-modify-writes of S (the pair and, off the diagonal, its conjugate).
// The row-block threads of one cell are adjacent lanes, so the loads of a cell
// and sample are shared through the cache; consecutive cells are consecutive
// addresses.

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace omni {
namespace {

constexpr int kXeThreads = 256;

// The P/2 + 1 pair sums of row r of a row block: acc[r][d] += t_r conj(t_{r + d}), t_e = Y of tile 2 rb + e mod P.
template <int P>
__device__ __forceinline__ void half_pairs_add(float2 (&acc)[2][P / 2 + 1], const float2 (&v)[P / 2 + 2]) {
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const float2 a = v[r];
#pragma unroll
    for (int d = 0; d <= P / 2; ++d) {
      const float2 b = v[r + d];
      acc[r][d].x = fmaf(a.x, b.x, fmaf(a.y, b.y, acc[r][d].x));
      acc[r][d].y = fmaf(a.y, b.x, fmaf(-a.x, b.y, acc[r][d].y));
    }
  }
}

// Adds the row block's sums into S[f][p][q][kappa] (element stride Mp between (p, q) planes), and their conjugates
// into S[f][q][p][kappa] off the diagonal; the duplicate d = P/2 of rows p >= P/2 is dropped.
template <int P>
__device__ __forceinline__ void half_pairs_store(const float2 (&acc)[2][P / 2 + 1], int rb, double2* Sf, int64_t Mp,
                                                 int64_t kappa, int accumulate) {
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int p = 2 * rb + r;
#pragma unroll
    for (int d = 0; d <= P / 2; ++d) {
      if (d == P / 2 && p >= P / 2) continue;
      const int q = (p + d) & (P - 1);
#pragma unroll
      for (int c = 0; c < (d ? 2 : 1); ++c) {
        double2* sp = Sf + ((int64_t)(c ? q : p) * P + (c ? p : q)) * Mp + kappa;
        double2 o = make_double2((double)acc[r][d].x, c ? -(double)acc[r][d].y : (double)acc[r][d].y);
        if (accumulate) {
          const double2 old = *sp;
          o.x += old.x;
          o.y += old.y;
        }
        *sp = o;
      }
    }
  }
}

template <int P>
__global__ __launch_bounds__(kXeThreads) void xengine_kernel(const float2* __restrict__ Y, int64_t Tc, int F,
                                                             int64_t Mp, double2* __restrict__ S, int accumulate) {
  constexpr int NRB = P / 2;               // row blocks per cell
  constexpr int CELLS = kXeThreads / NRB;  // cells per work-group
  constexpr int E = P / 2 + 2;             // tiles a row block touches
  const int tid = threadIdx.x;
  const int rb = tid % NRB;
  const int64_t kappa = (int64_t)blockIdx.x * CELLS + tid / NRB;
  const int f = blockIdx.y;
  if (kappa >= Mp) return;
  int64_t off[E];
#pragma unroll
  for (int e = 0; e < E; ++e) off[e] = (int64_t)((2 * rb + e) & (P - 1)) * Mp;
  float2 acc[2][P / 2 + 1];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int d = 0; d <= P / 2; ++d) acc[r][d] = make_float2(0.f, 0.f);
  for (int64_t t = 0; t < Tc; ++t) {
    const float2* y = Y + ((t * F + f) * (int64_t)P) * Mp + kappa;
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = y[off[e]];
    half_pairs_add<P>(acc, v);
  }
  half_pairs_store<P>(acc, rb, S + (int64_t)f * P * P * Mp, Mp, kappa, accumulate);
}

__global__ void narrow_kernel(const double2* __restrict__ src, float2* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = make_float2((float)src[i].x, (float)src[i].y);
}

template <int P>
hipError_t launch_xe(const float2* Y, int64_t Tc, int F, int64_t Mp, double2* S, int accumulate, hipStream_t st) {
  constexpr int CELLS = kXeThreads / (P / 2);
  const int64_t blocks = (Mp + CELLS - 1) / CELLS;
  if (blocks > INT32_MAX || F < 1 || F > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL((xengine_kernel<P>), dim3((unsigned)blocks, (unsigned)F), dim3(kXeThreads), 0, st, Y, Tc, F,
                     Mp, S, accumulate);
  return hipGetLastError();
}


// Fused y-axis transform + X-engine, for P n_y <= 256 (m_y = 2 n_y, P m_y <= 512).  Input: the x-axis front
// pass' output Y1[t][f][p][kappa_x][i_y] (complex float32).  A work-group owns R = 256 / (P n_y) rows kappa_x
// of one channel, 256 threads.  Per sample:
//   load   thread (row, p, i_y) brings one input value (eight samples ahead in registers) into LDS;
//   y-DFT  the same thread forms outputs kappa_y = k and k + n_y (k = its i_y) of line (row, p) of the
//          zero-padded m_y-point transform: with w = exp(-2 pi i / m_y), w^{(k + n_y) i} = (-1)^i w^{k i}, so
//          the even- and odd-i partial sums E, O give E + O and E - O; the thread's n_y twiddles w^{k i} stay
//          in registers (float32, from float64);
//   pairs  thread (row, kappa_y, row block of 2 tiles) adds its P + 2 cross products (the Hermitian half).
// Two barriers per two samples, LDS double-buffered.  Saves the y-axis front pass and the round trip of its
// output through HBM.
template <int P, int NY>
__global__ __launch_bounds__(kXeThreads) void xengine_fused_kernel(const float2* __restrict__ Y1, int64_t Tc, int F,
                                                                   int mx, const float2* __restrict__ twy,
                                                                   double2* __restrict__ S, int accumulate) {
  constexpr int MY = 2 * NY;
  constexpr int UNITS = MY * (P / 2);  // pair-stage threads per row
  constexpr int R = kXeThreads / UNITS;
  static_assert(R * P * NY == kXeThreads, "one input value and one output pair per thread");
  constexpr int kTb = 2;                              // samples per barrier pair
  __shared__ float2 in_buf[2][kTb][kXeThreads];       // [row][p][i_y]
  __shared__ float2 out_buf[2][kTb][2 * kXeThreads];  // [row][p][kappa_y]
  const int tid = threadIdx.x;
  const int f = blockIdx.y;
  const int kx0 = blockIdx.x * R;
  // (row, p, i_y) of this thread: its input value and its output pair (kappa_y = i_y, i_y + n_y)
  const int er = tid / (P * NY), ep = (tid / NY) % P, ei = tid % NY;
  const int64_t slab = (int64_t)P * mx * NY;
  const int64_t in_off = ((int64_t)ep * mx + kx0 + er) * NY + ei;
  float2 wk[NY];
#pragma unroll
  for (int i = 0; i < NY; ++i) wk[i] = twy[(ei * i) & (MY - 1)];
  // pair-stage unit of this thread: cell (row ur, kappa_y = uk), row block rb; LDS offsets of the tiles it touches.
  // kappa_y runs fastest over the lanes, so a read of tile e by 32 lanes is 256 contiguous bytes (with the row
  // block fastest, the lanes' tiles were 2 MY values apart: every lane of a read in the same banks).
  const int ur = tid / UNITS, rb = (tid % UNITS) / MY, uk = tid % MY;
  constexpr int E = P / 2 + 2;
  int off[E];
#pragma unroll
  for (int e = 0; e < E; ++e) off[e] = (ur * P + ((2 * rb + e) & (P - 1))) * MY + uk;
  float2 acc[2][P / 2 + 1];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int d = 0; d <= P / 2; ++d) acc[r][d] = make_float2(0.f, 0.f);
  constexpr int kPf = 8;
  float2 pf[kPf];
#pragma unroll
  for (int j = 0; j < kPf; ++j) pf[j] = j < Tc ? Y1[((int64_t)j * F + f) * slab + in_off] : make_float2(0.f, 0.f);
  int b = 0;
#pragma unroll 1
  for (int64_t t = 0; t < Tc; t += kTb, b ^= 1) {
    const int nt = (int)min<int64_t>(kTb, Tc - t);
#pragma unroll
    for (int s = 0; s < kTb; ++s) in_buf[b][s][tid] = pf[s];
#pragma unroll
    for (int j = 0; j < kPf - kTb; ++j) pf[j] = pf[j + kTb];
#pragma unroll
    for (int s = 0; s < kTb; ++s)
      pf[kPf - kTb + s] = t + kPf + s < Tc ? Y1[((t + kPf + s) * F + f) * slab + in_off] : make_float2(0.f, 0.f);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kTb; ++s) {
      const float2* line = &in_buf[b][s][(er * P + ep) * NY];
      float2 e = make_float2(0.f, 0.f), o = make_float2(0.f, 0.f);
#pragma unroll
      for (int i = 0; i < NY; ++i) {
        const float2 v = line[i];
        float2& z = (i & 1) ? o : e;
        z.x = fmaf(v.x, wk[i].x, fmaf(-v.y, wk[i].y, z.x));
        z.y = fmaf(v.x, wk[i].y, fmaf(v.y, wk[i].x, z.y));
      }
      float2* dst = &out_buf[b][s][(er * P + ep) * MY + ei];
      dst[0] = make_float2(e.x + o.x, e.y + o.y);
      dst[NY] = make_float2(e.x - o.x, e.y - o.y);
    }
    __syncthreads();
    for (int s = 0; s < nt; ++s) {
      const float2* plane = out_buf[b][s];
      float2 v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = plane[off[e]];
      half_pairs_add<P>(acc, v);
    }
  }
  const int64_t Mp = (int64_t)mx * MY;
  const int64_t kappa = (int64_t)(kx0 + ur) * MY + uk;
  half_pairs_store<P>(acc, rb, S + (int64_t)f * P * P * Mp, Mp, kappa, accumulate);
}

template <int P, int NY>
hipError_t launch_xf(const float2* Y1, int64_t Tc, int F, int mx, const float2* twy, double2* S, int accumulate,
                     hipStream_t st) {
  if constexpr (P * NY > kXeThreads || NY < 1) {
    return hipErrorInvalidValue;
  } else {
    constexpr int R = kXeThreads / (2 * NY * (P / 2));
    if (mx % R != 0 || F < 1 || F > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL((xengine_fused_kernel<P, NY>), dim3((unsigned)(mx / R), (unsigned)F), dim3(kXeThreads), 0, st,
                       Y1, Tc, F, mx, twy, S, accumulate);
    return hipGetLastError();
  }
}

template <int P>
hipError_t launch_xf_ny(const float2* Y1, int64_t Tc, int F, int mx, int ny, const float2* twy, double2* S,
                        int accumulate, hipStream_t st) {
  switch (ny) {
    case 1: return launch_xf<P, 1>(Y1, Tc, F, mx, twy, S, accumulate, st);
    case 2: return launch_xf<P, 2>(Y1, Tc, F, mx, twy, S, accumulate, st);
    case 4: return launch_xf<P, 4>(Y1, Tc, F, mx, twy, S, accumulate, st);
    case 8: return launch_xf<P, 8>(Y1, Tc, F, mx, twy, S, accumulate, st);
    case 16: return launch_xf<P, 16>(Y1, Tc, F, mx, twy, S, accumulate, st);
    case 32: return launch_xf<P, 32>(Y1, Tc, F, mx, twy, S, accumulate, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// The fused form applies when P n_y <= 256 (n_y a power of two up to 32).
bool xengine_fused_ok(int P, int ny) { return P >= 2 && ny >= 1 && ny <= 32 && (ny & (ny - 1)) == 0 && P * ny <= kXeThreads; }

hipError_t launch_xengine_fused(const float2* Y1, int64_t Tc, int F, int P, int mx, int ny, const float2* twy,
                                double2* S, int accumulate, hipStream_t st) {
  switch (P) {
    case 2: return launch_xf_ny<2>(Y1, Tc, F, mx, ny, twy, S, accumulate, st);
    case 4: return launch_xf_ny<4>(Y1, Tc, F, mx, ny, twy, S, accumulate, st);
    case 8: return launch_xf_ny<8>(Y1, Tc, F, mx, ny, twy, S, accumulate, st);
    case 16: return launch_xf_ny<16>(Y1, Tc, F, mx, ny, twy, S, accumulate, st);
    case 32: return launch_xf_ny<32>(Y1, Tc, F, mx, ny, twy, S, accumulate, st);
    default: return hipErrorInvalidValue;
  }
}

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
