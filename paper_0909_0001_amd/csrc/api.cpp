// C ABI of the hierarchical-grid correlator: validation, planning, device
// resources and launch sequencing.  See include/omniscope.h for the contract.
#include "omniscope.h"

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "direct.hpp"
#include "fold.hpp"
#include "plan.hpp"

namespace omni {
hipError_t launch_fused_fp32(int fmt, int cpt, const void* src, int64_t T, int64_t tps, const float2* tw,
                             double* partial, const FusedP& P, int grid, size_t lds, hipStream_t st);
hipError_t launch_reduce_scatter(const double* partial, const int32_t* kmap, double* A, int n_slices, int F,
                                 int n_split, int cells_wg, int64_t M, int accumulate, hipStream_t st);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t st);
hipError_t launch_inverse_axis(bool real_in, bool last, const void* src, void* dst, const double2* twi,
                               int64_t outer, int m, int n, int64_t inner, double scale, hipStream_t st);
hipError_t launch_twiddles(const int32_t* desc_dev, int n_tables, float2* tw32, double2* tw64, hipStream_t st);
hipError_t launch_fused8x4_fp32(int fmt, const void* src, int64_t T, int64_t tps, const float2* tw16, double* partial,
                                int F, int n_slices, int time_block, hipStream_t st);
hipError_t launch_fused8x4_mixed(int fmt, const void* src, int64_t T, int64_t tps,
                                 const float2* tw16, double* partial, int F, int n_slices, int time_block,
                                 hipStream_t st);
hipError_t launch_front_axis(int fmt, const void* src, void* dst, const float2* twm, int64_t tiles, int64_t outer,
                             int n, int m, int r, int64_t inner, int64_t src_tile, int64_t dst_tile, hipStream_t st,
                             bool half16, float scale);
hipError_t launch_front2_16x16(int fmt, const void* src, void* dst, const float2* tw32, int64_t tiles, int64_t rest,
                               float scale, hipStream_t st);
int fused_ct_lookup(int d, const int* n);
void fused_ct_params(int idx, int* r, int* s0);
hipError_t launch_fused_ct(int idx, int fmt, const void* src, int64_t T, int64_t tps, const float2* tw,
                           double* partial, int F, int n_slices, int time_block, int accumulate, hipStream_t st);
int fused16x3_cell(int cell);
int fused8844_cell(int cell);
hipError_t launch_fused8844_mixed(const void* src, int64_t T, int64_t tps, const float2* tw16, const float2* tw8,
                                  double* partial, int F, int n_slices, int time_block, int accumulate,
                                  double out_scale, hipStream_t st);
hipError_t launch_fused16x3_mixed(const void* src, int64_t T, int64_t tps, const float2* tw, double* partial, int F,
                                  int n_slices, int time_block, int accumulate, double out_scale, hipStream_t st);
int grid128_cell(int s, int cell);
int grid64_cell(int cell);
int grid32_cell(int cell);
hipError_t launch_grid128_mixed(const void* src, int64_t T, int64_t tps, const float2* tw256, double* partial, int F,
                                int n_slices, int time_block, double out_scale, hipStream_t st);
hipError_t launch_grid64_mixed(const void* src, int64_t T, int64_t tps, const float2* tw128, double* partial, int F,
                               int n_slices, int time_block, double out_scale, hipStream_t st);
hipError_t launch_grid32_mixed(const void* src, int64_t T, int64_t tps, const float2* tw64, double* partial, int F,
                               int n_slices, int time_block, double out_scale, hipStream_t st);
hipError_t launch_fengine(const void* raw, int64_t N, int64_t T, int F, const void* gains, bool ci8, void* out,
                          hipStream_t st);
hipError_t launch_xengine(const float2* Y, int64_t Tc, int F, int P, int64_t Mp, double2* S, int accumulate,
                          hipStream_t st);
hipError_t launch_narrow(const double2* src, float2* dst, int64_t n, hipStream_t st);
bool xengine_fused_ok(int P, int ny);
hipError_t launch_xengine_fused(const float2* Y1, int64_t Tc, int F, int P, int mx, int ny, const float2* twy,
                                double2* S, int accumulate, hipStream_t st);
hipError_t launch_even_cells(const double* A, double* E, int64_t rows, int na, int nb, int axes, hipStream_t st);
}  // namespace omni

using omni::AxisP;
using omni::FusedP;
using omni::PassP;

namespace {

thread_local std::string g_last_error;

// OMNI_LOG_LEVEL (environment, read once): 0 or unset = silent, 1 = every error a call returns, 2 = also each
// plan's description and every autotuner decision.  Lines go to stderr, prefixed "omniscope:".
int log_level() {
  static const int level = [] {
    const char* e = std::getenv("OMNI_LOG_LEVEL");
    return e ? std::atoi(e) : 0;
  }();
  return level;
}

void log_msg(int level, const char* fmt, ...) {
  if (log_level() < level) return;
  char line[1024];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(line, sizeof line, fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "omniscope: %s\n", line);
}

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  log_msg(1, "error %d: %s", code, msg.c_str());
  return code;
}

// A roctx range (shown by rocprofv3 --marker-trace) around an entry point.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

constexpr int kNT = 256;              // threads per fused work-group
constexpr int kMaxCPT = 32;           // Fourier cells per thread
constexpr int kCellsMax = kNT * kMaxCPT;
constexpr size_t kLdsMax = 160 * 1024;
constexpr int64_t kMaxN = int64_t(1) << 22;
constexpr size_t kPartialBudget = size_t(512) << 20;

// A fused-kernel schedule for a set of axes and channels.
struct FusedSetup {
  FusedP fp{};
  int cpt = 0;               // cells per thread (general kernel)
  size_t lds = 0;            // dynamic LDS bytes (general kernel)
  std::vector<int32_t> kmap; // cell of (split residue, work-group cell) -> natural frequency index
  int F = 0;                 // channels seen by the kernel
  int64_t N = 0, M = 0;      // samples and Fourier cells per channel tile
};

struct ArrayPlan {
  int levels = 0;
  std::vector<int> dims;    // original axes, 2 per level
  std::vector<double> A;    // [levels][2][2] or empty
  int F = 0;
  std::vector<int> n;       // axes with n > 1 (or a single axis when N == 1), in order
  std::vector<int> m;       // transform length per axis of n: 2 n (zero-padded), or n for a beam axis
  int nbeam = 0;            // beam-space plan: the last nbeam axes of n (the lowest level's) are pointings
  bool beams = false;       // beam-space plan (the lowest level's two axes are pointing indices in the output)
  bool beam_sub = false;    // beam-space plan run on the zero-padded transform: pointing b is its Fourier cell
                            // 2b along the lowest level's axes (nbeam counts those axes; the forward pass is
                            // the ordinary one)
  int64_t N = 0, M = 0, n_out = 0;
  FusedSetup fs;            // schedule of the fused kernel (all axes, or the axes after the front)
  int kernel = 0;  // 0: general; 1: 8x8x8x8 float32; 2: 8x8x8x8 mixed (MFMA); 3: compile-time shape (float32);
                   // 4: (16,16,16) behind a front pass, mixed (MFMA), float16 front workspace;
                   // 5: (8,8,4,4) behind two front passes, mixed (MFMA), float16 front workspace;
                   // 6, 7, 8: single-level 128 x 128, 64 x 64, 32 x 32, mixed (MFMA), 4-bit samples
  int ct_index = -1;         // entry of the compile-time shape table (kernel 3)
  int lcap = 32;             // longest short DFT the general kernel may use (autotuned)
  int wg_target = 1024;      // work-groups the time slicing aims for (general and sliced kernels; autotuned)
  int tb = 0;                // float32 block of the sliced kernels (0: the plan's time_block; autotuned)
  double tuned_ms = 0.0;     // best candidate's time in the autotuner (0: not tuned)
  // front mode: the first n_front axes are transformed by front passes over HBM
  int n_front = 0;
  bool single_split = true;   // the cells are divided along the first-processed axis only
  std::vector<int> front_r;   // fold modulus of each front axis
  int front_tw_base = 0;      // offset of the remaining axes' twiddles
  int64_t chunk_T = 0;        // time samples per front chunk
  int64_t chunk_cap = 0;      // caller's cap on chunk_T (0: none)
  int64_t y_bytes[2] = {0, 0};  // bytes of the two front workspaces (front pass k writes d_y[k % 2])
  std::vector<int32_t> tw_desc_fwd, tw_desc_inv;
  std::vector<int> inv_off;  // per axis offset into the twiddle tables
  int n_tw = 0;
  int max_slices = 1;
  int last_slices = 1;
  int inv_group = 1;         // channels per inverse-transform group
  // device resources
  float2* d_tw32 = nullptr;
  double2* d_tw64 = nullptr;
  int32_t* d_kmap = nullptr;
  double* d_A = nullptr;
  double* d_partial = nullptr;
  float2* d_ws[2] = {nullptr, nullptr};  // inverse-transform intermediates (complex float32)
  float2* d_y[2] = {nullptr, nullptr};
  // direct N^2 correlator (set up by its first call): per-channel int64 half-sums, block pairs, block boxes
  unsigned long long* d_dc_G = nullptr;
  int32_t* d_dc_pairs = nullptr;
  int32_t* d_dc_blk = nullptr;
  int64_t dc_pairs = 0;
  bool dc_geom_ok = false;   // dc_geom / dc_pairs derived and within the kernel's limits
  omni::DirectGeom dc_geom;
};

}  // namespace

constexpr int kTimingRing = 256;

constexpr int kStages = 4;  // forward, reduce, inverse, whole call
// Per-launch events of the main forward kernel (OMNI_STAGE_KERNEL): kKernRing calls x kKernMax launches.
constexpr int kKernRing = 32;
constexpr int kKernMax = 16;
// Front mode: each of the two workspaces holds at most kFrontBytes (8 GiB: the partial sums are
// read-modified-written once per chunk, so fewer, larger chunks save that traffic), and a chunk at most
// kChunkMax samples.
constexpr int64_t kFrontBytes = int64_t(8) << 30;
constexpr int64_t kFrontBytesMixed = int64_t(16) << 30;  // float16 front workspaces of the mixed form
constexpr int64_t kChunkMax = 256;

struct omni_plan_s {
  std::vector<ArrayPlan> arrays;
  bool timing = false;
  // [call % ring][stage][begin/end]
  std::vector<hipEvent_t> ev;
  // [call % kKernRing][launch][begin/end] and the launches recorded per call
  std::vector<hipEvent_t> kev;
  std::vector<int> kev_n;
  // OMNI_PLAN_GRAPH: one branch stream per array, fork / join events, the
  // captured graph and the call it was captured for
  bool graph = false;
  std::vector<hipStream_t> branch;
  std::vector<hipEvent_t> join;
  hipStream_t capture = nullptr;
  hipEvent_t fork = nullptr;
  hipEvent_t g_done = nullptr;  // recorded after every launch of the graph
  hipGraph_t g = nullptr;
  hipGraphExec_t gx = nullptr;
  int64_t g_T = -1;
  uint32_t g_flags = 0;
  std::vector<const void*> g_volt;
  std::vector<void*> g_vis;
  int64_t n_calls = 0;
  omni_dtype dtype = OMNI_CF32;
  omni_form form = OMNI_FORM_FP32;
  int time_block = 64;
  bool time_block_set = false;  // the caller chose time_block (the autotuner keeps it)
  bool host_only = false;
  int device = -1;
  int tune = OMNI_TUNE_OFF;
  std::string tune_cache;  // file of tuned schedules ("" = none)
};

namespace {

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// Kernels with a fixed shape that split the time axis into slices (one partial-sum set each): 1 (8x8x8x8
// float32), 2 (8x8x8x8 mixed) and 6-8 (single-level 128 x 128, 64 x 64, 32 x 32 mixed).
bool sliced_kernel(int k) { return k == 1 || k == 2 || (k >= 6 && k <= 8); }

// Default work-group target of the time slicing, per kernel: 8x8x8x8 float32: three 48 KiB work-groups a CU,
// two rounds over 256 CUs; 8x8x8x8 mixed: one 112 KiB work-group a CU, one round; 128 x 128: one 128 KiB
// work-group a CU, about four rounds; 64 x 64: one 96 KiB work-group a CU, four rounds; 32 x 32: 256 threads
// and 12 KiB, about five work-groups a CU, two rounds.
int default_wg_target(int k) {
  switch (k) {
    case 1: return 1536;
    case 2: return 256;
    case 8: return 2560;
    default: return 1024;
  }
}


int64_t prod(const std::vector<int>& v) {
  int64_t p = 1;
  for (int x : v) p *= x;
  return p;
}

// Antenna positions r = sum_l A_l (i_lx, i_ly) must be distinct (Sec. II.D: every grid
// point has a unique index tuple).  Positions are compared after rounding to a
// relative grain of 1e-9 of the layout's extent.
int check_geometry(const ArrayPlan& ap) {
  if (ap.A.empty()) return OMNI_OK;
  for (double v : ap.A)
    if (!std::isfinite(v)) return fail(OMNI_E_GEOM, "lattice matrix has a non-finite entry");
  const int64_t N = ap.N;
  if (N > (int64_t(1) << 22)) return OMNI_OK;
  std::vector<std::pair<double, double>> pos((size_t)N);
  const int d = (int)ap.dims.size();
  double ext = 0.0;
  for (int64_t a = 0; a < N; ++a) {
    int64_t rem = a;
    std::vector<int> idx(d);
    for (int k = d - 1; k >= 0; --k) {
      idx[k] = (int)(rem % ap.dims[k]);
      rem /= ap.dims[k];
    }
    double x = 0, y = 0;
    for (int l = 0; l < ap.levels; ++l) {
      const double* Al = &ap.A[4 * l];
      x += Al[0] * idx[2 * l] + Al[1] * idx[2 * l + 1];
      y += Al[2] * idx[2 * l] + Al[3] * idx[2 * l + 1];
    }
    pos[(size_t)a] = {x, y};
    ext = std::max(ext, std::max(std::fabs(x), std::fabs(y)));
  }
  const double grain = std::max(ext, 1.0) * 1e-9;
  std::vector<std::pair<long long, long long>> q(pos.size());
  for (size_t i = 0; i < pos.size(); ++i)
    q[i] = {std::llround(pos[i].first / grain), std::llround(pos[i].second / grain)};
  std::sort(q.begin(), q.end());
  for (size_t i = 1; i < q.size(); ++i)
    if (q[i] == q[i - 1]) return fail(OMNI_E_GEOM, "two antennas share a position (index tuples must be unique)");
  return OMNI_OK;
}

// Choose the fused schedule for axes n (F channels; the axes' forward twiddle
// tables start at tw_base in the plan's table).  See plan.hpp for the fold +
// short-DFT form.  With single_split the cells may only be divided along the
// first-processed axis (a split on a later axis repeats the earlier passes in
// every work-group of the split).
int plan_fused_axes(const std::vector<int>& n, int F, int tw_base, bool single_split, int lcap, FusedSetup& fs,
                    std::string* why, const int* r_force = nullptr, int s0_force = 0, const int* m_in = nullptr) {
  const int d = (int)n.size();
  FusedP& P = fs.fp;
  std::memset(&P, 0, sizeof(P));
  fs.F = F;
  fs.N = prod(n);
  fs.M = 1;
  for (int k = 0; k < (int)n.size(); ++k) fs.M *= m_in ? m_in[k] : 2 * n[k];
  P.d = d;
  P.F = F;
  P.N = (int32_t)fs.N;
  std::vector<int> m(d), r(d), L(d), R(d), step(d), E(d);
  std::vector<int64_t> in_str(d);
  in_str[d - 1] = 1;
  for (int k = d - 2; k >= 0; --k) in_str[k] = in_str[k + 1] * n[k + 1];
  for (int k = 0; k < d; ++k) {
    m[k] = m_in ? m_in[k] : 2 * n[k];
    int rr = 1;
    while (m[k] / rr > lcap && (m[k] % (2 * rr)) == 0) rr *= 2;
    if (m[k] / rr > omni::kMaxL) {
      *why = "axis length " + std::to_string(n[k]) + " has an odd factor above 16";
      return OMNI_E_SHAPE;
    }
    r[k] = rr;
  }
  // Processing order: the outermost axis is loaded and folded first, then the
  // others from the innermost outwards; the last one is squared.
  std::vector<int> order;
  order.push_back(0);
  for (int k = d - 1; k >= 1; --k) order.push_back(k);
  std::vector<int> split(d, 1), split_div(d, 1);
  int64_t n_split = 1;
  if (s0_force > 0) {
    split[0] = s0_force;
    n_split = s0_force;
  }
  for (int p = 0; p < (single_split ? 1 : d) && fs.M / n_split > kCellsMax && s0_force == 0; ++p) {
    const int k = order[p];
    while (fs.M / n_split > kCellsMax && m[k] % (2 * split[k]) == 0) {
      split[k] *= 2;
      n_split *= 2;
    }
  }
  if (fs.M / n_split > kCellsMax) {
    *why = "per-channel Fourier grid cannot be divided into work-group shares of <= 8192 cells";
    return OMNI_E_SHAPE;
  }
  {
    int64_t div = 1;
    for (int k = d - 1; k >= 0; --k) {
      split_div[k] = (int)div;
      div *= split[k];
    }
  }
  for (int k = 0; k < d; ++k) {
    r[k] = r_force ? r_force[k] : std::max(r[k], split[k]);
    L[k] = m[k] / r[k];
    R[k] = r[k] / split[k];
    step[k] = split[k];
    E[k] = R[k] * L[k];
  }
  const int last = order[d - 1];
  // LDS layouts: W holds every axis but the last at its transformed extent; Pw holds all cells.
  std::vector<int64_t> w_str(d), p_str(d);
  int64_t ws = 1, pst = 1;
  for (int k = d - 1; k >= 0; --k) {
    w_str[k] = ws;
    ws *= (k == last && d > 1) ? n[k] : E[k];
    p_str[k] = pst;
    pst *= E[k];
  }
  const int64_t cells = pst;
  int cpt = 1;
  while ((int64_t)cpt * kNT < cells) cpt *= 2;
  if (cpt > kMaxCPT) {
    *why = "work-group cell share too large";
    return OMNI_E_SHAPE;
  }
  fs.cpt = cpt;
  P.n_split = (int32_t)n_split;
  P.cells_wg = (int32_t)cells;
  P.w_elems = (int32_t)(d > 1 ? ws : 1);
  int off = 0;
  for (int k = 0; k < d; ++k) {
    AxisP& a = P.ax[k];
    a.n = n[k];
    a.m = m[k];
    a.r = r[k];
    a.L = L[k];
    a.R = R[k];
    a.rho_step = step[k];
    a.split = split[k];
    a.split_div = split_div[k];
    a.E = E[k];
    a.w_stride = (int32_t)w_str[k];
    a.p_stride = (int32_t)p_str[k];
    a.in_stride = (int32_t)in_str[k];
    a.tw_off = off;  // relative to tw_base: the kernel gets the table from tw_base on
    off += m[k];
  }
  (void)tw_base;
  P.n_tw = off;
  for (int p = 0; p < d; ++p) {
    PassP& ps = P.pass[p];
    const int ax = order[p];
    ps.axis = ax;
    int no = 0;
    int64_t lines = 1;
    for (int k = d - 1; k >= 0; --k) {
      if (k == ax) continue;
      bool done = false;
      for (int q = 0; q < p; ++q) done = done || order[q] == k;
      const int ext = done ? E[k] : n[k];
      ps.ext[no] = ext;
      ps.w_str[no] = (int32_t)w_str[k];
      ps.src_str[no] = (int32_t)(p == 0 ? in_str[k] : w_str[k]);
      ps.p_str[no] = (int32_t)p_str[k];
      lines *= ext;
      ++no;
    }
    ps.n_other = no;
    ps.lines = (int32_t)lines;
    ps.jobs = (int32_t)(lines * R[ax]);
  }
  fs.lds = (size_t)P.w_elems * 8 + (size_t)cpt * kNT * 4 + (size_t)P.n_tw * 8;
  if (fs.lds > kLdsMax) {
    *why = "LDS working set exceeds 160 KiB";
    return OMNI_E_SHAPE;
  }
  // Cell -> natural frequency index (row-major over these axes), for every split residue.
  fs.kmap.assign((size_t)fs.M, 0);
  std::vector<int64_t> nat_str(d);
  int64_t sst = 1;
  for (int k = d - 1; k >= 0; --k) {
    nat_str[k] = sst;
    sst *= m[k];
  }
  for (int c = 0; c < n_split; ++c) {
    for (int64_t cell = 0; cell < cells; ++cell) {
      int64_t rem = cell, nat = 0;
      for (int k = d - 1; k >= 0; --k) {
        const int pos = (int)(rem % E[k]);
        rem /= E[k];
        const int i = pos / L[k], q = pos % L[k];
        const int rho = (int)((c / split_div[k]) % split[k]) + i * step[k];
        const int kappa = r[k] * q + rho;
        nat += kappa * nat_str[k];
      }
      fs.kmap[(size_t)(c * cells + cell)] = (int32_t)nat;
    }
  }
  return OMNI_OK;
}

// Bytes of the two front workspaces for the plan's chunk: front pass k writes d_y[k % 2] (complex float32,
// or float16 (re, im) where the pass feeds a matrix-core kernel: the last pass before kernel 4, every pass
// before kernel 5); the fused 16 x 16 front pass of kernel 5 writes the last pass' output into d_y[1].
void size_front_workspaces(ArrayPlan& ap) {
  ap.y_bytes[0] = ap.y_bytes[1] = 0;
  const int s = ap.n_front;
  int64_t mm = 1, nn = ap.N;
  for (int k = 0; k < s; ++k) {
    mm *= 2 * ap.n[k];
    nn /= ap.n[k];
    const bool h16 = (ap.kernel == 4 && k == s - 1) || ap.kernel == 5;
    const int64_t b = ap.chunk_T * ap.F * mm * nn * (h16 ? 4 : 8);
    ap.y_bytes[k & 1] = std::max(ap.y_bytes[k & 1], b);
  }
}

// Matrix-core kernels behind the front passes: kernel 4 for the (16,16,16)
// grid behind one front pass, kernel 5 for (8,8,4,4) behind two.  Work-group
// = (slice, front channel), all the channel's cells, cell order given by
// fused16x3_cell / fused8844_cell.  The last front pass writes float16 planar
// operands (scaled by 1/n of its axis), which halves that workspace: twice the
// samples per chunk.
void plan_mixed_behind_front(ArrayPlan& ap, int kernel) {
  ap.kernel = kernel;
  FusedSetup& fs = ap.fs;
  const int s = ap.n_front;
  int64_t ms = 1, ns = 1;
  for (int k = 0; k < s; ++k) {
    ms *= 2 * ap.n[k];
    ns *= ap.n[k];
  }
  const int64_t rest_n = ap.N / ns;
  fs.N = rest_n;
  fs.M = ap.M / ms;
  fs.fp.n_split = 1;
  fs.fp.cells_wg = (int32_t)fs.M;
  fs.kmap.assign((size_t)fs.M, 0);
  for (int c = 0; c < (int)fs.M; ++c)
    fs.kmap[(size_t)c] = kernel == 4 ? omni::fused16x3_cell(c) : omni::fused8844_cell(c);
  // what `describe` reports for the matrix-core kernels (static LDS of the kernels)
  fs.cpt = 32;
  fs.lds = kernel == 4 ? 99840 : 50176;
  // bytes per time sample of the last (float16) front output
  const int64_t per_t = (int64_t)ap.F * ms * rest_n * 4;
  ap.chunk_T = std::max<int64_t>(1, std::min<int64_t>(kChunkMax, kFrontBytesMixed / per_t));
  if (ap.chunk_cap > 0) ap.chunk_T = std::min(ap.chunk_T, ap.chunk_cap);
  size_front_workspaces(ap);
}

// The 8x8x8x8 float32 kernel: work-group = (slice, channel, residue c of axis 0 mod 8);
// its cell i (of 32) in thread tid is written at i * 256 + tid and holds
// line l = tid + 256 (i / 16), output o = i % 16 of the last (axis 1) transform.
// Positions p in [0,16) along axes 1..3 hold kappa = 2 (p % 8) + p / 8.
void plan_fused8x4(ArrayPlan& ap) {
  ap.kernel = 1;
  FusedP& P = ap.fs.fp;
  P.n_split = 8;
  P.cells_wg = 8192;
  ap.fs.cpt = 32;
  auto kap = [](int p) { return 2 * (p & 7) + (p >> 3); };
  for (int c = 0; c < 8; ++c) {
    for (int i = 0; i < 32; ++i) {
      for (int tid = 0; tid < 256; ++tid) {
        const int l = tid + 256 * (i >> 4), o = i & 15;
        const int k0 = c + 8 * (l >> 8);
        const int k1 = kap(o), k2 = kap((l >> 4) & 15), k3 = kap(l & 15);
        ap.fs.kmap[(size_t)(c * 8192 + i * 256 + tid)] = ((k0 * 16 + k1) * 16 + k2) * 16 + k3;
      }
    }
  }
}

// The 8x8x8x8 mixed-precision kernel: work-group = (slice, channel, residue h of
// kappa_3 mod 2), 1024 threads; cell idx (of 32) of thread tid is written at
// idx * 1024 + tid.  With wave = tid / 64, lane = tid % 64, col = lane % 32,
// hh = lane / 32, idx = ((cc * 2 + tt) * 2 + i') * 4 + j and idx2 = 32 tt + col
// it holds kappa_0 = 8 i' + 4 hh + j, kappa_1 = wave, kappa_2 = 8 cc + idx2 % 8,
// kappa_3 = 2 (idx2 / 8) + h.
void plan_fused8x4_mixed(ArrayPlan& ap) {
  ap.kernel = 2;
  FusedP& P = ap.fs.fp;
  P.n_split = 2;
  P.cells_wg = 32768;
  ap.fs.cpt = 32;
  ap.fs.lds = 114688;
  for (int h = 0; h < 2; ++h) {
    for (int idx = 0; idx < 32; ++idx) {
      for (int tid = 0; tid < 1024; ++tid) {
        const int wave = tid >> 6, lane = tid & 63, col = lane & 31, hh = lane >> 5;
        const int cc = idx >> 4, tt = (idx >> 3) & 1, ip = (idx >> 2) & 1, j = idx & 3;
        const int idx2 = 32 * tt + col;
        const int k0 = 8 * ip + 4 * hh + j, k1 = wave, k2 = 8 * cc + (idx2 & 7), k3 = 2 * (idx2 >> 3) + h;
        ap.fs.kmap[(size_t)(h * 32768 + idx * 1024 + tid)] = ((k0 * 16 + k1) * 16 + k2) * 16 + k3;
      }
    }
  }
}

// The single-level 128 x 128 grid in the mixed form: work-group = (slice, channel, half s of axis 1's
// first-stage outputs), 1024 threads, 32768 cells each in the order given by grid128_cell.
// The 64 x 64 and 32 x 32 grids (kernels 7 and 8): one work-group per (slice, channel) owns all cells.
void plan_grid128(ArrayPlan& ap) {
  ap.kernel = 6;
  FusedSetup& fs = ap.fs;
  fs.F = ap.F;
  fs.N = ap.N;
  fs.M = ap.M;
  fs.fp.n_split = 2;
  fs.fp.cells_wg = 32768;
  fs.cpt = 32;
  fs.lds = 153600;
  fs.kmap.assign((size_t)ap.M, 0);
  for (int c = 0; c < 2; ++c)
    for (int cell = 0; cell < 32768; ++cell) fs.kmap[(size_t)(c * 32768 + cell)] = omni::grid128_cell(c, cell);
}

void plan_grid_small(ArrayPlan& ap, int kernel) {
  ap.kernel = kernel;
  FusedSetup& fs = ap.fs;
  fs.F = ap.F;
  fs.N = ap.N;
  fs.M = ap.M;
  fs.fp.n_split = 1;
  fs.fp.cells_wg = (int32_t)ap.M;
  fs.cpt = 16;
  fs.lds = kernel == 7 ? 98304 : 12288;
  fs.kmap.assign((size_t)ap.M, 0);
  for (int cell = 0; cell < (int)ap.M; ++cell)
    fs.kmap[(size_t)cell] = kernel == 7 ? omni::grid64_cell(cell) : omni::grid32_cell(cell);
}

// Front mode: the first s axes are transformed by front passes over HBM, after
// which every outer Fourier index is a channel of the remaining axes.  A front
// axis needs a power-of-two padded length of at most 64 (short DFTs of <= 32).
bool front_axis_ok(int n) { return is_pow2(2 * n) && 2 * n <= 64; }

int plan_front(ArrayPlan& ap, std::string* why) {
  const int d = (int)ap.n.size();
  int64_t MS = 1, NS = 1;
  for (int s = 1; s < d; ++s) {
    if (s - 1 >= d - ap.nbeam || !front_axis_ok(ap.n[s - 1])) break;
    MS *= 2 * ap.n[s - 1];
    NS *= ap.n[s - 1];
    std::vector<int> rest(ap.n.begin() + s, ap.n.end());
    std::string w2;
    if ((int64_t)ap.F * MS > INT32_MAX / 64) break;
    int tw_base = 0;
    for (int k = 0; k < s; ++k) tw_base += 2 * ap.n[k];
    FusedSetup fs;
    if (plan_fused_axes(rest, (int)(ap.F * MS), tw_base, true, ap.lcap, fs, &w2, nullptr, 0, ap.m.data() + s) ==
        OMNI_OK) {
      ap.fs = std::move(fs);
      ap.n_front = s;
      ap.front_tw_base = tw_base;
      ap.front_r.assign(s, 1);
      for (int k = 0; k < s; ++k) ap.front_r[k] = std::max(1, 2 * ap.n[k] / 16);
      // time chunk: the largest front output (after the last front pass) <= kFrontBytes
      const int64_t per_t = (int64_t)ap.F * MS * (ap.N / NS) * (int64_t)sizeof(float2);
      ap.chunk_T = std::max<int64_t>(1, std::min<int64_t>(kChunkMax, kFrontBytes / per_t));
      if (ap.chunk_cap > 0) ap.chunk_T = std::min(ap.chunk_T, ap.chunk_cap);
      size_front_workspaces(ap);
      return OMNI_OK;
    }
  }
  *why = "per-channel Fourier grid too large and no front split applies";
  return OMNI_E_SHAPE;
}

int build_array_core(ArrayPlan& ap, int levels, const int32_t* dims, const double* A, int32_t nchan, omni_form form,
                     omni_dtype dtype, bool beams) {
  if (levels < 1 || levels > omni::kMaxD / 2) return fail(OMNI_E_SHAPE, "levels must be in [1, 4]");
  if (!dims) return fail(OMNI_E_INVAL, "dims is NULL");
  if (nchan < 1) return fail(OMNI_E_INVAL, "nchan must be >= 1");
  ap.levels = levels;
  ap.dims.assign(dims, dims + 2 * levels);
  ap.F = nchan;
  int64_t N = 1;
  for (int v : ap.dims) {
    if (v < 1) return fail(OMNI_E_SHAPE, "every grid dimension must be >= 1");
    if (v > 4096) return fail(OMNI_E_SHAPE, "grid dimension above 4096");
    N *= v;
    if (N > kMaxN) return fail(OMNI_E_SHAPE, "more than 2^22 antennas");
  }
  ap.N = N;
  if (A) ap.A.assign(A, A + 4 * levels);
  ap.n.clear();
  for (int v : ap.dims)
    if (v > 1) ap.n.push_back(v);
  if (ap.n.empty()) ap.n.push_back(1);
  // beam-space plan: the lowest level's axes (the last two) are transformed without padding and never
  // inverted; its axes of more than one antenna are the last nbeam entries of n
  ap.nbeam = 0;
  if (beams) {
    if (levels < 2) return fail(OMNI_E_SHAPE, "a beam-space plan needs at least one level above the blocks");
    ap.nbeam = (ap.dims[(size_t)(2 * levels - 2)] > 1) + (ap.dims[(size_t)(2 * levels - 1)] > 1);
    int64_t outer = 1;
    for (int k = 0; k < 2 * levels - 2; ++k) outer *= ap.dims[(size_t)k];
    if (outer < 2) return fail(OMNI_E_SHAPE, "a beam-space plan needs more than one block");
  }
  ap.m.assign(ap.n.size(), 0);
  ap.M = 1;
  ap.n_out = 1;
  for (size_t k = 0; k < ap.n.size(); ++k) {
    const bool beam = (int)k >= (int)ap.n.size() - ap.nbeam;
    ap.m[k] = beam ? ap.n[k] : 2 * ap.n[k];
    ap.M *= ap.m[k];
    ap.n_out *= beam ? ap.n[k] : 2 * ap.n[k] - 1;
  }
  int rc = check_geometry(ap);
  if (rc) return rc;
  const int d = (int)ap.n.size();
  // forward (float32) and inverse (float64) twiddle tables, one per axis
  ap.tw_desc_fwd.clear();
  ap.tw_desc_inv.clear();
  ap.inv_off.assign(d, 0);
  int off = 0;
  for (int k = 0; k < d; ++k) {
    ap.tw_desc_fwd.insert(ap.tw_desc_fwd.end(), {ap.m[k], -1, off});
    ap.tw_desc_inv.insert(ap.tw_desc_inv.end(), {ap.m[k], +1, off});
    ap.inv_off[k] = off;
    off += ap.m[k];
  }
  ap.n_tw = off;
  std::string why, why2;
  ap.n_front = 0;
  rc = plan_fused_axes(ap.n, ap.F, 0, true, ap.lcap, ap.fs, &why, nullptr, 0, ap.m.data());
  // a beam-space plan whose grid needs a split takes front passes over its outer axes where they apply: each
  // work-group then owns whole pointing grids of one outer Fourier index instead of repeating the outer
  // passes in every work-group of the split
  if (rc == OMNI_OK && ap.nbeam > 0 && ap.fs.fp.n_split > 1) {
    ArrayPlan trial = ap;
    if (plan_front(trial, &why2) == OMNI_OK) ap = std::move(trial);
  }
  if (rc) rc = plan_front(ap, &why2);
  if (rc) {
    // last resort: residue splits along several axes (correct, repeats early passes)
    rc = plan_fused_axes(ap.n, ap.F, 0, false, ap.lcap, ap.fs, &why, nullptr, 0, ap.m.data());
    if (rc) return fail(rc, why + "; " + why2);
    ap.single_split = false;
  }
  // the fixed-shape kernels all assume zero-padded axes: a beam-space plan keeps the general kernel
  if (ap.nbeam > 0) {
    ap.max_slices = (int)std::max<size_t>(1, std::min<size_t>(1024, kPartialBudget / ((size_t)ap.F * ap.M * 8)));
    ap.inv_group = (int)std::max<int64_t>(1, std::min<int64_t>(ap.F, (int64_t(1) << 30) / (ap.M * 8)));
    return OMNI_OK;
  }
  const bool eight4 = ap.n == std::vector<int>{8, 8, 8, 8};
  if (!eight4 && ap.single_split) {
    // a compile-time-shape kernel for the axes the fused kernel sees (all, or those after the front)
    const std::vector<int> axes = ap.n_front ? std::vector<int>(ap.n.begin() + ap.n_front, ap.n.end()) : ap.n;
    const int idx = omni::fused_ct_lookup((int)axes.size(), axes.data());
    if (idx >= 0) {
      int rr[4] = {1, 1, 1, 1}, s0 = 1;
      omni::fused_ct_params(idx, rr, &s0);
      FusedSetup fs;
      std::string w3;
      if (plan_fused_axes(axes, ap.fs.F, 0, true, ap.lcap, fs, &w3, rr, s0) == OMNI_OK) {
        ap.fs = std::move(fs);
        ap.kernel = 3;
        ap.ct_index = idx;
      }
    }
  }
  if (form == OMNI_FORM_FP32 && eight4) plan_fused8x4(ap);
  if (form == OMNI_FORM_MIXED && eight4 && dtype != OMNI_CF32) plan_fused8x4_mixed(ap);
  if (form == OMNI_FORM_MIXED && dtype != OMNI_CF32 && ap.n_front == 1 &&
      std::vector<int>(ap.n.begin() + 1, ap.n.end()) == std::vector<int>{16, 16, 16})
    plan_mixed_behind_front(ap, 4);
  if (form == OMNI_FORM_MIXED && dtype != OMNI_CF32 && ap.n_front == 2 &&
      std::vector<int>(ap.n.begin() + 2, ap.n.end()) == std::vector<int>{8, 8, 4, 4})
    plan_mixed_behind_front(ap, 5);
  if (form == OMNI_FORM_MIXED && dtype == OMNI_CI4 && ap.n_front == 0 && ap.n == std::vector<int>{128, 128})
    plan_grid128(ap);
  if (form == OMNI_FORM_MIXED && dtype == OMNI_CI4 && ap.n_front == 0 && ap.n == std::vector<int>{64, 64})
    plan_grid_small(ap, 7);
  if (form == OMNI_FORM_MIXED && dtype == OMNI_CI4 && ap.n_front == 0 && ap.n == std::vector<int>{32, 32})
    plan_grid_small(ap, 8);
  if (sliced_kernel(ap.kernel)) ap.wg_target = default_wg_target(ap.kernel);
  const size_t per_slice = (size_t)ap.F * (size_t)ap.M * sizeof(double);
  ap.max_slices = (int)std::max<size_t>(1, std::min<size_t>(1024, kPartialBudget / per_slice));
  // inverse in groups of channels whose complex float32 workspace fits 1 GiB per buffer
  ap.inv_group = (int)std::max<int64_t>(1, std::min<int64_t>(ap.F, (int64_t(1) << 30) / (ap.M * 8)));
  return OMNI_OK;
}

// A beam-space plan (Appendix A steps 4-5).  The unpadded transform of a block, B_b = sum_j x_j
// exp(-2 pi i b.j / n), is the zero-padded one at the even cells: B_b = X[2b] (m = 2n).  So where the ordinary
// plan of the same grid has a fixed-shape kernel (matrix-core or compile-time shape), the beam-space plan runs
// that kernel unchanged and keeps the even cells of the lowest level's axes before the inverse along the outer
// axes; otherwise the general kernel transforms those axes without padding (a quarter of the cells).
int build_array(ArrayPlan& ap, int levels, const int32_t* dims, const double* A, int32_t nchan, omni_form form,
                omni_dtype dtype, bool beams) {
  if (!beams) return build_array_core(ap, levels, dims, A, nchan, form, dtype, false);
  if (levels < 2 || levels > omni::kMaxD / 2)
    return fail(OMNI_E_SHAPE, "a beam-space plan needs at least one level above the blocks");
  if (!dims) return fail(OMNI_E_INVAL, "dims is NULL");
  int64_t outer = 1;
  for (int k = 0; k < 2 * levels - 2; ++k) outer *= dims[k];
  if (outer < 2) return fail(OMNI_E_SHAPE, "a beam-space plan needs more than one block");
  const int64_t cap = ap.chunk_cap;
  int rc = build_array_core(ap, levels, dims, A, nchan, form, dtype, false);
  if (rc) return rc;
  ap.beams = true;
  if (ap.kernel != 0) {
    ap.beam_sub = true;
    ap.nbeam = (dims[2 * levels - 2] > 1) + (dims[2 * levels - 1] > 1);
    ap.n_out = 1;
    for (size_t k = 0; k < ap.n.size(); ++k)
      ap.n_out *= (int)k >= (int)ap.n.size() - ap.nbeam ? ap.n[k] : 2 * ap.n[k] - 1;
    return OMNI_OK;
  }
  ap = ArrayPlan();
  ap.chunk_cap = cap;
  rc = build_array_core(ap, levels, dims, A, nchan, form, dtype, true);
  ap.beams = true;
  return rc;
}

void free_array(ArrayPlan& ap) {
  hipFree(ap.d_tw32);
  hipFree(ap.d_tw64);
  hipFree(ap.d_kmap);
  hipFree(ap.d_A);
  hipFree(ap.d_partial);
  hipFree(ap.d_ws[0]);
  hipFree(ap.d_ws[1]);
  hipFree(ap.d_y[0]);
  hipFree(ap.d_y[1]);
  hipFree(ap.d_dc_G);
  hipFree(ap.d_dc_pairs);
  hipFree(ap.d_dc_blk);
  ap.d_dc_G = nullptr;
  ap.d_dc_pairs = ap.d_dc_blk = nullptr;
  ap.d_tw32 = nullptr;
  ap.d_tw64 = nullptr;
  ap.d_kmap = nullptr;
  ap.d_A = nullptr;
  ap.d_partial = nullptr;
  ap.d_ws[0] = ap.d_ws[1] = nullptr;
  ap.d_y[0] = ap.d_y[1] = nullptr;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(e_ == hipErrorOutOfMemory ? OMNI_E_NOMEM : OMNI_E_HIP,                  \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                      \
  } while (0)

int alloc_array(ArrayPlan& ap) {
  const size_t accA = (size_t)ap.F * ap.M * sizeof(double);
  HIP_TRY(hipMalloc(&ap.d_tw32, (size_t)ap.n_tw * sizeof(float2)));
  HIP_TRY(hipMalloc(&ap.d_tw64, (size_t)ap.n_tw * sizeof(double2)));
  HIP_TRY(hipMalloc(&ap.d_kmap, ap.fs.kmap.size() * sizeof(int32_t)));
  HIP_TRY(hipMalloc(&ap.d_A, accA));
  HIP_TRY(hipMalloc(&ap.d_partial, accA * (size_t)ap.max_slices));
  const size_t ws = (size_t)ap.inv_group * ap.M * sizeof(float2);
  HIP_TRY(hipMalloc(&ap.d_ws[0], ws));
  HIP_TRY(hipMalloc(&ap.d_ws[1], ws));
  if (ap.n_front > 0) {
    for (int b = 0; b < 2; ++b)
      if (ap.y_bytes[b] > 0) HIP_TRY(hipMalloc(&ap.d_y[b], (size_t)ap.y_bytes[b]));
  }
  HIP_TRY(hipMemcpy(ap.d_kmap, ap.fs.kmap.data(), ap.fs.kmap.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  int32_t* d_desc = nullptr;
  const size_t nd = std::max(ap.tw_desc_fwd.size(), ap.tw_desc_inv.size());
  HIP_TRY(hipMalloc(&d_desc, nd * sizeof(int32_t)));
  hipError_t e = hipMemcpy(d_desc, ap.tw_desc_fwd.data(), ap.tw_desc_fwd.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = omni::launch_twiddles(d_desc, (int)ap.tw_desc_fwd.size() / 3, ap.d_tw32, nullptr, 0);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess)
    e = hipMemcpy(d_desc, ap.tw_desc_inv.data(), ap.tw_desc_inv.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = omni::launch_twiddles(d_desc, (int)ap.tw_desc_inv.size() / 3, nullptr, ap.d_tw64, 0);
  if (e == hipSuccess) e = omni::launch_fill_f64(ap.d_A, (int64_t)ap.F * ap.M, 0.0, 0);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  hipFree(d_desc);
  if (e != hipSuccess) return fail(OMNI_E_HIP, std::string("twiddle setup: ") + hipGetErrorString(e));
  return OMNI_OK;
}

int check_device(int* dev) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return fail(OMNI_E_NODEV, "no HIP device");
  HIP_TRY(hipGetDevice(dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, *dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(OMNI_E_NODEV, std::string("device is ") + prop.gcnArchName + ", library is built for gfx950");
  return OMNI_OK;
}

int fmt_of(omni_dtype t) { return (int)t; }

size_t sample_bytes(omni_dtype t) { return t == OMNI_CF32 ? 8 : t == OMNI_CI8 ? 2 : 1; }

hipEvent_t stage_event(omni_plan_s* p, int stage, int end) {
  return p->ev[(size_t)(((p->n_calls % kTimingRing) * kStages + stage) * 2 + end)];
}

// Records the stage's begin event before the first array and its end event after the last.
void mark(omni_plan_s* p, int stage, int end, bool edge, hipStream_t st) {
  if (p->timing && edge) hipEventRecord(stage_event(p, stage, end), st);
}

// Brackets one launch of the main forward kernel (begin: end = 0, end: end = 1) on `st` (timing plans that
// are not graph plans; at most kKernMax launches per call).
void kmark(omni_plan_s* p, int end, hipStream_t st) {
  if (!p->timing || p->graph) return;
  const int slot = (int)(p->n_calls % kKernRing);
  const int k = p->kev_n[(size_t)slot];
  if (k >= kKernMax) return;
  hipEventRecord(p->kev[(size_t)((slot * kKernMax + k) * 2 + end)], st);
  if (end) p->kev_n[(size_t)slot] = k + 1;
}

// General fused kernel over T samples of `src` (format fmt) with setup fs; float64
// partial sums into ap.d_partial; returns the number of time slices used.
int launch_general(ArrayPlan& ap, const FusedSetup& fs, int fmt, const void* src, int64_t T, int time_block,
                   const float2* tw, hipStream_t st, int* slices) {
  FusedP P = fs.fp;
  const int64_t per_slice_groups = (int64_t)fs.F * P.n_split;
  int64_t ns = std::max<int64_t>(1, (ap.wg_target + per_slice_groups - 1) / per_slice_groups);
  ns = std::min<int64_t>(ns, ap.max_slices);
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, T / 4));
  const int64_t tps = (T + ns - 1) / ns;
  ns = (T + tps - 1) / tps;
  P.n_slices = (int32_t)ns;
  P.time_block = time_block;
  const int64_t groups = ns * fs.F;
  P.xcd_groups = (groups % 8 == 0) ? 1 : 0;
  const int64_t grid = groups * P.n_split;
  if (grid > INT32_MAX) return fail(OMNI_E_SHAPE, "grid too large");
  *slices = (int)ns;
  HIP_TRY(omni::launch_fused_fp32(fmt, fs.cpt, src, T, tps, tw, ap.d_partial, P, (int)grid, fs.lds, st));
  return OMNI_OK;
}

// Compile-time-shape kernel over T samples; same slicing policy as the general kernel.  With
// `accumulate` the kernel adds into the partial sums (at most max_ns slices, those of an earlier launch).
int launch_ct(ArrayPlan& ap, int fmt, const void* src, int64_t T, int time_block, const float2* tw, hipStream_t st,
              int* slices, int accumulate = 0, int64_t max_ns = INT32_MAX) {
  const int64_t per_slice_groups = (int64_t)ap.fs.F * ap.fs.fp.n_split;
  int64_t ns = std::max<int64_t>(1, (ap.wg_target + per_slice_groups - 1) / per_slice_groups);
  ns = std::min<int64_t>(ns, ap.max_slices);
  ns = std::min<int64_t>(ns, max_ns);
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, T / 4));
  const int64_t tps = (T + ns - 1) / ns;
  ns = (T + tps - 1) / tps;
  if (ns * per_slice_groups > INT32_MAX) return fail(OMNI_E_SHAPE, "grid too large");
  *slices = (int)ns;
  HIP_TRY(omni::launch_fused_ct(ap.ct_index, fmt, src, T, tps, tw, ap.d_partial, ap.fs.F, (int)ns, time_block,
                                accumulate, st));
  return OMNI_OK;
}

// Launch a sliced kernel over T samples: about `target` work-groups (fewer when T is short or the partial
// sums would not fit), float32 blocks of `tb` samples.  *slices receives the slice count.
int launch_sliced(omni_plan_s* p, ArrayPlan& ap, const void* volt, int64_t T, int64_t target, int tb,
                  hipStream_t st, int* slices) {
  const int64_t per_slice_groups = (int64_t)ap.F * (ap.kernel == 1 ? 8 : (ap.kernel == 2 || ap.kernel == 6) ? 2 : 1);
  int64_t ns = std::max<int64_t>(1, (target + per_slice_groups / 2) / per_slice_groups);
  ns = std::min<int64_t>(ns, ap.max_slices);
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, T / 8));
  const int64_t tps = (T + ns - 1) / ns;
  ns = (T + tps - 1) / tps;
  *slices = (int)ns;
  const int fmt = fmt_of(p->dtype);
  switch (ap.kernel) {
    case 1:
      HIP_TRY(omni::launch_fused8x4_fp32(fmt, volt, T, tps, ap.d_tw32, ap.d_partial, ap.F, (int)ns, tb, st));
      break;
    case 2:
      HIP_TRY(omni::launch_fused8x4_mixed(fmt, volt, T, tps, ap.d_tw32, ap.d_partial, ap.F, (int)ns, tb, st));
      break;
    case 6:  // the four stages scale by 1/16, 1/8, 1/8, 1/16: |X|^2 carries 2^-28
      HIP_TRY(omni::launch_grid128_mixed(volt, T, tps, ap.d_tw32, ap.d_partial, ap.F, (int)ns, tb, 268435456.0, st));
      break;
    case 7:  // four stages of 1/8: 2^-24
      HIP_TRY(omni::launch_grid64_mixed(volt, T, tps, ap.d_tw32, ap.d_partial, ap.F, (int)ns, tb, 16777216.0, st));
      break;
    case 8:  // two stages of 1/32: 2^-20
      HIP_TRY(omni::launch_grid32_mixed(volt, T, tps, ap.d_tw32, ap.d_partial, ap.F, (int)ns, tb, 1048576.0, st));
      break;
    default:
      return fail(OMNI_E_STATE, "not a sliced kernel");
  }
  return OMNI_OK;
}

int correlate_array(omni_plan_s* p, ArrayPlan& ap, const void* volt, int64_t T, void* vis, hipStream_t st,
                    uint32_t flags, int stage) {
  const bool accumulate = (flags & OMNI_NO_RESET) != 0;
  if (stage == 0 && T > 0 && ap.n_front > 0) {
    // Front mode: per chunk of samples, front passes to HBM, then the fused
    // kernel on the remaining axes.  The general kernel's partial sums are
    // reduced into the accumulator after every chunk; the compile-time-shape
    // kernel adds the later chunks into the first chunk's slices, reduced once.
    const int s = ap.n_front;
    int first_slices = 0;
    for (int64_t c0 = 0; c0 < T; c0 += ap.chunk_T) {
      const int64_t tc = std::min<int64_t>(ap.chunk_T, T - c0);
      const void* cur = static_cast<const char*>(volt) + (size_t)(c0 * ap.F * ap.N) * sample_bytes(p->dtype);
      int fmt = fmt_of(p->dtype);
      int64_t outer = 1, inner = ap.N, tw_off = 0;
      // the three-level mixed path: both 16 x 16 front passes in one kernel (8-bit or 4-bit samples, 16-byte
      // aligned rows); else one pass per axis
      int k0 = 0;
      const int64_t rest = ap.N / 256;
      if (ap.kernel == 5 && s == 2 && ap.n[0] == 16 && ap.n[1] == 16 && (fmt == 1 || fmt == 2) && rest % 32 == 0 &&
          (reinterpret_cast<uintptr_t>(cur) & 15) == 0 && ((rest * (fmt == 1 ? 2 : 1)) & 15) == 0) {
        HIP_TRY(omni::launch_front2_16x16(fmt, cur, ap.d_y[1], ap.d_tw32, tc * ap.F, rest, 1.f / 16.f, st));
        k0 = 2;
        cur = ap.d_y[1];
      }
      for (int k = k0; k < s; ++k) {
        const int nk = ap.n[k], mk = 2 * nk;
        inner /= nk;
        float2* dst = ap.d_y[k & 1];
        // float16 planar output: the last pass before a matrix-core kernel (its operands), and for the
        // three-level kernel also the first (halves the traffic between the two front passes)
        const bool h16 = (ap.kernel == 4 && k == s - 1) || ap.kernel == 5;
        HIP_TRY(omni::launch_front_axis(fmt, cur, dst, ap.d_tw32 + tw_off, tc * ap.F, outer, nk, mk, ap.front_r[k],
                                        inner, outer * nk * inner, outer * mk * inner, st, h16,
                                        h16 ? 1.f / (float)nk : 1.f));
        outer *= mk;
        tw_off += mk;
        cur = dst;
        fmt = h16 ? 3 : 0;
      }
      int slices = 1;
      if (ap.kernel == 4) {
        // all front channels of the chunk in one slice (2048 work-groups for 64 channels)
        // the front pass scaled by 1/n_0 and each of the three passes by 1/16: undo on |X|^2
        const double unscale = (double)ap.n[0] * 4096.0;
        kmark(p, 0, st);
        HIP_TRY(omni::launch_fused16x3_mixed(cur, tc, tc, ap.d_tw32 + ap.front_tw_base, ap.d_partial, (int)ap.fs.F, 1,
                                             p->time_block, c0 > 0 ? 1 : 0, unscale * unscale, st));
        kmark(p, 1, st);
        first_slices = 1;
        continue;
      }
      if (ap.kernel == 5) {
        // the front passes scaled by 1/n_0 and 1/n_1, the kernel's passes by 1/16, 1/8, 1/8: undo on |X|^2
        const double unscale = (double)ap.n[0] * (double)ap.n[1] * 1024.0;
        const float2* tw = ap.d_tw32 + ap.front_tw_base;  // tables of the rest axes: 16, 16, 8, 8 entries
        kmark(p, 0, st);
        HIP_TRY(omni::launch_fused8844_mixed(cur, tc, tc, tw, tw + 32, ap.d_partial, (int)ap.fs.F, 1, p->time_block,
                                             c0 > 0 ? 1 : 0, unscale * unscale, st));
        kmark(p, 1, st);
        first_slices = 1;
        continue;
      }
      if (ap.kernel == 3) {
        kmark(p, 0, st);
        int rc = c0 == 0 ? launch_ct(ap, 0, cur, tc, p->time_block, ap.d_tw32 + ap.front_tw_base, st, &first_slices)
                         : launch_ct(ap, 0, cur, tc, p->time_block, ap.d_tw32 + ap.front_tw_base, st, &slices, 1,
                                     first_slices);
        kmark(p, 1, st);
        if (rc) return rc;
        continue;
      }
      kmark(p, 0, st);
      int rc = launch_general(ap, ap.fs, 0, cur, tc, p->time_block, ap.d_tw32 + ap.front_tw_base, st, &slices);
      kmark(p, 1, st);
      if (rc) return rc;
      HIP_TRY(omni::launch_reduce_scatter(ap.d_partial, ap.d_kmap, ap.d_A, slices, ap.fs.F, ap.fs.fp.n_split,
                                          ap.fs.fp.cells_wg, ap.fs.M, (accumulate || c0 > 0) ? 1 : 0, st));
    }
    if (ap.kernel >= 3)
      HIP_TRY(omni::launch_reduce_scatter(ap.d_partial, ap.d_kmap, ap.d_A, first_slices, ap.fs.F, ap.fs.fp.n_split,
                                          ap.fs.fp.cells_wg, ap.fs.M, accumulate ? 1 : 0, st));
  } else if (stage == 0 && T > 0 && sliced_kernel(ap.kernel)) {
    kmark(p, 0, st);
    int rc = launch_sliced(p, ap, volt, T, ap.wg_target, ap.tb > 0 ? ap.tb : p->time_block, st, &ap.last_slices);
    kmark(p, 1, st);
    if (rc) return rc;
  } else if (stage == 0 && T > 0 && ap.kernel == 3) {
    kmark(p, 0, st);
    int rc = launch_ct(ap, fmt_of(p->dtype), volt, T, p->time_block, ap.d_tw32, st, &ap.last_slices);
    kmark(p, 1, st);
    if (rc) return rc;
  } else if (stage == 0 && T > 0) {
    kmark(p, 0, st);
    int rc = launch_general(ap, ap.fs, fmt_of(p->dtype), volt, T, p->time_block, ap.d_tw32, st, &ap.last_slices);
    kmark(p, 1, st);
    if (rc) return rc;
  }
  if (stage == 1) {
    if (T > 0 && ap.n_front == 0) {
      HIP_TRY(omni::launch_reduce_scatter(ap.d_partial, ap.d_kmap, ap.d_A, ap.last_slices, ap.F, ap.fs.fp.n_split,
                                          ap.fs.fp.cells_wg, ap.M, accumulate ? 1 : 0, st));
    } else if (T == 0 && !accumulate) {
      HIP_TRY(omni::launch_fill_f64(ap.d_A, (int64_t)ap.F * ap.M, 0.0, st));
    }
  }
  if (stage == 2 && !(flags & OMNI_NO_FINALIZE)) {
    // inverse along the zero-padded axes only (a beam-space plan keeps its pointing axes, the innermost, as
    // they are: they ride along in `inner`), normalised by the product of their lengths
    const int d = (int)ap.n.size() - ap.nbeam;
    double m_inv = 1.0;
    for (int k = 0; k < d; ++k) m_inv *= ap.m[k];
    for (int f0 = 0; f0 < ap.F; f0 += ap.inv_group) {
      const int g = std::min(ap.inv_group, ap.F - f0);
      const void* src = ap.d_A + (size_t)f0 * ap.M;
      if (ap.beam_sub && ap.nbeam > 0) {
        // pointings = the even cells of the lowest level's (zero-padded) axes, gathered into d_ws[1]
        const int na = ap.n[ap.n.size() - ap.nbeam], nb = ap.nbeam == 2 ? ap.n.back() : 1;
        const int64_t rows = (int64_t)g * (ap.M / (ap.nbeam == 2 ? 4LL * na * nb : 2LL * na));
        HIP_TRY(omni::launch_even_cells(static_cast<const double*>(src), reinterpret_cast<double*>(ap.d_ws[1]),
                                        rows, na, nb, ap.nbeam, st));
        src = ap.d_ws[1];
      }
      int64_t outer = g;
      for (int k = 0; k < d; ++k) {
        int64_t inner = 1;
        for (int j = k + 1; j < (int)ap.n.size(); ++j) inner *= (ap.beam_sub && j >= d) ? ap.n[j] : ap.m[j];
        const bool last = (k == d - 1);
        void* dst = last ? (void*)(static_cast<float2*>(vis) + (size_t)f0 * ap.n_out) : (void*)ap.d_ws[k & 1];
        HIP_TRY(omni::launch_inverse_axis(k == 0, last, src, dst, ap.d_tw64 + ap.inv_off[k], outer, ap.m[k],
                                          ap.n[k], inner, 1.0 / m_inv, st));
        src = dst;
        outer *= 2 * ap.n[k] - 1;
      }
    }
  }
  return OMNI_OK;
}

// Autotuner for the general fused kernel: times every candidate schedule
// (longest short DFT lcap x work-group target of the time slicing) on an
// all-zero input of a few samples with HIP events, keeps the fastest, and
// remembers the choice in the plan's tune_cache file (one line per array:
// key lcap wg_target ms), if one is named.
std::string tune_key(const ArrayPlan& ap, omni_dtype dtype) {
  std::string k = "gfx950:";
  for (int v : ap.n) k += std::to_string(v) + "x";
  k += ":F" + std::to_string(ap.F) + ":t" + std::to_string((int)dtype) + ":k" + std::to_string(ap.kernel);
  return k;
}

bool tune_cache_lookup(const std::string& path, const std::string& key, int* lcap, int* wgt) {
  if (path.empty()) return false;
  FILE* fp = std::fopen(path.c_str(), "r");
  if (!fp) return false;
  char k[256];
  int a, b;
  double ms;
  bool found = false;
  while (std::fscanf(fp, "%255s %d %d %lf", k, &a, &b, &ms) == 4)
    if (key == k) {
      *lcap = a;
      *wgt = b;
      found = true;
    }
  std::fclose(fp);
  return found;
}

void tune_cache_store(const std::string& path, const std::string& key, int lcap, int wgt, double ms) {
  if (path.empty()) return;
  FILE* fp = std::fopen(path.c_str(), "a");
  if (!fp) return;
  std::fprintf(fp, "%s %d %d %.4f\n", key.c_str(), lcap, wgt, ms);
  std::fclose(fp);
}

// Times the candidate schedules on zero input and keeps the fastest: for the
// general kernel, short-DFT cap x time slicing; for the compile-time-shape
// kernel (fixed fold moduli), time slicing only; for the sliced fixed-shape
// kernels, time slicing x float32 block.  The kernels behind front passes take
// all channels of a chunk in one launch and have no schedule to tune.
// Sliced kernels (fixed shape): time slicing (work-group target) x float32 block.  The block is tuned only in
// the mixed form and only when the caller left time_block at its default (longer float32 blocks stay far
// inside the mixed form's error budget; the float32 form keeps its 64-sample block).  A cached schedule is
// taken as stored (cache line: key block wg_target ms).
int tune_sliced(omni_plan_s* p, ArrayPlan& ap) {
  const std::string key = tune_key(ap, p->dtype);
  int c_tb = 0, c_wg = 0;
  if (p->tune == OMNI_TUNE_CACHE && tune_cache_lookup(p->tune_cache, key, &c_tb, &c_wg) && c_tb > 0 && c_wg > 0) {
    ap.tb = c_tb;
    ap.wg_target = c_wg;
    log_msg(2, "autotuner: %s -> block %d, work-group target %d (from the cache)", key.c_str(), c_tb, c_wg);
    return OMNI_OK;
  }
  const size_t bytes_t = (size_t)ap.F * (size_t)ap.N * sample_bytes(p->dtype);
  const int64_t Tt = std::max<int64_t>(16, std::min<int64_t>(2048, (int64_t(1) << 30) / (int64_t)bytes_t));
  std::vector<int> tbs;
  if (p->form == OMNI_FORM_MIXED && !p->time_block_set)
    tbs = {256, 1024};
  else
    tbs = {p->time_block};
  std::vector<int> wgs = {256, 512, 1024, 2048, 4096};
  if (std::find(wgs.begin(), wgs.end(), ap.wg_target) == wgs.end()) wgs.push_back(ap.wg_target);
  void* zero = nullptr;
  HIP_TRY(hipMalloc(&zero, bytes_t * (size_t)Tt));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipMemset(zero, 0, bytes_t * (size_t)Tt);
  if (he == hipSuccess) he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  double best = 1e30;
  int best_tb = ap.tb, best_wg = ap.wg_target;
  int rc = OMNI_OK;
  for (int tb : tbs) {
    for (int wg : wgs) {
      if (he != hipSuccess || rc != OMNI_OK) break;
      float ms = 0.f;
      int slices = 1;
      for (int rep = 0; rep < 2 && rc == OMNI_OK && he == hipSuccess; ++rep) {
        he = hipEventRecord(e0, 0);
        if (he == hipSuccess) rc = launch_sliced(p, ap, zero, Tt, wg, tb, 0, &slices);
        if (he == hipSuccess && rc == OMNI_OK) he = hipEventRecord(e1, 0);
        if (he == hipSuccess && rc == OMNI_OK) he = hipEventSynchronize(e1);
        if (he == hipSuccess && rc == OMNI_OK) he = hipEventElapsedTime(&ms, e0, e1);
      }
      if (he == hipSuccess && rc == OMNI_OK && ms < best) {
        best = ms;
        best_tb = tb;
        best_wg = wg;
      }
    }
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(zero);
  if (rc) return rc;
  if (he != hipSuccess) return fail(OMNI_E_HIP, std::string("autotuner: ") + hipGetErrorString(he));
  ap.tb = best_tb;
  ap.wg_target = best_wg;
  ap.tuned_ms = best;
  tune_cache_store(p->tune_cache, key, best_tb, best_wg, best);
  log_msg(2, "autotuner: %s -> block %d, work-group target %d (%.3f ms on %lld samples)", key.c_str(), best_tb,
          best_wg, best, (long long)Tt);
  return OMNI_OK;
}

int tune_array(omni_plan_s* p, ArrayPlan& ap) {
  if (sliced_kernel(ap.kernel)) return tune_sliced(p, ap);
  if (ap.kernel != 0 && ap.kernel != 3) return OMNI_OK;
  const bool ct = ap.kernel == 3;
  const std::string key = tune_key(ap, p->dtype);
  int lc = 0, wg = 0;
  const bool cached = p->tune == OMNI_TUNE_CACHE && tune_cache_lookup(p->tune_cache, key, &lc, &wg);
  const bool front = ap.n_front > 0;
  const std::vector<int> axes = front ? std::vector<int>(ap.n.begin() + ap.n_front, ap.n.end()) : ap.n;
  const int Fk = ap.fs.F;
  const int fmt = front ? 0 : fmt_of(p->dtype);
  const size_t bytes_t = (size_t)Fk * (size_t)ap.fs.N * (front ? sizeof(float2) : sample_bytes(p->dtype));
  const int64_t Tt = std::max<int64_t>(4, std::min<int64_t>(256, (int64_t(256) << 20) / (int64_t)bytes_t));
  void* zero = nullptr;
  HIP_TRY(hipMalloc(&zero, bytes_t * (size_t)Tt));
  HIP_TRY(hipMemset(zero, 0, bytes_t * (size_t)Tt));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const float2* tw = ap.d_tw32 + (front ? ap.front_tw_base : 0);
  double best = 1e30;
  FusedSetup best_fs;
  int best_lc = ap.lcap, best_wg = ap.wg_target;
  const int lcaps[3] = {8, 16, 32};
  const int wgts[3] = {512, 1024, 2048};
  for (int li = 0; li < 3; ++li) {
    for (int wi = 0; wi < 3; ++wi) {
      if (cached && (lcaps[li] != lc || wgts[wi] != wg)) continue;
      if (ct && lcaps[li] != ap.lcap) continue;
      FusedSetup fs;
      std::string why;
      if (ct) {
        fs = ap.fs;
      } else if (plan_fused_axes(axes, Fk, 0, front ? true : ap.single_split, lcaps[li], fs, &why, nullptr, 0,
                                 ap.m.data() + ap.n_front)) {
        continue;
      }
      const int keep_wg = ap.wg_target;
      ap.wg_target = wgts[wi];
      float ms = 0.f;
      int slices = 1;
      int rc = OMNI_OK;
      for (int rep = 0; rep < 2 && rc == OMNI_OK; ++rep) {
        HIP_TRY(hipEventRecord(e0, 0));
        rc = ct ? launch_ct(ap, fmt, zero, Tt, p->time_block, tw, 0, &slices)
                : launch_general(ap, fs, fmt, zero, Tt, p->time_block, tw, 0, &slices);
        HIP_TRY(hipEventRecord(e1, 0));
        HIP_TRY(hipEventSynchronize(e1));
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      }
      ap.wg_target = keep_wg;
      if (rc == OMNI_OK && ms < best) {
        best = ms;
        best_fs = std::move(fs);
        best_lc = lcaps[li];
        best_wg = wgts[wi];
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(zero);
  if (best < 1e30) {
    ap.fs = std::move(best_fs);
    ap.lcap = best_lc;
    ap.wg_target = best_wg;
    ap.tuned_ms = best;
    HIP_TRY(hipMemcpy(ap.d_kmap, ap.fs.kmap.data(), ap.fs.kmap.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    if (!cached) tune_cache_store(p->tune_cache, key, best_lc, best_wg, best);
    log_msg(2, "autotuner: %s -> short-DFT cap %d, work-group target %d (%.3f ms)%s", key.c_str(), best_lc, best_wg,
            best, cached ? " (cached schedule re-timed)" : "");
  }
  return OMNI_OK;
}

// Streams and events of an OMNI_PLAN_GRAPH plan (default priority, non-blocking streams).
int make_graph_resources(omni_plan_s* p) {
  p->graph = true;
  p->branch.assign(p->arrays.size(), nullptr);
  p->join.assign(p->arrays.size(), nullptr);
  HIP_TRY(hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&p->fork, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&p->g_done, hipEventDisableTiming));
  for (size_t i = 0; i < p->arrays.size(); ++i) {
    HIP_TRY(hipStreamCreateWithFlags(&p->branch[i], hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&p->join[i], hipEventDisableTiming));
  }
  return OMNI_OK;
}

// The executable graph may still be running from the caller's last launch:
// wait for that launch before the graph is destroyed.
void drop_graph(omni_plan_s* p) {
  if (p->gx && p->g_done) hipEventSynchronize(p->g_done);
  if (p->gx) hipGraphExecDestroy(p->gx);
  if (p->g) hipGraphDestroy(p->g);
  p->gx = nullptr;
  p->g = nullptr;
  p->g_T = -1;
}

// Everything a plan owns on the device (safe on a partly built plan).
void destroy_plan_resources(omni_plan_s* p) {
  drop_graph(p);
  for (auto& e : p->ev)
    if (e) hipEventDestroy(e);
  p->ev.clear();
  for (auto& e : p->kev)
    if (e) hipEventDestroy(e);
  p->kev.clear();
  for (auto& e : p->join)
    if (e) hipEventDestroy(e);
  for (auto& s : p->branch)
    if (s) hipStreamDestroy(s);
  p->join.clear();
  p->branch.clear();
  if (p->fork) hipEventDestroy(p->fork);
  if (p->g_done) hipEventDestroy(p->g_done);
  if (p->capture) hipStreamDestroy(p->capture);
  p->fork = nullptr;
  p->g_done = nullptr;
  p->capture = nullptr;
  for (auto& ap : p->arrays) free_array(ap);
}

// Capture one correlate call of a graph plan: the fork event on the capture
// stream, each array's three stages on its branch stream, the joins back.
int capture_call(omni_plan_s* p, const void* const* volt, int64_t T, void* const* vis, uint32_t flags) {
  drop_graph(p);
  HIP_TRY(hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal));
  int rc = OMNI_OK;
  hipError_t e = hipEventRecord(p->fork, p->capture);
  for (size_t i = 0; i < p->arrays.size() && rc == OMNI_OK && e == hipSuccess; ++i) {
    e = hipStreamWaitEvent(p->branch[i], p->fork, 0);
    for (int stage = 0; stage < 3 && rc == OMNI_OK && e == hipSuccess; ++stage)
      rc = correlate_array(p, p->arrays[i], T > 0 ? volt[i] : nullptr, T,
                           (flags & OMNI_NO_FINALIZE) ? nullptr : vis[i], p->branch[i], flags, stage);
    if (rc == OMNI_OK && e == hipSuccess) e = hipEventRecord(p->join[i], p->branch[i]);
    if (rc == OMNI_OK && e == hipSuccess) e = hipStreamWaitEvent(p->capture, p->join[i], 0);
  }
  hipGraph_t g = nullptr;
  const hipError_t e_end = hipStreamEndCapture(p->capture, &g);  // always end the capture
  if (rc != OMNI_OK || e != hipSuccess || e_end != hipSuccess) {
    if (g) hipGraphDestroy(g);
    if (rc != OMNI_OK) return rc;
    return fail(OMNI_E_HIP, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e_end));
  }
  p->g = g;
  HIP_TRY(hipGraphInstantiate(&p->gx, p->g, nullptr, nullptr, 0));
  p->g_T = T;
  p->g_flags = flags;
  p->g_volt.assign(volt ? volt : nullptr, volt ? volt + p->arrays.size() : nullptr);
  p->g_vis.assign(vis ? vis : nullptr, vis ? vis + p->arrays.size() : nullptr);
  return OMNI_OK;
}

bool same_call(const omni_plan_s* p, const void* const* volt, int64_t T, void* const* vis, uint32_t flags) {
  if (!p->gx || p->g_T != T || p->g_flags != flags) return false;
  for (size_t i = 0; i < p->arrays.size(); ++i) {
    const void* v = (T > 0 && volt) ? volt[i] : nullptr;
    const void* o = ((flags & OMNI_NO_FINALIZE) || !vis) ? nullptr : vis[i];
    const void* gv = (T > 0 && !p->g_volt.empty()) ? p->g_volt[i] : nullptr;
    const void* go = ((flags & OMNI_NO_FINALIZE) || p->g_vis.empty()) ? nullptr : p->g_vis[i];
    if (v != gv || o != go) return false;
  }
  return true;
}

int make_plan(omni_plan_t* out, const std::vector<omni_array_desc>& arrays, const omni_opts* opts) {
  if (!out) return fail(OMNI_E_INVAL, "out is NULL");
  *out = nullptr;
  omni_opts o{OMNI_CF32, OMNI_FORM_FP32, 0, 0, OMNI_TUNE_OFF, nullptr, 0};
  if (opts) o = *opts;
  if (o.dtype < OMNI_CF32 || o.dtype > OMNI_CI4) return fail(OMNI_E_INVAL, "unknown dtype");
  if (o.form != OMNI_FORM_FP32 && o.form != OMNI_FORM_MIXED) return fail(OMNI_E_INVAL, "unknown form");
  if (o.time_block < 0) return fail(OMNI_E_INVAL, "time_block < 0");
  if (o.flags & ~(OMNI_PLAN_HOST_ONLY | OMNI_PLAN_TIMING | OMNI_PLAN_GRAPH | OMNI_PLAN_BEAMS))
    return fail(OMNI_E_INVAL, "unknown plan flag");
  if (o.tune < OMNI_TUNE_OFF || o.tune > OMNI_TUNE_SEARCH) return fail(OMNI_E_INVAL, "unknown tune mode");
  if (o.chunk_T < 0) return fail(OMNI_E_INVAL, "chunk_T < 0");
  omni_plan_s* p = new (std::nothrow) omni_plan_s;
  if (!p) return fail(OMNI_E_NOMEM, "host allocation failed");
  p->dtype = o.dtype;
  p->form = o.form;
  // default float32 block: 64 samples; 1024 in the mixed form, whose matrix-core kernels add each block into
  // float64 partial sums in HBM (a float32 sum of 1024 non-negative terms stays within 2^-14 relative,
  // far inside the form's 2e-3)
  p->time_block = o.time_block > 0 ? o.time_block : (o.form == OMNI_FORM_MIXED ? 1024 : 64);
  p->time_block_set = o.time_block > 0;
  p->host_only = (o.flags & OMNI_PLAN_HOST_ONLY) != 0;
  p->timing = (o.flags & OMNI_PLAN_TIMING) != 0 && !p->host_only;
  p->tune = o.tune;
  if (o.tune_cache) p->tune_cache = o.tune_cache;
  p->arrays.resize(arrays.size());
  for (size_t i = 0; i < arrays.size(); ++i) {
    p->arrays[i].chunk_cap = o.chunk_T;
    int rc = build_array(p->arrays[i], arrays[i].levels, arrays[i].dims, arrays[i].A, arrays[i].nchan, p->form,
                         p->dtype, (o.flags & OMNI_PLAN_BEAMS) != 0);
    if (rc) {
      delete p;
      return rc;
    }
  }
  if (!p->host_only) {
    int rc = check_device(&p->device);
    if (rc) {
      delete p;
      return rc;
    }
    if (p->timing) {
      p->ev.assign((size_t)kTimingRing * kStages * 2, nullptr);
      p->kev.assign((size_t)kKernRing * kKernMax * 2, nullptr);
      p->kev_n.assign((size_t)kKernRing, 0);
      for (auto* v : {&p->ev, &p->kev})
        for (auto& e : *v) {
          if (hipEventCreate(&e) != hipSuccess) {
            destroy_plan_resources(p);
            delete p;
            return fail(OMNI_E_HIP, "hipEventCreate failed");
          }
        }
    }
    if (o.flags & OMNI_PLAN_GRAPH) {
      rc = make_graph_resources(p);
      if (rc) {
        destroy_plan_resources(p);
        delete p;
        return rc;
      }
    }
    for (auto& ap : p->arrays) {
      rc = alloc_array(ap);
      if (rc == OMNI_OK && p->tune != OMNI_TUNE_OFF) rc = tune_array(p, ap);
      if (rc) {
        destroy_plan_resources(p);
        delete p;
        return rc;
      }
    }
  }
  *out = p;
  if (log_level() >= 2) {
    size_t need = 0;
    omni_plan_describe(p, nullptr, 0, &need);
    std::string d(need, '\0');
    omni_plan_describe(p, d.data(), need, nullptr);
    log_msg(2, "plan %s", d.c_str());
  }
  return OMNI_OK;
}

// Direct correlator geometry (host only, allocates nothing): blocks of 128 consecutive antennas, the
// strides of the centred output, the number of block pairs I <= J, and the check that every pair's Delta box
// fits the kernel's LDS bins (bound: prod_k (2 max_B ext_k(B) + 1) over the blocks' per-axis extents).
int direct_geometry(ArrayPlan& ap) {
  using omni::kDirectMaxD;
  using omni::kDirectTile;
  if (ap.dc_geom_ok) return OMNI_OK;
  const int d = (int)ap.dims.size();
  if (d < 1 || d > kDirectMaxD) return fail(OMNI_E_SHAPE, "direct correlator: 1 to 8 axes");
  if (ap.N % kDirectTile != 0) return fail(OMNI_E_SHAPE, "direct correlator: N must be a multiple of 128");
  const int64_t nbk = ap.N / kDirectTile;
  const int64_t n_pairs = nbk * (nbk + 1) / 2;
  // one work-group of 512 threads per block pair: the grid's x extent in threads must stay below 2^32
  if (n_pairs >= (int64_t(1) << 23)) return fail(OMNI_E_SHAPE, "direct correlator: N too large (2^23 block pairs or more)");
  omni::DirectGeom g;
  g.d = d;
  int64_t n_out = 1;
  for (int k = d - 1; k >= 0; --k) {
    g.n[k] = ap.dims[(size_t)k];
    g.gstride[k] = n_out;
    n_out *= 2 * (int64_t)ap.dims[(size_t)k] - 1;
  }
  g.n_out = n_out;
  int ext[kDirectMaxD] = {}, lo[kDirectMaxD] = {}, hi[kDirectMaxD] = {}, c[kDirectMaxD] = {};
  for (int64_t B = 0; B < nbk; ++B) {
    for (int64_t r = 0; r < kDirectTile; ++r) {
      int64_t a = B * kDirectTile + r;
      for (int k = d - 1; k >= 0; --k) {
        c[k] = (int)(a % ap.dims[(size_t)k]);
        a /= ap.dims[(size_t)k];
      }
      for (int k = 0; k < d; ++k) {
        lo[k] = r == 0 ? c[k] : std::min(lo[k], c[k]);
        hi[k] = r == 0 ? c[k] : std::max(hi[k], c[k]);
      }
    }
    for (int k = 0; k < d; ++k) ext[k] = std::max(ext[k], hi[k] - lo[k]);
  }
  int64_t box = 1;
  for (int k = 0; k < d; ++k) box *= 2 * (int64_t)ext[k] + 1;
  if (box > omni::kDirectMaxBins)
    return fail(OMNI_E_SHAPE, "direct correlator: a block pair spans " + std::to_string(box) +
                                  " index differences (at most " + std::to_string(omni::kDirectMaxBins) + ")");
  ap.dc_pairs = n_pairs;
  ap.dc_geom = g;
  ap.dc_geom_ok = true;
  return OMNI_OK;
}

// Direct correlator buffers of omni_direct_correlate (allocated by its first call): the block boxes, the block
// pairs I <= J (I-major), and the int64 half-sum buffer.
int direct_setup(ArrayPlan& ap) {
  using omni::kDirectMaxD;
  using omni::kDirectTile;
  int rc = direct_geometry(ap);
  if (rc) return rc;
  const int d = (int)ap.dims.size();
  const int64_t nbk = ap.N / kDirectTile;
  std::vector<int32_t> blk((size_t)(nbk * kDirectMaxD * 2), 0);
  std::vector<int> c((size_t)d, 0);
  for (int64_t B = 0; B < nbk; ++B) {
    int32_t* b = &blk[(size_t)(B * kDirectMaxD * 2)];
    for (int64_t r = 0; r < kDirectTile; ++r) {
      int64_t a = B * kDirectTile + r;
      for (int k = d - 1; k >= 0; --k) {
        c[(size_t)k] = (int)(a % ap.dims[(size_t)k]);
        a /= ap.dims[(size_t)k];
      }
      for (int k = 0; k < d; ++k) {
        if (r == 0 || c[(size_t)k] < b[2 * k]) b[2 * k] = c[(size_t)k];
        if (r == 0 || c[(size_t)k] > b[2 * k + 1]) b[2 * k + 1] = c[(size_t)k];
      }
    }
  }
  std::vector<int32_t> pairs((size_t)(2 * ap.dc_pairs));
  size_t q = 0;
  for (int64_t I = 0; I < nbk; ++I)
    for (int64_t J = I; J < nbk; ++J) {
      pairs[q++] = (int32_t)I;
      pairs[q++] = (int32_t)J;
    }
  HIP_TRY(hipMalloc(&ap.d_dc_blk, blk.size() * sizeof(int32_t)));
  HIP_TRY(hipMalloc(&ap.d_dc_pairs, pairs.size() * sizeof(int32_t)));
  HIP_TRY(hipMalloc(&ap.d_dc_G, (size_t)ap.F * (size_t)ap.dc_geom.n_out * 2 * sizeof(unsigned long long)));
  HIP_TRY(hipMemcpy(ap.d_dc_blk, blk.data(), blk.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ap.d_dc_pairs, pairs.data(), pairs.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  return OMNI_OK;
}

// Argument checks shared by both direct-correlator entry points.
int direct_check_args(omni_plan_t plan, const void* volt, int64_t T, const void* vis) {
  if (!plan) return fail(OMNI_E_INVAL, "plan is NULL");
  if (plan->host_only) return fail(OMNI_E_STATE, "plan was made with OMNI_PLAN_HOST_ONLY");
  if (plan->arrays.size() != 1) return fail(OMNI_E_STATE, "direct correlator: single-array plans only");
  if (plan->arrays[0].beams) return fail(OMNI_E_STATE, "direct correlator: not for beam-space plans");
  if (plan->dtype != OMNI_CI8 && plan->dtype != OMNI_CI4)
    return fail(OMNI_E_STATE, "direct correlator: integer samples (ci8, ci4) only");
  if (T < 0) return fail(OMNI_E_INVAL, "T < 0");
  if (T > 0 && !volt) return fail(OMNI_E_INVAL, "volt is NULL");
  if (!vis) return fail(OMNI_E_INVAL, "vis is NULL");
  const int sb = plan->dtype == OMNI_CI8 ? 2 : 1;
  if (T > 0 && (reinterpret_cast<uintptr_t>(volt) & (uintptr_t)(4 * sb - 1)))
    return fail(OMNI_E_INVAL, sb == 2 ? "voltage pointer not 8-byte aligned" : "voltage pointer not 4-byte aligned");
  int cur = -1;
  hipGetDevice(&cur);
  if (cur != plan->device) return fail(OMNI_E_STATE, "current HIP device is not the plan's device");
  return OMNI_OK;
}

// The launches of one direct-correlator call on buffers G (int64 half-sums), pairs and blk.
int direct_run(omni_plan_t plan, ArrayPlan& ap, const void* volt, int64_t T, void* vis, hipStream_t st,
               unsigned long long* G, const int32_t* pairs, const int32_t* blk) {
  const omni::DirectGeom& g = ap.dc_geom;
  const int sb = plan->dtype == OMNI_CI8 ? 2 : 1;
  HIP_TRY(omni::launch_direct_zero(G, (int64_t)ap.F * g.n_out * 2, st));
  const int64_t tstride = (int64_t)ap.F * ap.N * sb;  // bytes per time sample
  for (int64_t t0 = 0; t0 < T; t0 += omni::kDirectMaxT) {
    const int64_t tc = std::min<int64_t>(omni::kDirectMaxT, T - t0);
    HIP_TRY(omni::launch_direct_tiles((int)plan->dtype, static_cast<const uint8_t*>(volt) + t0 * tstride, tc, ap.N,
                                      ap.F, pairs, ap.dc_pairs, blk, g, G, st));
  }
  HIP_TRY(omni::launch_direct_finalize(G, vis, g.n_out, ap.F, st));
  return OMNI_OK;
}

}  // namespace

extern "C" {

int omni_plan(omni_plan_t* out, int32_t levels, const int32_t* dims, const double* A, int32_t nchan,
              const omni_opts* opts) {
  TraceRange range("omni_plan");
  try {
    omni_array_desc a{levels, dims, A, nchan};
    return make_plan(out, {a}, opts);
  } catch (...) {
    return fail(OMNI_E_NOMEM, "unexpected host exception");
  }
}

int omni_plan_batch(omni_plan_t* out, int32_t n_arrays, const omni_array_desc* arrays, const omni_opts* opts) {
  TraceRange range("omni_plan_batch");
  try {
    if (n_arrays < 1 || !arrays) return fail(OMNI_E_INVAL, "need at least one array");
    return make_plan(out, std::vector<omni_array_desc>(arrays, arrays + n_arrays), opts);
  } catch (...) {
    return fail(OMNI_E_NOMEM, "unexpected host exception");
  }
}

int omni_correlate_batch(omni_plan_t plan, const void* const* volt, int64_t T, void* const* vis, void* stream,
                         uint32_t flags) {
  TraceRange range("omni_correlate");
  try {
    if (!plan) return fail(OMNI_E_INVAL, "plan is NULL");
    if (plan->host_only) return fail(OMNI_E_STATE, "plan was made with OMNI_PLAN_HOST_ONLY");
    if (T < 0) return fail(OMNI_E_INVAL, "T < 0");
    if (flags & ~(OMNI_NO_RESET | OMNI_NO_FINALIZE)) return fail(OMNI_E_INVAL, "unknown correlate flag");
    const size_t na = plan->arrays.size();
    if (T > 0 && !volt) return fail(OMNI_E_INVAL, "volt is NULL");
    if (!(flags & OMNI_NO_FINALIZE) && !vis) return fail(OMNI_E_INVAL, "vis is NULL");
    for (size_t i = 0; i < na; ++i) {
      if (T > 0 && !volt[i]) return fail(OMNI_E_INVAL, "a voltage pointer is NULL");
      if (T > 0 && (reinterpret_cast<uintptr_t>(volt[i]) & 3u))
        return fail(OMNI_E_INVAL, "voltage pointer not 4-byte aligned");
      if (!(flags & OMNI_NO_FINALIZE) && !vis[i]) return fail(OMNI_E_INVAL, "a visibility pointer is NULL");
    }
    int cur = -1;
    hipGetDevice(&cur);
    if (cur != plan->device) return fail(OMNI_E_STATE, "current HIP device is not the plan's device");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (plan->timing) plan->kev_n[(size_t)(plan->n_calls % kKernRing)] = 0;
    mark(plan, OMNI_STAGE_CALL, 0, true, st);
    if (plan->graph) {
      if (!same_call(plan, volt, T, vis, flags)) {
        // Re-capturing a live plan is switched off: the process crashed inside such a call on the GPU
        // (after a series of captures) and the cause has not been found.  One plan, one call shape.
        if (plan->gx)
          return fail(OMNI_E_STATE,
                      "graph plan: T, flags and buffers must repeat the first (captured) call; make another plan");
        int rc = capture_call(plan, volt, T, vis, flags);
        if (rc) return rc;
      }
      HIP_TRY(hipGraphLaunch(plan->gx, st));
      HIP_TRY(hipEventRecord(plan->g_done, st));
    } else {
      for (int stage = 0; stage < 3; ++stage) {
        for (size_t i = 0; i < na; ++i) {
          mark(plan, stage, 0, i == 0, st);
          int rc = correlate_array(plan, plan->arrays[i], T > 0 ? volt[i] : nullptr, T,
                                   (flags & OMNI_NO_FINALIZE) ? nullptr : vis[i], st, flags, stage);
          if (rc) return rc;
          mark(plan, stage, 1, i + 1 == na, st);
        }
      }
    }
    mark(plan, OMNI_STAGE_CALL, 1, true, st);
    if (plan->timing) ++plan->n_calls;
    return OMNI_OK;
  } catch (...) {
    return fail(OMNI_E_NOMEM, "unexpected host exception");
  }
}

int omni_correlate(omni_plan_t plan, const void* volt, int64_t T, void* vis, void* stream, uint32_t flags) {
  if (plan && plan->arrays.size() != 1) return fail(OMNI_E_STATE, "batch plan: use omni_correlate_batch");
  const void* v[1] = {volt};
  void* o[1] = {vis};
  return omni_correlate_batch(plan, v, T, o, stream, flags);
}

int omni_direct_correlate(omni_plan_t plan, const void* volt, int64_t T, void* vis, void* stream) {
  TraceRange range("omni_direct_correlate");
  try {
    int rc = direct_check_args(plan, volt, T, vis);
    if (rc) return rc;
    ArrayPlan& ap = plan->arrays[0];
    if (!ap.d_dc_G) {
      rc = direct_setup(ap);
      if (rc) return rc;
    }
    return direct_run(plan, ap, volt, T, vis, reinterpret_cast<hipStream_t>(stream), ap.d_dc_G, ap.d_dc_pairs,
                      ap.d_dc_blk);
  } catch (...) {
    return fail(OMNI_E_NOMEM, "unexpected host exception");
  }
}

int omni_direct_correlate_noalloc(omni_plan_t plan, const void* volt, int64_t T, void* vis, void* stream) {
  TraceRange range("omni_direct_correlate_noalloc");
  try {
    int rc = direct_check_args(plan, volt, T, vis);
    if (rc) return rc;
    ArrayPlan& ap = plan->arrays[0];
    rc = direct_geometry(ap);
    if (rc) return rc;
    // scratch layout: int64 half-sums G [F][cells][2], then the block pairs, then the block boxes
    const int64_t nbk = ap.N / omni::kDirectTile;
    const size_t g_bytes = (size_t)ap.F * (size_t)ap.dc_geom.n_out * 2 * sizeof(unsigned long long);
    const size_t p_bytes = (size_t)(2 * ap.dc_pairs) * sizeof(int32_t);
    const size_t b_bytes = (size_t)(nbk * omni::kDirectMaxD * 2) * sizeof(int32_t);
    const size_t p_off = (g_bytes + 255) / 256 * 256, b_off = p_off + (p_bytes + 255) / 256 * 256;
    const size_t need = b_off + b_bytes, cap = omni::direct_noalloc_capacity();
    if (need > cap)
      return fail(OMNI_E_NOMEM, "direct correlator without allocation: the call needs " + std::to_string(need) +
                                    " bytes of scratch (F x cells x 16 + block lists), the fixed scratch holds " +
                                    std::to_string(cap));
    void* base = nullptr;
    HIP_TRY(omni::direct_noalloc_scratch(&base));
    char* sp = static_cast<char*>(base);
    auto* G = reinterpret_cast<unsigned long long*>(sp);
    auto* pairs = reinterpret_cast<int32_t*>(sp + p_off);
    auto* blk = reinterpret_cast<int32_t*>(sp + b_off);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(omni::launch_direct_setup(ap.dc_geom, nbk, blk, pairs, st));
    return direct_run(plan, ap, volt, T, vis, st, G, pairs, blk);
  } catch (...) {
    return fail(OMNI_E_NOMEM, "unexpected host exception");
  }
}

int omni_n_arrays(omni_plan_t plan, int32_t* n) {
  if (!plan || !n) return fail(OMNI_E_INVAL, "NULL argument");
  *n = (int32_t)plan->arrays.size();
  return OMNI_OK;
}

int omni_vis_shape(omni_plan_t plan, int32_t array, int32_t* ndim, int64_t* shape) {
  if (!plan || !ndim || !shape) return fail(OMNI_E_INVAL, "NULL argument");
  if (array < 0 || (size_t)array >= plan->arrays.size()) return fail(OMNI_E_INVAL, "array index out of range");
  const ArrayPlan& ap = plan->arrays[(size_t)array];
  *ndim = 1 + (int32_t)ap.dims.size();
  shape[0] = ap.F;
  for (size_t k = 0; k < ap.dims.size(); ++k)
    shape[k + 1] = ap.beams && k + 2 >= ap.dims.size() ? ap.dims[k] : 2 * ap.dims[k] - 1;
  return OMNI_OK;
}

int omni_baselines(omni_plan_t plan, int32_t array, double* uv) {
  if (!plan || !uv) return fail(OMNI_E_INVAL, "NULL argument");
  if (array < 0 || (size_t)array >= plan->arrays.size()) return fail(OMNI_E_INVAL, "array index out of range");
  const ArrayPlan& ap = plan->arrays[(size_t)array];
  if (ap.A.empty()) return fail(OMNI_E_STATE, "plan has no lattice matrices");
  if (ap.beams) return fail(OMNI_E_STATE, "beam-space plan: its cells along the lowest level are pointings");
  const int d = (int)ap.dims.size();
  std::vector<int> out(d);
  int64_t cells = 1;
  for (int k = 0; k < d; ++k) {
    out[k] = 2 * ap.dims[k] - 1;
    cells *= out[k];
  }
  for (int64_t c = 0; c < cells; ++c) {
    int64_t rem = c;
    double x = 0, y = 0;
    std::vector<int> delta(d);
    for (int k = d - 1; k >= 0; --k) {
      delta[k] = (int)(rem % out[k]) - (ap.dims[k] - 1);
      rem /= out[k];
    }
    for (int l = 0; l < ap.levels; ++l) {
      const double* Al = &ap.A[4 * l];
      x += Al[0] * delta[2 * l] + Al[1] * delta[2 * l + 1];
      y += Al[2] * delta[2 * l] + Al[3] * delta[2 * l + 1];
    }
    uv[2 * c] = x;
    uv[2 * c + 1] = y;
  }
  return OMNI_OK;
}

int omni_accumulator_bytes(omni_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return fail(OMNI_E_INVAL, "NULL argument");
  size_t b = 0;
  for (const auto& ap : plan->arrays) b += (size_t)ap.F * ap.M * sizeof(double);
  *bytes = b;
  return OMNI_OK;
}

static int acc_copy(omni_plan_t plan, void* buf, size_t bytes, void* stream, bool get) {
  if (!plan || !buf) return fail(OMNI_E_INVAL, "NULL argument");
  if (plan->host_only) return fail(OMNI_E_STATE, "host-only plan has no accumulator");
  size_t need = 0;
  omni_accumulator_bytes(plan, &need);
  if (bytes != need) return fail(OMNI_E_INVAL, "buffer size must equal omni_accumulator_bytes");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  size_t off = 0;
  for (auto& ap : plan->arrays) {
    const size_t b = (size_t)ap.F * ap.M * sizeof(double);
    char* hb = static_cast<char*>(buf) + off;
    if (get)
      HIP_TRY(hipMemcpyAsync(hb, ap.d_A, b, hipMemcpyDefault, st));
    else
      HIP_TRY(hipMemcpyAsync(ap.d_A, hb, b, hipMemcpyDefault, st));
    off += b;
  }
  HIP_TRY(hipStreamSynchronize(st));
  return OMNI_OK;
}

int omni_accumulator_get(omni_plan_t plan, void* buf, size_t bytes, void* stream) {
  return acc_copy(plan, buf, bytes, stream, true);
}

int omni_accumulator_set(omni_plan_t plan, const void* buf, size_t bytes, void* stream) {
  return acc_copy(plan, const_cast<void*>(buf), bytes, stream, false);
}

int omni_plan_describe(omni_plan_t plan, char* buf, size_t len, size_t* needed) {
  if (!plan) return fail(OMNI_E_INVAL, "plan is NULL");
  std::string s = "{\"form\":\"";
  s += plan->form == OMNI_FORM_FP32 ? "fp32" : "mixed";
  s += "\",\"dtype\":" + std::to_string((int)plan->dtype) + ",\"time_block\":" + std::to_string(plan->time_block);
  s += ",\"arrays\":[";
  for (size_t i = 0; i < plan->arrays.size(); ++i) {
    const ArrayPlan& ap = plan->arrays[i];
    const FusedP& P = ap.fs.fp;
    if (i) s += ",";
    const char* kname = ap.kernel == 1   ? "fused8x4_fp32"
                        : ap.kernel == 2 ? "fused8x4_mixed"
                        : ap.kernel == 3 ? "fused_ct_fp32"
                        : ap.kernel == 4 ? "fused16x3_mixed"
                        : ap.kernel == 5 ? "fused8844_mixed"
                        : ap.kernel == 6 ? "grid128_mixed"
                        : ap.kernel == 7 ? "grid64_mixed"
                        : ap.kernel == 8 ? "grid32_mixed"
                                         : "fused_fp32";
    s += std::string("{\"kernel\":\"") + kname + "\",\"beams\":\"" +
         (ap.beams ? (ap.beam_sub ? "subset" : "unpadded") : "no") + "\",\"mode\":\"" +
         (ap.n_front ? "front" : "direct") +
         "\",\"n_front\":" + std::to_string(ap.n_front) + ",\"chunk_T\":" + std::to_string(ap.chunk_T) +
         ",\"N\":" + std::to_string(ap.N) + ",\"M\":" + std::to_string(ap.M) + ",\"F\":" + std::to_string(ap.F) +
         ",\"kernel_channels\":" + std::to_string(ap.fs.F) + ",\"n_split\":" + std::to_string(P.n_split) +
         ",\"cells_wg\":" + std::to_string(P.cells_wg) + ",\"cells_per_thread\":" + std::to_string(ap.fs.cpt) +
         ",\"lds_bytes\":" + std::to_string(ap.fs.lds) + ",\"max_slices\":" + std::to_string(ap.max_slices) +
         ",\"inverse_group\":" + std::to_string(ap.inv_group) + ",\"lcap\":" + std::to_string(ap.lcap) +
         ",\"wg_target\":" + std::to_string(ap.wg_target) +
         ",\"block\":" + std::to_string(ap.tb > 0 ? ap.tb : plan->time_block) +
         ",\"tuned_ms\":" + std::to_string(ap.tuned_ms) +
         ",\"axes\":[";
    for (int k = 0; k < P.d; ++k) {
      const AxisP& a = P.ax[k];
      if (k) s += ",";
      s += "{\"n\":" + std::to_string(a.n) + ",\"m\":" + std::to_string(a.m) + ",\"r\":" + std::to_string(a.r) +
           ",\"L\":" + std::to_string(a.L) + ",\"R\":" + std::to_string(a.R) +
           ",\"split\":" + std::to_string(a.split) + "}";
    }
    s += "],\"order\":[";
    for (int p = 0; p < P.d; ++p) s += (p ? "," : "") + std::to_string(P.pass[p].axis);
    s += "]}";
  }
  s += "]}";
  if (needed) *needed = s.size() + 1;
  if (buf && len) {
    const size_t n = std::min(len - 1, s.size());
    std::memcpy(buf, s.data(), n);
    buf[n] = 0;
  }
  return OMNI_OK;
}

int omni_stage_times(omni_plan_t plan, int32_t stage, int32_t max, float* ms, int32_t* n) {
  if (!plan || !n || (max > 0 && !ms)) return fail(OMNI_E_INVAL, "NULL argument");
  if (!plan->timing) return fail(OMNI_E_STATE, "plan was not made with OMNI_PLAN_TIMING");
  if (stage < 0 || stage > OMNI_STAGE_KERNEL) return fail(OMNI_E_INVAL, "unknown stage");
  if (plan->graph && stage != OMNI_STAGE_CALL)
    return fail(OMNI_E_STATE, "a graph plan records only the whole call (its arrays' stages overlap)");
  if (stage == OMNI_STAGE_KERNEL) {
    const int64_t cnt = std::min<int64_t>(std::min<int64_t>(plan->n_calls, kKernRing), max);
    for (int64_t j = 0; j < cnt; ++j) {
      const int slot = (int)((plan->n_calls - cnt + j) % kKernRing);
      const int k = plan->kev_n[(size_t)slot];
      float sum = 0.f;
      for (int i = 0; i < k; ++i) {
        hipEvent_t b = plan->kev[(size_t)((slot * kKernMax + i) * 2)], e = plan->kev[(size_t)((slot * kKernMax + i) * 2 + 1)];
        HIP_TRY(hipEventSynchronize(e));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, b, e));
        sum += t;
      }
      ms[j] = k ? sum / (float)k : 0.f;
    }
    *n = (int32_t)cnt;
    return OMNI_OK;
  }
  const int64_t avail = std::min<int64_t>(plan->n_calls, kTimingRing);
  const int64_t cnt = std::min<int64_t>(avail, max);
  for (int64_t j = 0; j < cnt; ++j) {
    const int64_t call = plan->n_calls - cnt + j;
    hipEvent_t b = plan->ev[(size_t)(((call % kTimingRing) * kStages + stage) * 2 + 0)];
    hipEvent_t e = plan->ev[(size_t)(((call % kTimingRing) * kStages + stage) * 2 + 1)];
    HIP_TRY(hipEventSynchronize(e));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, b, e));
    ms[j] = t;
  }
  *n = (int32_t)cnt;
  return OMNI_OK;
}

int omni_destroy(omni_plan_t plan) {
  if (!plan) return OMNI_OK;
  if (!plan->host_only) hipDeviceSynchronize();
  destroy_plan_resources(plan);
  delete plan;
  return OMNI_OK;
}

const char* omni_strerror(int code) {
  switch (code) {
    case OMNI_OK: return "success";
    case OMNI_E_INVAL: return "invalid argument";
    case OMNI_E_SHAPE: return "unsupported grid shape";
    case OMNI_E_GEOM: return "invalid array geometry";
    case OMNI_E_NODEV: return "no usable gfx950 device";
    case OMNI_E_NOMEM: return "out of memory";
    case OMNI_E_HIP: return "HIP runtime error";
    case OMNI_E_STATE: return "invalid call for this plan";
    default: return "unknown status";
  }
}

const char* omni_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// F-engine (Appendix A, steps 2-3).
// ---------------------------------------------------------------------------

extern "C" int omni_fengine(const void* raw, int64_t N, int64_t T, int32_t F, const void* gains, int32_t dtype,
                            void* volt, void* stream) {
  TraceRange range("omni_fengine");
  if (N < 1 || T < 0) return fail(OMNI_E_INVAL, "N must be >= 1 and T >= 0");
  if (F != 16 && F != 32 && F != 64) return fail(OMNI_E_SHAPE, "F-engine: F must be 16, 32 or 64 channels");
  if (dtype != OMNI_CI4 && dtype != OMNI_CI8) return fail(OMNI_E_INVAL, "F-engine output must be ci4 or ci8");
  if (T == 0) return OMNI_OK;
  if (!raw || !gains || !volt) return fail(OMNI_E_INVAL, "NULL argument");
  if ((reinterpret_cast<uintptr_t>(raw) & 15) != 0) return fail(OMNI_E_INVAL, "raw samples must be 16-byte aligned");
  if ((reinterpret_cast<uintptr_t>(gains) & 7) != 0) return fail(OMNI_E_INVAL, "gains must be 8-byte aligned");
  if (dtype == OMNI_CI8 && (reinterpret_cast<uintptr_t>(volt) & 1) != 0)
    return fail(OMNI_E_INVAL, "ci8 output must be 2-byte aligned");
  if (N > (int64_t(1) << 31) || T > (int64_t(1) << 40) / (2 * F * N))
    return fail(OMNI_E_SHAPE, "F-engine: N or T too large");
  HIP_TRY(omni::launch_fengine(raw, N, T, F, gains, dtype == OMNI_CI8, volt, static_cast<hipStream_t>(stream)));
  return OMNI_OK;
}

// ---------------------------------------------------------------------------
// Hybrid tiles (Sec. III).
// ---------------------------------------------------------------------------

struct omni_hybrid_s {
  int device = -1;
  int P = 0, nx = 0, ny = 0, F = 0;
  omni_dtype dtype = OMNI_CF32;
  int64_t N = 0, mx = 0, my = 0, Mp = 0, chunk_T = 1;
  bool fused = false;              // the y-axis transform runs inside the pair stage (P m_y <= 512)
  std::vector<double> offsets, A;  // metadata for omni_hybrid_baselines (may be empty)
  float2* d_tw32 = nullptr;        // forward tables: w_mx^q then w_my^q (float32)
  double2* d_tw64 = nullptr;       // inverse tables (float64)
  float2* d_y[2] = {nullptr, nullptr};  // the two front passes' outputs for one chunk
  double2* d_S = nullptr;          // [F][P][P][mx][my] cross-power sums
  float2* d_ws[2] = {nullptr, nullptr};  // inverse intermediates
};

namespace {

constexpr int64_t kHybridChunkBytes = int64_t(4) << 30;

void hybrid_free(omni_hybrid_s* h) {
  hipFree(h->d_tw32);
  hipFree(h->d_tw64);
  hipFree(h->d_y[0]);
  hipFree(h->d_y[1]);
  hipFree(h->d_S);
  hipFree(h->d_ws[0]);
  hipFree(h->d_ws[1]);
}

int hybrid_alloc(omni_hybrid_s* h) {
  const int64_t tiles = h->chunk_T * h->F;
  const int64_t pairs = (int64_t)h->F * h->P * h->P;
  HIP_TRY(hipMalloc(&h->d_tw32, (size_t)(h->mx + h->my) * sizeof(float2)));
  HIP_TRY(hipMalloc(&h->d_tw64, (size_t)(h->mx + h->my) * sizeof(double2)));
  HIP_TRY(hipMalloc(&h->d_y[0], (size_t)(tiles * h->P * h->mx * h->ny) * sizeof(float2)));
  if (!h->fused) HIP_TRY(hipMalloc(&h->d_y[1], (size_t)(tiles * h->P * h->Mp) * sizeof(float2)));
  HIP_TRY(hipMalloc(&h->d_S, (size_t)(pairs * h->Mp) * sizeof(double2)));
  HIP_TRY(hipMalloc(&h->d_ws[0], (size_t)(pairs * h->Mp) * sizeof(float2)));
  HIP_TRY(hipMalloc(&h->d_ws[1], (size_t)(pairs * (2 * h->nx - 1) * h->my) * sizeof(float2)));
  const int32_t desc[12] = {(int32_t)h->mx, -1, 0, (int32_t)h->my, -1, (int32_t)h->mx,
                            (int32_t)h->mx, +1, 0, (int32_t)h->my, +1, (int32_t)h->mx};
  int32_t* d_desc = nullptr;
  HIP_TRY(hipMalloc(&d_desc, sizeof(desc)));
  hipError_t e = hipMemcpy(d_desc, desc, sizeof(desc), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = omni::launch_twiddles(d_desc, 2, h->d_tw32, nullptr, 0);
  if (e == hipSuccess) e = omni::launch_twiddles(d_desc + 6, 2, nullptr, h->d_tw64, 0);
  if (e == hipSuccess) e = omni::launch_fill_f64(reinterpret_cast<double*>(h->d_S), 2 * pairs * h->Mp, 0.0, 0);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  hipFree(d_desc);
  if (e != hipSuccess) return fail(OMNI_E_HIP, std::string("hybrid plan setup: ") + hipGetErrorString(e));
  return OMNI_OK;
}

bool hybrid_side_ok(int n) { return front_axis_ok(n); }

}  // namespace

extern "C" {

int omni_hybrid_plan(omni_hybrid_t* out, int32_t P, int32_t nx, int32_t ny, int32_t nchan, int32_t dtype,
                     const double* offsets, const double* A) {
  TraceRange range("omni_hybrid_plan");
  if (!out) return fail(OMNI_E_INVAL, "NULL argument");
  *out = nullptr;
  if (P != 2 && P != 4 && P != 8 && P != 16 && P != 32) return fail(OMNI_E_SHAPE, "hybrid tiles: P must be 2, 4, 8, 16 or 32");
  if (!hybrid_side_ok(nx) || !hybrid_side_ok(ny))
    return fail(OMNI_E_SHAPE, "hybrid tiles: tile sides must be 1, 2, 4, 8, 16 or 32");
  if (nchan < 1 || nchan > 65535) return fail(OMNI_E_INVAL, "nchan must be in [1, 65535]");
  if (dtype != OMNI_CF32 && dtype != OMNI_CI8 && dtype != OMNI_CI4) return fail(OMNI_E_INVAL, "unknown sample format");
  auto h = std::make_unique<omni_hybrid_s>();
  h->P = P;
  h->nx = nx;
  h->ny = ny;
  h->F = nchan;
  h->dtype = (omni_dtype)dtype;
  h->N = (int64_t)P * nx * ny;
  h->mx = 2 * nx;
  h->my = 2 * ny;
  h->Mp = h->mx * h->my;
  if (offsets) h->offsets.assign(offsets, offsets + 2 * P);
  if (A) h->A.assign(A, A + 4);
  const int64_t per_t = (int64_t)h->F * h->P * h->Mp * (int64_t)sizeof(float2);
  h->chunk_T = std::max<int64_t>(1, std::min<int64_t>(kChunkMax, kHybridChunkBytes / per_t));
  // the fused pair stage: a work-group owns 512 / (P m_y) rows kappa_x, which must divide m_x
  if (omni::xengine_fused_ok(P, ny)) {
    const int64_t rows = 512 / (P * h->my);
    h->fused = rows >= 1 && h->mx % rows == 0;
  }
  int rc = check_device(&h->device);
  if (rc) return rc;
  rc = hybrid_alloc(h.get());
  if (rc) {
    hybrid_free(h.get());
    return rc;
  }
  *out = h.release();
  return OMNI_OK;
}

int omni_hybrid_correlate(omni_hybrid_t h, const void* volt, int64_t T, void* vis, void* stream, uint32_t flags) {
  TraceRange range("omni_hybrid_correlate");
  if (!h) return fail(OMNI_E_INVAL, "NULL hybrid plan");
  if (T < 0) return fail(OMNI_E_INVAL, "T < 0");
  if (T > 0 && !volt) return fail(OMNI_E_INVAL, "volt is NULL");
  if (!(flags & OMNI_NO_FINALIZE) && !vis) return fail(OMNI_E_INVAL, "vis is NULL");
  if (flags & ~(OMNI_NO_RESET | OMNI_NO_FINALIZE)) return fail(OMNI_E_INVAL, "unknown flag");
  const size_t sb = sample_bytes(h->dtype);
  if (T > 0 && (reinterpret_cast<uintptr_t>(volt) & (sb == 1 ? 0 : sb == 2 ? 1 : 3)) != 0)
    return fail(OMNI_E_INVAL, "volt is not aligned to its sample size");
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != h->device) return fail(OMNI_E_STATE, "current HIP device is not the plan's device");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool accumulate = (flags & OMNI_NO_RESET) != 0;
  const int64_t pairs = (int64_t)h->F * h->P * h->P;
  if (T == 0 && !accumulate)
    HIP_TRY(omni::launch_fill_f64(reinterpret_cast<double*>(h->d_S), 2 * pairs * h->Mp, 0.0, st));
  for (int64_t c0 = 0; c0 < T; c0 += h->chunk_T) {
    const int64_t tc = std::min<int64_t>(h->chunk_T, T - c0);
    const void* src = static_cast<const char*>(volt) + (size_t)(c0 * h->F * h->N) * sb;
    // each tile's zero-padded 2-D transform: axis x, then axis y
    HIP_TRY(omni::launch_front_axis(fmt_of(h->dtype), src, h->d_y[0], h->d_tw32, tc * h->F, h->P, h->nx, (int)h->mx,
                                    std::max<int>(1, (int)h->mx / 16), h->ny, h->N, h->P * h->mx * h->ny, st, false,
                                    1.f));
    const int acc = (accumulate || c0 > 0) ? 1 : 0;
    if (h->fused) {
      // y-axis transform inside the pair stage
      HIP_TRY(omni::launch_xengine_fused(h->d_y[0], tc, h->F, h->P, (int)h->mx, h->ny, h->d_tw32 + h->mx, h->d_S, acc,
                                         st));
      continue;
    }
    HIP_TRY(omni::launch_front_axis(0, h->d_y[0], h->d_y[1], h->d_tw32 + h->mx, tc * h->F, h->P * h->mx, h->ny,
                                    (int)h->my, std::max<int>(1, (int)h->my / 16), 1, h->P * h->mx * h->ny,
                                    h->P * h->Mp, st, false, 1.f));
    HIP_TRY(omni::launch_xengine(h->d_y[1], tc, h->F, h->P, h->Mp, h->d_S, acc, st));
  }
  if (!(flags & OMNI_NO_FINALIZE)) {
    HIP_TRY(omni::launch_narrow(h->d_S, h->d_ws[0], pairs * h->Mp, st));
    HIP_TRY(omni::launch_inverse_axis(false, false, h->d_ws[0], h->d_ws[1], h->d_tw64, pairs, (int)h->mx, h->nx,
                                      h->my, 1.0, st));
    HIP_TRY(omni::launch_inverse_axis(false, true, h->d_ws[1], vis, h->d_tw64 + h->mx, pairs * (2 * h->nx - 1),
                                      (int)h->my, h->ny, 1, 1.0 / (double)h->Mp, st));
  }
  return OMNI_OK;
}

int omni_hybrid_baselines(omni_hybrid_t h, double* uv) {
  if (!h || !uv) return fail(OMNI_E_INVAL, "NULL argument");
  if (h->offsets.empty() || h->A.empty()) return fail(OMNI_E_STATE, "plan has no tile offsets or lattice matrix");
  size_t i = 0;
  for (int p = 0; p < h->P; ++p)
    for (int q = 0; q < h->P; ++q)
      for (int dx = -(h->nx - 1); dx < h->nx; ++dx)
        for (int dy = -(h->ny - 1); dy < h->ny; ++dy) {
          uv[i++] = h->offsets[2 * p] - h->offsets[2 * q] + (h->A[0] * dx + h->A[1] * dy);
          uv[i++] = h->offsets[2 * p + 1] - h->offsets[2 * q + 1] + (h->A[2] * dx + h->A[3] * dy);
        }
  return OMNI_OK;
}

int omni_hybrid_destroy(omni_hybrid_t h) {
  if (!h) return OMNI_OK;
  hipDeviceSynchronize();
  hybrid_free(h);
  delete h;
  return OMNI_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Physical-baseline fold (Sec. II.D) and baseline distributions (Sec. III).
// ---------------------------------------------------------------------------

struct omni_fold_s {
  int device = -1;
  int F = 0;                 // channels of the array (capacity of dmax)
  omni::FoldGeom g;
  omni::RadialGeom rg;
  int64_t npix = 0, nbins = 0, origin = -1;
  int boxcar = 1;
  uint32_t* d_cell = nullptr;  // cells sorted by pixel [cells]
  uint32_t* d_off = nullptr;   // per-pixel offsets into d_cell [npix + 1]
  uint32_t* d_pix = nullptr;   // pixels sorted by radial bin [npix]
  uint32_t* d_boff = nullptr;  // per-bin offsets into d_pix [nbins + 1]
  double* d_dmax = nullptr;    // per-channel largest pixel [F]
};

namespace {

void fold_free(omni_fold_s* f) {
  hipFree(f->d_cell);
  hipFree(f->d_off);
  hipFree(f->d_pix);
  hipFree(f->d_boff);
  hipFree(f->d_dmax);
}

int bits_for(int64_t v) {
  int b = 1;
  while (b < 32 && (int64_t(1) << b) <= v) ++b;
  return b;
}

// Sort (key, value) pairs held in k0/v0 into k1/v1 and build the offsets of the groups 0..n_groups - 1;
// checks that every element fell into a group.
int sort_into_groups(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n, int64_t n_groups,
                     uint32_t* off) {
  size_t tmp_bytes = 0;
  const int kb = bits_for(n_groups);
  HIP_TRY(omni::sort_pairs(nullptr, &tmp_bytes, k0, k1, v0, v1, n, kb, nullptr));
  void* tmp = nullptr;
  HIP_TRY(hipMalloc(&tmp, std::max<size_t>(tmp_bytes, 16)));
  hipError_t e = omni::sort_pairs(tmp, &tmp_bytes, k0, k1, v0, v1, n, kb, nullptr);
  if (e == hipSuccess) e = omni::launch_group_offsets(k1, n, off, n_groups, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  hipFree(tmp);
  if (e != hipSuccess) return fail(OMNI_E_HIP, std::string("fold plan sort: ") + hipGetErrorString(e));
  uint32_t last = 0;
  HIP_TRY(hipMemcpy(&last, off + n_groups, sizeof(uint32_t), hipMemcpyDeviceToHost));
  if ((int64_t)last != n) return fail(OMNI_E_HIP, "fold plan: an element fell outside every group");
  return OMNI_OK;
}

int fold_build(omni_fold_s* f) {
  const int64_t cells = f->g.cells;
  uint32_t *k0 = nullptr, *v0 = nullptr, *k1 = nullptr;
  const int64_t n_tmp = std::max(cells, f->npix);
  auto release = [&]() {
    hipFree(k0);
    hipFree(v0);
    hipFree(k1);
  };
  hipError_t e = hipMalloc(&k0, (size_t)n_tmp * 4);
  if (e == hipSuccess) e = hipMalloc(&v0, (size_t)n_tmp * 4);
  if (e == hipSuccess) e = hipMalloc(&k1, (size_t)n_tmp * 4);
  if (e == hipSuccess) e = hipMalloc(&f->d_cell, (size_t)cells * 4);
  if (e == hipSuccess) e = hipMalloc(&f->d_off, (size_t)(f->npix + 1) * 4);
  if (e == hipSuccess) e = hipMalloc(&f->d_pix, (size_t)f->npix * 4);
  if (e == hipSuccess) e = hipMalloc(&f->d_dmax, (size_t)f->F * sizeof(double));
  if (e == hipSuccess) e = omni::launch_fold_keys(f->g, k0, v0, nullptr);
  if (e != hipSuccess) {
    release();
    return fail(e == hipErrorOutOfMemory ? OMNI_E_NOMEM : OMNI_E_HIP, std::string("fold plan: ") + hipGetErrorString(e));
  }
  int rc = sort_into_groups(k0, v0, k1, f->d_cell, cells, f->npix, f->d_off);
  if (rc) {
    release();
    return rc;
  }
  // radial bins of the pixels
  uint32_t* d_max = nullptr;
  e = hipMalloc(&d_max, sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(d_max, 0, sizeof(uint32_t));
  if (e == hipSuccess) e = omni::launch_radial_keys(f->rg, k0, v0, d_max, nullptr);
  uint32_t max_bin = 0;
  if (e == hipSuccess) e = hipMemcpy(&max_bin, d_max, sizeof(uint32_t), hipMemcpyDeviceToHost);
  hipFree(d_max);
  if (e == hipSuccess && (int64_t)max_bin >= (int64_t(1) << 31)) e = hipErrorInvalidValue;
  if (e == hipSuccess) {
    f->nbins = (int64_t)max_bin + 1;
    e = hipMalloc(&f->d_boff, (size_t)(f->nbins + 1) * 4);
  }
  if (e != hipSuccess) {
    release();
    return fail(e == hipErrorOutOfMemory ? OMNI_E_NOMEM : OMNI_E_HIP,
                std::string("fold plan radial bins: ") + hipGetErrorString(e));
  }
  rc = sort_into_groups(k0, v0, k1, f->d_pix, f->npix, f->nbins, f->d_boff);
  release();
  return rc;
}

bool finite_positive(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

extern "C" {

int omni_fold_plan(omni_fold_t* out, omni_plan_t plan, int32_t array, const omni_fold_opts* opts) {
  TraceRange range("omni_fold_plan");
  if (!out || !plan) return fail(OMNI_E_INVAL, "NULL argument");
  *out = nullptr;
  if (array < 0 || (size_t)array >= plan->arrays.size()) return fail(OMNI_E_INVAL, "array index out of range");
  const ArrayPlan& ap = plan->arrays[(size_t)array];
  if (ap.beams) return fail(OMNI_E_STATE, "beam-space plan: its cells along the lowest level are pointings");
  omni_fold_opts o = {1.0, 1.0, 1.0, 1.0, 1, 0};
  if (opts) o = *opts;
  if (!finite_positive(o.du) || !finite_positive(o.dv) || !finite_positive(o.dr) || !finite_positive(o.radius_scale))
    return fail(OMNI_E_INVAL, "du, dv, dr and radius_scale must be finite and positive");
  if (o.boxcar < 1 || o.boxcar % 2 == 0) return fail(OMNI_E_INVAL, "boxcar width must be odd and >= 1");
  if (ap.A.empty()) return fail(OMNI_E_STATE, "plan has no lattice matrices");
  if (plan->host_only) return fail(OMNI_E_STATE, "host-only plan");
  if (ap.levels > omni::kFoldMaxLevels) return fail(OMNI_E_SHAPE, "too many levels for the fold");
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != plan->device) return fail(OMNI_E_STATE, "current HIP device is not the plan's device");
  auto f = std::make_unique<omni_fold_s>();
  f->device = plan->device;
  f->F = ap.F;
  f->boxcar = o.boxcar;
  omni::FoldGeom& g = f->g;
  g.levels = ap.levels;
  g.cells = 1;
  for (int k = 0; k < 2 * ap.levels; ++k) {
    g.n[k] = ap.dims[(size_t)k];
    g.cells *= 2 * g.n[k] - 1;
  }
  // largest |b_x|, |b_y| over the cells: each lattice vector at its extreme lag
  double X = 0.0, Y = 0.0;
  for (int l = 0; l < ap.levels; ++l) {
    for (int c = 0; c < 4; ++c) g.A[l][c] = ap.A[(size_t)(4 * l + c)];
    const double nx1 = g.n[2 * l] - 1, ny1 = g.n[2 * l + 1] - 1;
    X += std::fabs(g.A[l][0]) * nx1 + std::fabs(g.A[l][1]) * ny1;
    Y += std::fabs(g.A[l][2]) * nx1 + std::fabs(g.A[l][3]) * ny1;
  }
  g.du = o.du;
  g.dv = o.dv;
  const double cxd = std::nearbyint(X / o.du), cyd = std::nearbyint(Y / o.dv);
  if (!(cxd < 1e9 && cyd < 1e9)) return fail(OMNI_E_SHAPE, "fold image too large");
  g.cx = (int64_t)cxd;
  g.cy = (int64_t)cyd;
  g.nx = 2 * g.cx + 1;
  g.ny = 2 * g.cy + 1;
  f->npix = g.nx * g.ny;
  if (f->npix >= (int64_t(1) << 31)) return fail(OMNI_E_SHAPE, "fold image above 2^31 pixels (choose larger du, dv)");
  if (g.cells >= (int64_t(1) << 32)) return fail(OMNI_E_SHAPE, "too many visibility cells for the fold");
  f->origin = o.zero_origin ? g.cy * g.nx + g.cx : -1;
  f->rg.cx = g.cx;
  f->rg.cy = g.cy;
  f->rg.nx = g.nx;
  f->rg.ny = g.ny;
  f->rg.du = o.du;
  f->rg.dv = o.dv;
  f->rg.dr = o.dr;
  f->rg.scale = o.radius_scale;
  const int rc = fold_build(f.get());
  if (rc) {
    fold_free(f.get());
    return rc;
  }
  *out = f.release();
  return OMNI_OK;
}

int omni_fold_shape(omni_fold_t fold, int64_t* ny, int64_t* nx, int64_t* nbins) {
  if (!fold || !ny || !nx || !nbins) return fail(OMNI_E_INVAL, "NULL argument");
  *ny = fold->g.ny;
  *nx = fold->g.nx;
  *nbins = fold->nbins;
  return OMNI_OK;
}

int omni_fold(omni_fold_t fold, const void* vis, int32_t nchan, void* image, void* stream) {
  TraceRange range("omni_fold");
  if (!fold || !vis || !image) return fail(OMNI_E_INVAL, "NULL argument");
  if (nchan < 1 || nchan > fold->F) return fail(OMNI_E_SHAPE, "nchan must be in [1, F] of the array");
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != fold->device) return fail(OMNI_E_STATE, "current HIP device is not the fold's device");
  HIP_TRY(omni::launch_fold_gather(static_cast<const float2*>(vis), fold->g.cells, fold->d_cell, fold->d_off,
                                   fold->npix, nchan, fold->origin, static_cast<double2*>(image),
                                   static_cast<hipStream_t>(stream)));
  return OMNI_OK;
}

int omni_baseline_profile(omni_fold_t fold, const void* image, int32_t nchan, void* map, void* hist, void* smooth,
                          void* stream) {
  TraceRange range("omni_baseline_profile");
  if (!fold || !image) return fail(OMNI_E_INVAL, "NULL argument");
  if (smooth && !hist) return fail(OMNI_E_INVAL, "smooth needs hist");
  if (nchan < 1 || nchan > fold->F) return fail(OMNI_E_SHAPE, "nchan must be in [1, F] of the array");
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != fold->device) return fail(OMNI_E_STATE, "current HIP device is not the fold's device");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double2* im = static_cast<const double2*>(image);
  if (map) {
    HIP_TRY(omni::launch_channel_max(im, fold->npix, nchan, fold->d_dmax, st));
    HIP_TRY(omni::launch_asinh_map(im, fold->npix, nchan, fold->d_dmax, static_cast<double*>(map), st));
  }
  if (hist)
    HIP_TRY(omni::launch_radial_sum(im, fold->npix, nchan, fold->d_pix, fold->d_boff, fold->nbins,
                                    static_cast<double*>(hist), st));
  if (smooth)
    HIP_TRY(omni::launch_boxcar(static_cast<const double*>(hist), fold->nbins, nchan, fold->boxcar,
                                static_cast<double*>(smooth), st));
  return OMNI_OK;
}

int omni_fold_destroy(omni_fold_t fold) {
  if (!fold) return OMNI_OK;
  hipDeviceSynchronize();
  fold_free(fold);
  delete fold;
  return OMNI_OK;
}

}  // extern "C"
