// Host-side exercise of the planner and the argument checks of every entry point, built with AddressSanitizer
// on the host code of the library (tests/test_planner_asan.py builds and runs it).  Runs without a GPU: plans are
// host-only (geometry, shapes, baselines, description) and device entry points are driven only into their
// argument checks.  Any out-of-bounds access or use after free aborts the process with a report; a wrong status
// code exits with 1.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "omniscope.h"

namespace {

int failures = 0;

void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s (last error: %s)\n", what, omni_last_error());
    ++failures;
  }
}

omni_opts host_opts(omni_dtype dtype, omni_form form, uint32_t extra = 0) {
  omni_opts o{};
  o.dtype = dtype;
  o.form = form;
  o.flags = OMNI_PLAN_HOST_ONLY | extra;
  return o;
}

// Every geometry query of a host-only plan, with buffers sized exactly from the plan's own answers.
void query_plan(omni_plan_t p) {
  int32_t na = 0;
  expect(omni_n_arrays(p, &na) == OMNI_OK && na >= 1, "n_arrays");
  for (int32_t a = 0; a < na; ++a) {
    int32_t nd = 0;
    int64_t shape[17] = {};
    expect(omni_vis_shape(p, a, &nd, shape) == OMNI_OK && nd >= 2 && nd <= 17, "vis_shape");
    int64_t cells = 1;
    for (int i = 1; i < nd; ++i) cells *= shape[i];
    std::vector<double> uv((size_t)cells * 2);
    const int rc = omni_baselines(p, a, uv.data());
    expect(rc == OMNI_OK || rc == OMNI_E_STATE, "baselines");
  }
  size_t bytes = 0;
  expect(omni_accumulator_bytes(p, &bytes) == OMNI_OK && bytes > 0, "accumulator_bytes");
  size_t need = 0;
  expect(omni_plan_describe(p, nullptr, 0, &need) == OMNI_OK && need > 1, "describe size");
  std::vector<char> buf(need);
  expect(omni_plan_describe(p, buf.data(), buf.size(), nullptr) == OMNI_OK && buf[need - 1] == 0, "describe");
  char small[8];
  expect(omni_plan_describe(p, small, sizeof small, nullptr) == OMNI_OK && small[7] == 0, "describe truncated");
  // device entry points on a host-only plan: refused before any device access
  expect(omni_correlate(p, nullptr, 0, nullptr, nullptr, 0) != OMNI_OK || na != 1, "correlate on host-only plan");
  expect(omni_direct_correlate(p, nullptr, 1, nullptr, nullptr) != OMNI_OK, "direct on host-only plan");
  float ms[4];
  int32_t n = 0;
  omni_stage_times(p, 0, 4, ms, &n);
}

}  // namespace

int main() {
  // valid geometries: one to four levels, odd and even sides, rotated and sheared lattices, a batch
  {
    const int32_t dims[] = {16, 16};
    omni_plan_t p = nullptr;
    omni_opts o = host_opts(OMNI_CI4, OMNI_FORM_MIXED);
    expect(omni_plan(&p, 1, dims, nullptr, 64, &o) == OMNI_OK, "plan 16x16");
    query_plan(p);
    omni_destroy(p);
  }
  {
    const int32_t dims[] = {3, 3, 3, 3, 5, 3};
    const double A[] = {40, -10, 10, 40, 8, 2, 0, 8, 1, 0, 0, 1};
    omni_plan_t p = nullptr;
    omni_opts o = host_opts(OMNI_CI8, OMNI_FORM_FP32);
    expect(omni_plan(&p, 3, dims, A, 3, &o) == OMNI_OK, "plan 3-level");
    query_plan(p);
    omni_destroy(p);
  }
  {
    const int32_t dims[] = {2, 3, 1, 4, 3, 1, 2, 2};
    const double A[] = {64, 0, 0, 64, 16, 0, 0, 16, 4, 1, 0, 4, 1, 0, 0, 1};
    omni_plan_t p = nullptr;
    omni_opts o = host_opts(OMNI_CF32, OMNI_FORM_FP32);
    expect(omni_plan(&p, 4, dims, A, 2, &o) == OMNI_OK, "plan 4-level");
    query_plan(p);
    omni_destroy(p);
  }
  {
    const int32_t d0[] = {32, 32}, d1[] = {8, 8, 8, 8}, d2[] = {4, 4, 16, 16};
    omni_array_desc arr[] = {{1, d0, nullptr, 4}, {2, d1, nullptr, 2}, {2, d2, nullptr, 1}};
    omni_plan_t p = nullptr;
    omni_opts o = host_opts(OMNI_CI4, OMNI_FORM_MIXED, OMNI_PLAN_BEAMS);
    const int rc = omni_plan_batch(&p, 3, arr, &o);  // refused (a one-level array has no blocks): a status
    expect(rc == OMNI_OK || !p, "batch plan with beams");
    if (rc == OMNI_OK) {
      query_plan(p);
      omni_destroy(p);
    }
    o = host_opts(OMNI_CI4, OMNI_FORM_MIXED);
    expect(omni_plan_batch(&p, 3, arr, &o) == OMNI_OK, "batch plan");
    query_plan(p);
    omni_destroy(p);
  }
  // invalid plans: each refused with a status, nothing allocated
  {
    omni_plan_t p = nullptr;
    omni_opts o = host_opts(OMNI_CI8, OMNI_FORM_FP32);
    const int32_t zero[] = {0, 4};
    expect(omni_plan(&p, 1, zero, nullptr, 1, &o) != OMNI_OK && !p, "zero side");
    const int32_t dims5[] = {2, 2, 2, 2, 2, 2, 2, 2, 2, 2};
    expect(omni_plan(&p, 5, dims5, nullptr, 1, &o) != OMNI_OK && !p, "d > 8");
    expect(omni_plan(&p, 0, dims5, nullptr, 1, &o) != OMNI_OK && !p, "levels = 0");
    const int32_t d2[] = {4, 4};
    const double nan_a[] = {NAN, 0, 0, 1};
    expect(omni_plan(&p, 1, d2, nan_a, 1, &o) == OMNI_E_GEOM && !p, "non-finite A");
    const int32_t dc[] = {2, 2, 2, 2};
    const double collide[] = {1, 0, 0, 1, 1, 0, 0, 1};  // inner grid on the outer lattice: positions repeat
    expect(omni_plan(&p, 2, dc, collide, 1, &o) == OMNI_E_GEOM && !p, "colliding positions");
    expect(omni_plan(&p, 1, d2, nullptr, 0, &o) != OMNI_OK && !p, "nchan = 0");
    expect(omni_plan(nullptr, 1, d2, nullptr, 1, &o) == OMNI_E_INVAL, "out NULL");
    omni_opts bad = o;
    bad.flags |= 0x80u;
    expect(omni_plan(&p, 1, d2, nullptr, 1, &bad) == OMNI_E_INVAL && !p, "unknown flag");
    bad = o;
    bad.dtype = (omni_dtype)9;
    expect(omni_plan(&p, 1, d2, nullptr, 1, &bad) == OMNI_E_INVAL && !p, "unknown dtype");
    expect(omni_plan_batch(&p, 0, nullptr, &o) == OMNI_E_INVAL && !p, "empty batch");
  }
  // device entry points driven into their argument checks
  {
    expect(omni_fengine(nullptr, 0, 1, 64, nullptr, OMNI_CI4, nullptr, nullptr) == OMNI_E_INVAL, "fengine N = 0");
    expect(omni_fengine(nullptr, 4, 1, 48, nullptr, OMNI_CI4, nullptr, nullptr) == OMNI_E_SHAPE, "fengine F = 48");
    expect(omni_fengine(nullptr, 4, 0, 64, nullptr, OMNI_CI4, nullptr, nullptr) == OMNI_OK, "fengine T = 0");
    omni_hybrid_t h = nullptr;
    expect(omni_hybrid_plan(&h, 3, 4, 4, 1, OMNI_CI4, nullptr, nullptr) != OMNI_OK && !h, "hybrid P = 3");
    expect(omni_hybrid_correlate(nullptr, nullptr, 0, nullptr, nullptr, 0) == OMNI_E_INVAL, "hybrid NULL");
    expect(omni_fold_plan(nullptr, nullptr, 0, nullptr) == OMNI_E_INVAL, "fold NULL");
    expect(omni_destroy(nullptr) == OMNI_OK, "destroy NULL");
    expect(omni_hybrid_destroy(nullptr) == OMNI_OK, "hybrid destroy NULL");
    expect(omni_fold_destroy(nullptr) == OMNI_OK, "fold destroy NULL");
  }
  for (int c = 1; c >= -8; --c) expect(omni_strerror(c) != nullptr, "strerror");
  if (failures) return 1;
  std::printf("planner host checks passed\n");
  return 0;
}
