// Host dispatch of the general fused correlator (float32 form) over its instantiations, which live in
// fused_fp32_{cf32,ci8,ci4}_{lo,hi}.hip (kernel templates in fused_fp32.hpp).
#include "fused_fp32.hpp"

namespace omni {

hipError_t launch_fused_fp32(int fmt, int cpt, const void* src, int64_t T, int64_t tps, const float2* tw,
                             double* partial, const FusedP& P, int grid, size_t lds, hipStream_t st) {
  const bool lo = cpt <= 4;
  switch (fmt) {
    case FMT_CF32:
      return (lo ? launch_fused_fp32_cf32_lo : launch_fused_fp32_cf32_hi)(cpt, src, T, tps, tw, partial, P, grid, lds, st);
    case FMT_CI8:
      return (lo ? launch_fused_fp32_ci8_lo : launch_fused_fp32_ci8_hi)(cpt, src, T, tps, tw, partial, P, grid, lds, st);
    case FMT_CI4:
      return (lo ? launch_fused_fp32_ci4_lo : launch_fused_fp32_ci4_hi)(cpt, src, T, tps, tw, partial, P, grid, lds, st);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace omni
