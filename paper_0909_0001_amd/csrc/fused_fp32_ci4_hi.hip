// General fused correlator (float32 form): instantiations for ci4 samples, 8, 16, 32 cells per thread.
#include "fused_fp32.hpp"

namespace omni {

hipError_t launch_fused_fp32_ci4_hi(int cpt, const void* src, int64_t T, int64_t tps, const float2* tw,
                                    double* partial, const FusedP& P, int grid, size_t lds, hipStream_t st) {
  switch (cpt) {
    case 8: return launch_fused_t<FMT_CI4, 8>(src, T, tps, tw, partial, P, grid, lds, st);
    case 16: return launch_fused_t<FMT_CI4, 16>(src, T, tps, tw, partial, P, grid, lds, st);
    case 32: return launch_fused_t<FMT_CI4, 32>(src, T, tps, tw, partial, P, grid, lds, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace omni
