// General fused correlator (float32 form): instantiations for ci4 samples, 1, 2, 4 cells per thread.
#include "fused_fp32.hpp"

namespace omni {

hipError_t launch_fused_fp32_ci4_lo(int cpt, const void* src, int64_t T, int64_t tps, const float2* tw,
                                    double* partial, const FusedP& P, int grid, size_t lds, hipStream_t st) {
  switch (cpt) {
    case 1: return launch_fused_t<FMT_CI4, 1>(src, T, tps, tw, partial, P, grid, lds, st);
    case 2: return launch_fused_t<FMT_CI4, 2>(src, T, tps, tw, partial, P, grid, lds, st);
    case 4: return launch_fused_t<FMT_CI4, 4>(src, T, tps, tw, partial, P, grid, lds, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace omni
