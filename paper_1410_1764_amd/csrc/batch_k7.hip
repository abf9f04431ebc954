// batch_k7.hip -- kernel kind 7 of the batched patch path: LDS-staged 4th
// order in z-blocked 32x8x2 tiles (mixed precision, no dissipation).
// The point code fences every mixed derivative, as in the single-grid
// z-blocked kernels, so that it fits two waves per SIMD.
#define CHEMORA_BSSN_FENCE 3
#include "batch_stage.h"

namespace chemora {

template <>
hipError_t launch_batch_kind<7>(int precision, bool ko, bool par, int stage, const Batch& b,
                                  unsigned grid, hipStream_t s) {
  return launch_stage_kind<7>(precision, ko, par, stage, b, grid, s);
}

template <>
int batch_per_cu<7>(int precision, bool ko, bool par) {
  return per_cu_kind<7>(precision, ko, par);
}

}  // namespace chemora
