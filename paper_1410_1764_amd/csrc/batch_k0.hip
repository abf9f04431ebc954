// batch_k0.hip -- kernel kind 0 of the batched patch path: the cached-load instances (stencil neighbours through the caches, a tile of
// tz planes per patch).
#include "batch_stage.h"

namespace chemora {

template <>
hipError_t launch_batch_kind<0>(int precision, bool ko, bool par, int stage, const Batch& b,
                                  unsigned grid, hipStream_t s) {
  return launch_stage_kind<0>(precision, ko, par, stage, b, grid, s);
}

template <>
int batch_per_cu<0>(int precision, bool ko, bool par) {
  return per_cu_kind<0>(precision, ko, par);
}

}  // namespace chemora
