// batch_k1.hip -- kernel kind 1 of the batched patch path: LDS-staged 4th order, 32x8 tiles.
#include "batch_stage.h"

namespace chemora {

template <>
hipError_t launch_batch_kind<1>(int precision, bool ko, bool par, int stage, const Batch& b,
                                  unsigned grid, hipStream_t s) {
  return launch_stage_kind<1>(precision, ko, par, stage, b, grid, s);
}

template <>
int batch_per_cu<1>(int precision, bool ko, bool par) {
  return per_cu_kind<1>(precision, ko, par);
}

}  // namespace chemora
