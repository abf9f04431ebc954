// batch_k3.hip -- kernel kind 3 of the batched patch path: LDS-staged 6th order, 32x8 tiles.
#include "batch_stage.h"

namespace chemora {

template <>
hipError_t launch_batch_kind<3>(int precision, bool ko, int stage, const Batch& b,
                                  unsigned grid, hipStream_t s) {
  return launch_stage_kind<3>(precision, ko, stage, b, grid, s);
}

template <>
int batch_per_cu<3>(int precision, bool ko) {
  return per_cu_kind<3>(precision, ko);
}

}  // namespace chemora
