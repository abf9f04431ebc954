// batch_k5.hip -- kernel kind 5 of the batched patch path: LDS-staged 6th order, 16x16 tiles.
#include "batch_stage.h"

namespace chemora {

template <>
hipError_t launch_batch_kind<5>(int precision, bool ko, int stage, const Batch& b,
                                  unsigned grid, hipStream_t s) {
  return launch_stage_kind<5>(precision, ko, stage, b, grid, s);
}

template <>
int batch_per_cu<5>(int precision, bool ko) {
  return per_cu_kind<5>(precision, ko);
}

}  // namespace chemora
