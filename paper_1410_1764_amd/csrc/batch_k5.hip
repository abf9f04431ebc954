// batch_k5.hip -- kernel kind 5 of the batched patch path: LDS-staged 6th order, 16x16 tiles.
#include "batch_stage.h"

namespace chemora {

template <>
hipError_t launch_batch_kind<5>(int precision, bool ko, bool par, int stage, const Batch& b,
                                  unsigned grid, hipStream_t s) {
  return launch_stage_kind<5>(precision, ko, par, stage, b, grid, s);
}

template <>
int batch_per_cu<5>(int precision, bool ko, bool par) {
  return per_cu_kind<5>(precision, ko, par);
}

}  // namespace chemora
