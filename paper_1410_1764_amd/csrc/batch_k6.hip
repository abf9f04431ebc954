// batch_k6.hip -- kernel kind 6 of the batched patch path: LDS-staged 8th order, 16x16 tiles.
#include "batch_stage.h"

namespace chemora {

template <>
hipError_t launch_batch_kind<6>(int precision, bool ko, bool par, int stage, const Batch& b,
                                  unsigned grid, hipStream_t s) {
  return launch_stage_kind<6>(precision, ko, par, stage, b, grid, s);
}

template <>
int batch_per_cu<6>(int precision, bool ko, bool par) {
  return per_cu_kind<6>(precision, ko, par);
}

}  // namespace chemora
