// batch_k3.hip -- kernel kind 3 of the batched patch path: LDS-staged 6th order, 32x8 tiles.
#include "batch_stage.h"

namespace chemora {

template <>
hipError_t launch_batch_kind<3>(int precision, bool ko, bool par, int stage, const Batch& b,
                                  unsigned grid, hipStream_t s) {
  return launch_stage_kind<3>(precision, ko, par, stage, b, grid, s);
}

template <>
int batch_per_cu<3>(int precision, bool ko, bool par) {
  return per_cu_kind<3>(precision, ko, par);
}

}  // namespace chemora
