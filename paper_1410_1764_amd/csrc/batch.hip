// batch.hip -- placeholder until the persistent batch kernel lands.
#include "internal.h"

extern "C" {
int chemora_batch_step(const chemora_patch*, int32_t, void*, double, double, int32_t,
                       chemora_stream) {
  return CHEMORA_ERR_UNSUPPORTED;
}
int64_t chemora_batch_meta_bytes(int32_t) { return -1; }
int chemora_batch_release(void*) { return CHEMORA_ERR_UNSUPPORTED; }
int chemora_autotune(const chemora_patch*, int32_t, void*, const char*) {
  return CHEMORA_ERR_UNSUPPORTED;
}
int chemora_batch_tile(const int32_t[3], int32_t, int32_t[3]) { return CHEMORA_ERR_UNSUPPORTED; }
}
