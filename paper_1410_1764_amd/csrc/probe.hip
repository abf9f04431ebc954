// probe.hip -- streaming copy used as the bandwidth / hardware-counter
// reference: every byte read once and written once, 16-byte accesses.
#include "internal.h"

namespace chemora {
namespace {

__global__ void __launch_bounds__(256) copy_kernel(double2* __restrict__ dst,
                                                   const double2* __restrict__ src, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride)
    dst[t] = src[t];
}

}  // namespace

hipError_t launch_probe_copy(void* dst, const void* src, long long nbytes, hipStream_t s) {
  const long long n = nbytes / 16;
  if (n == 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 256 * 32) blocks = 256 * 32;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<double2*>(dst), static_cast<const double2*>(src), n);
  return hipGetLastError();
}

}  // namespace chemora
