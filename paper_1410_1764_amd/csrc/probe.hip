// probe.hip -- streaming copy used as the bandwidth / hardware-counter
// reference: every byte read once and written once, 16-byte accesses.
#include "internal.h"

namespace chemora {
namespace {

// Each workgroup copies contiguous chunks of 4 x 256 16-byte elements with
// all four loads of a thread in flight before its stores (a grid-stride
// loop with one element per step measured ~10 % lower bandwidth).
typedef double d2v __attribute__((ext_vector_type(2)));
constexpr int kUnroll = 4;

__global__ void __launch_bounds__(256) copy_kernel(d2v* __restrict__ dst,
                                                   const d2v* __restrict__ src, long long n) {
  const long long chunk = (long long)kUnroll * 256;
  for (long long base = (long long)blockIdx.x * chunk; base < n;
       base += (long long)gridDim.x * chunk) {
    d2v v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const long long t = base + u * 256 + threadIdx.x;
      if (t < n) v[u] = src[t];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const long long t = base + u * 256 + threadIdx.x;
      if (t < n) dst[t] = v[u];
    }
  }
}

}  // namespace

hipError_t launch_probe_copy(void* dst, const void* src, long long nbytes, hipStream_t s) {
  const long long n = nbytes / 16;
  if (n == 0) return hipSuccess;
  long long blocks = (n + kUnroll * 256 - 1) / (kUnroll * 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<d2v*>(dst), static_cast<const d2v*>(src), n);
  return hipGetLastError();
}

}  // namespace chemora
