// probe.hip -- reference kernels for the roofline denominators: a streaming
// copy (every byte read once and written once, 16-byte accesses; also the
// hardware-counter calibration) and an FMA throughput probe (FP64, and FP32
// as this library compiles it: unpacked).
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

// FMA throughput: every thread runs kChains independent FMA chains for
// iters steps (dependent chains, so the latency of one is hidden by the
// others and by the other waves); the sum of the chains is stored so that
// nothing is eliminated.  2 * kChains * iters flops per thread.
constexpr int kChains = 16;

__device__ __forceinline__ float fma_op(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_op(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__global__ void __launch_bounds__(256) fma_kernel(T* out, T b, T c, int iters) {
  T a[kChains];
#pragma unroll
  for (int q = 0; q < kChains; ++q) a[q] = (T)(threadIdx.x + q) * (T)1e-3;
#pragma unroll 4
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < kChains; ++q) a[q] = fma_op(a[q], b, c);
  }
  T s = (T)0;
#pragma unroll
  for (int q = 0; q < kChains; ++q) s += a[q];
  out[(long long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

long long probe_fma_threads() { return 8192LL * 256; }  // 8 waves per SIMD on 256 CUs

hipError_t launch_probe_fma(int precision, void* out, int iters, double* flops, hipStream_t s) {
  const long long threads = probe_fma_threads();
  const dim3 grid((unsigned)(threads / 256));
  if (precision == CHEMORA_MIXED)
    hipLaunchKernelGGL(fma_kernel<float>, grid, dim3(256), 0, s, static_cast<float*>(out),
                       0.999999f, 1e-7f, iters);
  else
    hipLaunchKernelGGL(fma_kernel<double>, grid, dim3(256), 0, s, static_cast<double*>(out),
                       0.999999, 1e-7, iters);
  *flops = 2.0 * kChains * (double)iters * (double)threads;
  return hipGetLastError();
}

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
