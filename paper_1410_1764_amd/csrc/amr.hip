// amr.hip -- coupling of two refinement levels at ratio 2 (Sec. IV: the
// mesh-refinement driver fills a fine patch's ghost zones from the next
// coarser level and writes fine results back onto it).
//
// Geometry is integer: with h_c = 2 h_f on every axis and the fine origin
// `off` fine spacings from the coarse origin (checked on the host), fine
// point i sits at fine-unit coordinate q = off + i from the coarse origin;
// q even coincides with coarse point q/2, q odd lies half-way between
// coarse points (q-1)/2 and (q+1)/2.
//
// Prolongation (prolong_box.h): every fine ghost point gets, per axis, the
// coarse value (coincident) or the degree-5 Lagrange interpolant through six
// coarse points (half-way); the tensor product over the axes; up to three
// coarse time levels combined with Lagrange weights in time that the host
// computes.  One 512-thread workgroup per (box, grid function), boxes of
// about 3000 fine points (32 x 32 slab columns, 32-point band boxes 32
// planes deep up to g = 5; 32 x 16 and 16 planes above, so that the LDS
// stays within 64 KiB).
//
// Restriction (injection): every coarse interior point that coincides with a
// fine interior point takes that fine value.  One thread per (point, grid
// function) over the overlap box computed on the host.
#include "prolong_box.h"

namespace chemora {

namespace {

struct ProlongArgs {
  Geo C, F;
  int off[3];
  const double* yc[kMaxTimeLevels];
  double wt[kMaxTimeLevels];
  int ntimes;
  double* yf;
  BoxGrid bg;
};

constexpr int kProlongThreads = 512;  // 8 waves per box

// One workgroup per (box, grid function).  Workgroup b runs on XCD b % 8;
// xcd_tile gives each XCD a contiguous range of boxes, so that neighbouring
// boxes' shared footprint lines meet in one L2.
__global__ void __launch_bounds__(kProlongThreads) prolong_kernel(ProlongArgs a) {
  extern __shared__ double lds[];
  Box x;
  box_geometry(a.bg, a.C, a.F, a.off, xcd_tile((int)blockIdx.x, (int)gridDim.x), x);
  const int v = (int)blockIdx.y;
  const double* lev[kMaxTimeLevels];
#pragma unroll
  for (int l = 0; l < kMaxTimeLevels; ++l) lev[l] = a.yc[l] + (long long)v * a.C.sv;
  prolong_box(x, a.C, a.F, lev, a.wt, a.ntimes, a.yf + a.F.off0 + (long long)v * a.F.sv, lds,
              lds + a.bg.lds_a);
}

struct RestrictArgs {
  Geo C, F;
  int off[3];
  int lo[3], cnt[3];  // coarse interior box that coincides with fine interior points
  double* yc;
  const double* yf;
};

__global__ void __launch_bounds__(256) restrict_kernel(RestrictArgs a) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)a.cnt[0] * a.cnt[1] * a.cnt[2];
  if (p >= total) return;
  const int v = blockIdx.y;
  const int i = a.lo[0] + (int)(p % a.cnt[0]);
  const long long r = p / a.cnt[0];
  const int j = a.lo[1] + (int)(r % a.cnt[1]);
  const int k = a.lo[2] + (int)(r / a.cnt[1]);
  const int fi = 2 * i - a.off[0], fj = 2 * j - a.off[1], fk = 2 * k - a.off[2];
  const Geo &C = a.C, &F = a.F;
  a.yc[C.off0 + (long long)v * C.sv + i + (long long)j * C.sy + (long long)k * C.sz] =
      a.yf[F.off0 + (long long)v * F.sv + fi + (long long)fj * F.sy + (long long)fk * F.sz];
}

}  // namespace

hipError_t launch_prolong(const Geo& C, const double* const* yc, const double* wt, int ntimes,
                          const Geo& F, const int off[3], int nvar, double* yf, hipStream_t s) {
  ProlongArgs a{};
  a.C = C;
  a.F = F;
  for (int d = 0; d < 3; ++d) a.off[d] = off[d];
  for (int l = 0; l < ntimes; ++l) {
    a.yc[l] = yc[l];
    a.wt[l] = wt[l];
  }
  a.ntimes = ntimes;
  a.yf = yf;
  // box shapes: the largest of these whose LDS fits in 64 KiB
  const int shapes[3][3] = {{32, 32, 32}, {32, 16, 16}, {32, 8, 16}};
  for (const auto& sh : shapes) {
    a.bg = make_box_grid(F, sh[0], sh[1], 32, 32, sh[2]);
    if (8LL * (a.bg.lds_a + a.bg.lds_b) <= 65536) break;
  }
  if (8LL * (a.bg.lds_a + a.bg.lds_b) > 65536 || a.bg.boxes < 1 || nvar > 65535)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)a.bg.boxes, (unsigned)nvar);
  hipLaunchKernelGGL(prolong_kernel, grid, dim3(kProlongThreads),
                     (size_t)8 * (a.bg.lds_a + a.bg.lds_b), s, a);
  return hipGetLastError();
}

hipError_t launch_restrict(const Geo& C, double* yc, const Geo& F, const double* yf,
                           const int off[3], const int lo[3], const int cnt[3], int nvar,
                           hipStream_t s) {
  RestrictArgs a{};
  a.C = C;
  a.F = F;
  for (int d = 0; d < 3; ++d) {
    a.off[d] = off[d];
    a.lo[d] = lo[d];
    a.cnt[d] = cnt[d];
  }
  a.yc = yc;
  a.yf = yf;
  const long long total = (long long)cnt[0] * cnt[1] * cnt[2];
  if (total == 0) return hipSuccess;
  const dim3 grid((unsigned)((total + 255) / 256), (unsigned)nvar);
  hipLaunchKernelGGL(restrict_kernel, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace chemora
