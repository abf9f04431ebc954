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
// Prolongation: every fine ghost point gets, per axis, the coarse value
// (coincident) or the degree-5 Lagrange interpolant through the six coarse
// points at offsets -2 .. 3 from the lower neighbour (half-way), weights
// (3, -25, 150, 150, -25, 3) / 256; the tensor product over the axes.  Up to
// three coarse time levels are combined with Lagrange weights in time that
// the host computes.  One thread per (ghost point, grid function): the ghost
// shell is enumerated as the two z slabs, then the two y slabs of the
// interior planes, then the two x slabs of the interior rows, so that the
// threads of a wave share their y and z stencils and walk contiguous x.
// Along x the six taps are always read (a coincident point's weights are
// one-hot, its six-point window clamped into the coarse block), because
// neighbouring lanes alternate between coincident and half-way points; the
// y and z tap counts are uniform along a row.
//
// Restriction (injection): every coarse interior point that coincides with a
// fine interior point takes that fine value.  One thread per (point, grid
// function) over the overlap box computed on the host.
#include "internal.h"

namespace chemora {

namespace {

constexpr double kW[6] = {3.0 / 256, -25.0 / 256, 150.0 / 256, 150.0 / 256, -25.0 / 256,
                          3.0 / 256};

struct ProlongArgs {
  Geo C, F;
  int off[3];
  const double* yc[kMaxTimeLevels];
  double wt[kMaxTimeLevels];
  int ntimes;
  double* yf;
  long long seg_a, seg_b, total;  // ghost counts: z slabs, then + y slabs, then + x slabs
};

__device__ __forceinline__ int floor_half(int q) { return q >> 1; }  // floor(q / 2)

// Fine ghost number p -> fine point (i, j, k).
__device__ __forceinline__ void ghost_point(const ProlongArgs& a, long long p, int& i, int& j,
                                            int& k) {
  const int g = a.F.g, n0 = a.F.n[0], n1 = a.F.n[1], n2 = a.F.n[2];
  const int ex = n0 + 2 * g, ey = n1 + 2 * g;
  if (p < a.seg_a) {
    const long long plane = (long long)ex * ey;
    const int s = (int)(p / plane);
    const int r = (int)(p - s * plane);
    k = s < g ? s - g : n2 + s - g;
    j = r / ex - g;
    i = r % ex - g;
  } else if (p < a.seg_b) {
    p -= a.seg_a;
    const long long slab = 2LL * g * ex;
    k = (int)(p / slab);
    const int r = (int)(p - k * slab);
    const int s = r / ex;
    j = s < g ? s - g : n1 + s - g;
    i = r % ex - g;
  } else {
    p -= a.seg_b;
    const long long plane = 2LL * g * n1;
    k = (int)(p / plane);
    const int r = (int)(p - k * plane);
    j = r / (2 * g);
    const int s = r % (2 * g);
    i = s < g ? s - g : n0 + s - g;
  }
}

__global__ void __launch_bounds__(256) prolong_kernel(ProlongArgs a) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.total) return;
  const int v = blockIdx.y;
  int i, j, k;
  ghost_point(a, p, i, j, k);
  const Geo& C = a.C;

  // x: always six taps, window clamped into the coarse extended range
  const int qx = a.off[0] + i, bx = floor_half(qx);
  int x0;
  double wx[6];
  if (qx & 1) {
    x0 = bx - 2;
    for (int m = 0; m < 6; ++m) wx[m] = kW[m];
  } else {
    x0 = min(max(bx - 2, -C.g), C.n[0] + C.g - 6);
    for (int m = 0; m < 6; ++m) wx[m] = (x0 + m == bx) ? 1.0 : 0.0;
  }
  // y, z: one tap (coincident) or six (half-way)
  const int qy = a.off[1] + j, qz = a.off[2] + k;
  const int ny = (qy & 1) ? 6 : 1, nz = (qz & 1) ? 6 : 1;
  const int y0 = (qy & 1) ? floor_half(qy) - 2 : floor_half(qy);
  const int z0 = (qz & 1) ? floor_half(qz) - 2 : floor_half(qz);

  const long long base = C.off0 + (long long)v * C.sv + x0 + (long long)y0 * C.sy +
                         (long long)z0 * C.sz;
  double val = 0.0;
  for (int l = 0; l < a.ntimes; ++l) {
    const double* src = a.yc[l] + base;
    double acc = 0.0;
    for (int c = 0; c < nz; ++c) {
      const double wz = nz == 1 ? 1.0 : kW[c];
      double plane = 0.0;
      for (int b = 0; b < ny; ++b) {
        const double wy = ny == 1 ? 1.0 : kW[b];
        const double* row = src + (long long)c * C.sz + (long long)b * C.sy;
        double r = 0.0;
#pragma unroll
        for (int m = 0; m < 6; ++m) r += wx[m] * row[m];
        plane += wy * r;
      }
      acc += wz * plane;
    }
    val += a.wt[l] * acc;
  }
  const Geo& F = a.F;
  a.yf[F.off0 + (long long)v * F.sv + i + (long long)j * F.sy + (long long)k * F.sz] = val;
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
  const long long g = F.g, ex = F.n[0] + 2 * g, ey = F.n[1] + 2 * g;
  a.seg_a = 2 * g * ex * ey;
  a.seg_b = a.seg_a + (long long)F.n[2] * 2 * g * ex;
  a.total = a.seg_b + (long long)F.n[2] * F.n[1] * 2 * g;
  const dim3 grid((unsigned)((a.total + 255) / 256), (unsigned)nvar);
  hipLaunchKernelGGL(prolong_kernel, grid, dim3(256), 0, s, a);
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
