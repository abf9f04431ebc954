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
// the host computes.
//
// The interpolation is separable, so a workgroup takes a tile of fine
// ghost points in one fine z-plane and works through it axis by axis in
// LDS: (1) each coarse (x, y) point of the tile's footprint is interpolated
// in z and combined in time (loads coalesced along x, each coarse value read
// once per tile and level); (2) those are interpolated in y to the tile's
// fine rows; (3) in x to its fine points, which are stored.  A point costs
// about 20 coarse loads instead of the 6 x 6 x 6 per level of a direct
// evaluation.  The ghost shell is cut into tiles as the two z slabs (64 x 4
// tiles over whole planes), the two y bands of the interior planes (32 x g)
// and the two x bands of the interior rows (g x 32); grid.y runs over the
// grid functions.
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
  int nta, ntb, ntc;  // tiles per slab plane (A), per band row (B), per band column (C)
  int blocks_a, blocks_b;  // first block of segments B and C
};

constexpr int kTA_X = 64, kTA_Y = 4;  // z-slab tiles
constexpr int kTB_X = 32;             // y-band tiles: 32 x g
constexpr int kTC_Y = 32;             // x-band tiles: g x 32
constexpr int kFootX = kTA_X / 2 + 7;                      // coarse footprint bounds
constexpr int kFootY = (kTC_Y > 2 * kMaxGhost ? kTC_Y : 2 * kMaxGhost) / 2 + 7;
constexpr int kRowsMax = kTC_Y > kMaxGhost ? kTC_Y : kMaxGhost;

__device__ __forceinline__ int floor_half(int q) { return q >> 1; }  // floor(q / 2)

// Coarse window [lo, hi] that fine points q0 .. q1 (fine units) reach along
// an axis, clamped into the coarse extended range [-g, n + g).
__device__ __forceinline__ void footprint(int q0, int q1, int n, int g, int& lo, int& cnt) {
  lo = max(floor_half(q0) - 2, -g);
  const int hi = min(floor_half(q1) + 3, n + g - 1);
  cnt = hi - lo + 1;
}

__global__ void __launch_bounds__(256) prolong_kernel(ProlongArgs a) {
  __shared__ double sz_[kFootY * kFootX];   // z- and time-interpolated coarse footprint
  __shared__ double sy_[kRowsMax * kFootX];  // then y-interpolated to the fine rows
  const Geo &C = a.C, &F = a.F;
  const int g = F.g, ex = F.n[0] + 2 * g;
  const int v = blockIdx.y;
  int b = blockIdx.x, i0, j0, k, wx, wy;
  if (b < a.blocks_a) {  // z slabs: whole extended planes
    const int per = a.nta * ((F.n[1] + 2 * g + kTA_Y - 1) / kTA_Y);
    const int s = b / per, r = b - s * per;
    k = s < g ? s - g : F.n[2] + s - g;
    const int tx = r % a.nta, ty = r / a.nta;
    i0 = -g + tx * kTA_X;
    j0 = -g + ty * kTA_Y;
    wx = min(kTA_X, ex - tx * kTA_X);
    wy = min(kTA_Y, F.n[1] + 2 * g - ty * kTA_Y);
  } else if (b < a.blocks_b) {  // y bands of the interior planes
    b -= a.blocks_a;
    const int per = 2 * a.ntb;
    k = b / per;
    const int r = b - k * per, band = r / a.ntb, tx = r % a.ntb;
    i0 = -g + tx * kTB_X;
    j0 = band == 0 ? -g : F.n[1];
    wx = min(kTB_X, ex - tx * kTB_X);
    wy = g;
  } else {  // x bands of the interior rows
    b -= a.blocks_b;
    const int per = 2 * a.ntc;
    k = b / per;
    const int r = b - k * per, band = r / a.ntc, ty = r % a.ntc;
    i0 = band == 0 ? -g : F.n[0];
    j0 = ty * kTC_Y;
    wx = g;
    wy = min(kTC_Y, F.n[1] - ty * kTC_Y);
  }
  const int qx0 = a.off[0] + i0, qy0 = a.off[1] + j0, qz = a.off[2] + k;
  int cx0, fx, cy0, fy;
  footprint(qx0, qx0 + wx - 1, C.n[0], C.g, cx0, fx);
  footprint(qy0, qy0 + wy - 1, C.n[1], C.g, cy0, fy);
  const bool zhalf = qz & 1;
  const int nz = zhalf ? 6 : 1;
  const int z0 = zhalf ? floor_half(qz) - 2 : floor_half(qz);

  // (1) z and time
  const long long cbase = C.off0 + (long long)v * C.sv + (long long)z0 * C.sz;
  for (int e = threadIdx.x; e < fx * fy; e += blockDim.x) {
    const int cy = e / fx, cx = e - cy * fx;
    const long long o = cbase + (cx0 + cx) + (long long)(cy0 + cy) * C.sy;
    double val = 0.0;
    for (int l = 0; l < a.ntimes; ++l) {
      const double* src = a.yc[l] + o;
      double acc;
      if (zhalf) {
        acc = 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) acc += kW[c] * src[(long long)c * C.sz];
      } else {
        acc = src[0];
      }
      val += a.wt[l] * acc;
    }
    sz_[cy * kFootX + cx] = val;
  }
  __syncthreads();
  // (2) y, to the tile's fine rows
  for (int e = threadIdx.x; e < fx * wy; e += blockDim.x) {
    const int j = e / fx, cx = e - j * fx;
    const int qy = qy0 + j;
    double val;
    if (qy & 1) {
      const int r0 = floor_half(qy) - 2 - cy0;
      val = 0.0;
#pragma unroll
      for (int m = 0; m < 6; ++m) val += kW[m] * sz_[(r0 + m) * kFootX + cx];
    } else {
      val = sz_[(floor_half(qy) - cy0) * kFootX + cx];
    }
    sy_[j * kFootX + cx] = val;
  }
  __syncthreads();
  // (3) x, to the fine points
  for (int e = threadIdx.x; e < wx * wy; e += blockDim.x) {
    const int j = e / wx, i = e - j * wx;
    const int qx = qx0 + i;
    const double* row = sy_ + j * kFootX;
    double val;
    if (qx & 1) {
      const int c0 = floor_half(qx) - 2 - cx0;
      val = 0.0;
#pragma unroll
      for (int m = 0; m < 6; ++m) val += kW[m] * row[c0 + m];
    } else {
      val = row[floor_half(qx) - cx0];
    }
    a.yf[F.off0 + (long long)v * F.sv + (i0 + i) + (long long)(j0 + j) * F.sy +
         (long long)k * F.sz] = val;
  }
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
  const int g = F.g, ex = F.n[0] + 2 * g, ey = F.n[1] + 2 * g;
  a.nta = (ex + kTA_X - 1) / kTA_X;
  a.ntb = (ex + kTB_X - 1) / kTB_X;
  a.ntc = (F.n[1] + kTC_Y - 1) / kTC_Y;
  const long long na = 2LL * g * a.nta * ((ey + kTA_Y - 1) / kTA_Y);
  const long long nb = (long long)F.n[2] * 2 * a.ntb;
  const long long nc = (long long)F.n[2] * 2 * a.ntc;
  if (na + nb + nc > 0x7fffffffLL) return hipErrorInvalidValue;
  a.blocks_a = (int)na;
  a.blocks_b = (int)(na + nb);
  const dim3 grid((unsigned)(na + nb + nc), (unsigned)nvar);
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
