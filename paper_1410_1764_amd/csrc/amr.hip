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
// The interpolation is separable, so a workgroup takes a box of fine ghost
// points and works through it axis by axis: (1) the coarse points of the
// box's footprint are loaded into LDS once, combined in time (loads
// coalesced along x); (2)-(4) three passes each interpolate one axis from
// coarse to fine points, the first two LDS to LDS, the last straight to
// the fine block.  Every coarse value a box needs is read once per time
// level.  The ghost shell is cut into boxes of about 3000 fine points: the
// two z slabs in SX x SY columns of all g slab planes (axis order z, y, x:
// the thin axis first), the y bands of the interior planes in 32 x g x ZC
// boxes (y, z, x) and the x bands of the interior rows in g x 32 x ZC boxes
// (x, y, z); SX, SY, ZC and the LDS size follow from g on the host (32, 32,
// 32 up to g = 5; 32, 16, 16 above).  grid.y runs over the grid functions.
//
// Restriction (injection): every coarse interior point that coincides with a
// fine interior point takes that fine value.  One thread per (point, grid
// function) over the overlap box computed on the host.
#include <algorithm>

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
  int sbx, sby, zc;        // slab box extent in x and y; planes per band box
  int sx, sy, bx, cy, nzc;  // slab boxes along x, y; y-band boxes along x; x-band boxes
                            // along y; z chunks of the bands
  int blocks_a, blocks_b;  // first box of segments B (y bands) and C (x bands)
  int boxes, nvar;         // boxes per grid function (grid.x), grid functions (grid.y)
  int lds_b;               // offset (doubles) of the second LDS buffer
};

constexpr int kProlongThreads = 512;  // 8 waves per box
constexpr int kBandX = 32;  // y-band box: 32 x g points
constexpr int kBandY = 32;  // x-band box: g x 32 points

__device__ __forceinline__ int floor_half(int q) { return q >> 1; }  // floor(q / 2)

// Coarse window [lo, lo + cnt) that fine points q0 .. q1 (fine units) reach
// along an axis, clamped into the coarse extended range [-g, n + g): the
// host checks that every fine point's own stencil lies inside it, but the
// window of a box whose last point is coincident would reach one further.
__device__ __forceinline__ void footprint(int q0, int q1, int n, int g, int& lo, int& cnt) {
  lo = max(floor_half(q0) - 2, -g);
  cnt = min(floor_half(q1) + 3, n + g - 1) - lo + 1;
}

// value at fine coordinate q from coarse values src[(c - lo) * stride]:
// the coincident value or the 6-point interpolant
__device__ __forceinline__ double interp(const double* src, int stride, int q, int lo) {
  if (q & 1) {
    const double* p = src + (floor_half(q) - 2 - lo) * stride;
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) acc += kW[m] * p[m * stride];
    return acc;
  }
  return src[(floor_half(q) - lo) * stride];
}

// One pass: interpolate axis D of src (extents ext[0..2], x fastest) from its
// coarse window (first coarse index c0[D]) to w[D] fine points starting at
// fine coordinate q0[D]; ext[D] becomes w[D].  Output to LDS dst, or, when
// dst is null, to the fine block at out (strides 1, sy, sz).
template <int D>
__device__ __forceinline__ void pass(const double* src, double* dst, int ext[3], const int w[3],
                                     const int q0[3], const int c0[3], double* out, long long sy,
                                     long long sz) {
  const int ne0 = D == 0 ? w[0] : ext[0], ne1 = D == 1 ? w[1] : ext[1];
  const int ne2 = D == 2 ? w[2] : ext[2];
  const int n01 = ne0 * ne1, total = n01 * ne2;
  const int st1 = ext[0], st2 = ext[0] * ext[1];
  const int std_ = D == 0 ? 1 : (D == 1 ? st1 : st2);
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int z = e / n01, r = e - z * n01, y = r / ne0, x = r - y * ne0;
    const int cd = D == 0 ? x : (D == 1 ? y : z);
    const int base = (D == 0 ? 0 : x) + (D == 1 ? 0 : y) * st1 + (D == 2 ? 0 : z) * st2;
    const double v = interp(src + base, std_, q0[D] + cd, c0[D]);
    if (dst)
      dst[e] = v;
    else
      out[x + y * sy + z * sz] = v;
  }
  ext[D] = w[D];
}

// the three passes of a box in axis order D0, D1, D2: A -> B -> A -> fine block
template <int D0, int D1, int D2>
__device__ __forceinline__ void passes(double* A, double* B, int ext[3], const int w[3],
                                       const int q0[3], const int c0[3], double* out,
                                       long long sy, long long sz) {
  pass<D0>(A, B, ext, w, q0, c0, nullptr, 0, 0);
  __syncthreads();
  pass<D1>(B, A, ext, w, q0, c0, nullptr, 0, 0);
  __syncthreads();
  pass<D2>(A, nullptr, ext, w, q0, c0, out, sy, sz);
}

// One box of fine ghost points: grid function, fine corner, extents, axis
// order of the passes, and its coarse footprint.
struct Box {
  int v, i0, j0, k0;
  int seg;  // 0 z slab (pass order z, y, x), 1 y band (y, z, x), 2 x band (x, y, z)
  int w[3], q0[3], c0[3], ext[3];
  long long cbase;  // element of footprint corner (c0) of grid function v
  int nfoot;
};

__device__ __forceinline__ void box_of(const ProlongArgs& a, int item, Box& x) {
  const Geo &C = a.C, &F = a.F;
  const int g = F.g;
  x.v = item / a.boxes;
  int b = item - x.v * a.boxes;
  if (b < a.blocks_a) {  // z slabs: an SX x SY column of all g slab planes
    const int per = a.sx * a.sy;
    const int s = b / per, r = b - s * per, tx = r % a.sx, ty = r / a.sx;
    x.k0 = s == 0 ? -g : F.n[2];
    x.i0 = -g + tx * a.sbx;
    x.j0 = -g + ty * a.sby;
    x.w[0] = min(a.sbx, F.n[0] + g - x.i0);
    x.w[1] = min(a.sby, F.n[1] + g - x.j0);
    x.w[2] = g;
    x.seg = 0;
  } else if (b < a.blocks_b) {  // y bands of the interior planes
    b -= a.blocks_a;
    const int zc = b / (2 * a.bx), r = b - zc * 2 * a.bx, band = r / a.bx, tx = r % a.bx;
    x.k0 = zc * a.zc;
    x.i0 = -g + tx * kBandX;
    x.j0 = band == 0 ? -g : F.n[1];
    x.w[0] = min(kBandX, F.n[0] + g - x.i0);
    x.w[1] = g;
    x.w[2] = min(a.zc, F.n[2] - x.k0);
    x.seg = 1;
  } else {  // x bands of the interior rows
    b -= a.blocks_b;
    const int zc = b / (2 * a.cy), r = b - zc * 2 * a.cy, band = r / a.cy, ty = r % a.cy;
    x.k0 = zc * a.zc;
    x.i0 = band == 0 ? -g : F.n[0];
    x.j0 = ty * kBandY;
    x.w[0] = g;
    x.w[1] = min(kBandY, F.n[1] - x.j0);
    x.w[2] = min(a.zc, F.n[2] - x.k0);
    x.seg = 2;
  }
  x.q0[0] = a.off[0] + x.i0;
  x.q0[1] = a.off[1] + x.j0;
  x.q0[2] = a.off[2] + x.k0;
  for (int d = 0; d < 3; ++d)
    footprint(x.q0[d], x.q0[d] + x.w[d] - 1, C.n[d], C.g, x.c0[d], x.ext[d]);
  x.cbase = C.off0 + (long long)x.v * C.sv + x.c0[0] + (long long)x.c0[1] * C.sy +
            (long long)x.c0[2] * C.sz;
  x.nfoot = x.ext[0] * x.ext[1] * x.ext[2];
}

// kU footprint elements per thread and round, all their loads issued before
// the first is used (one memory latency per round, not per element)
constexpr int kU = 8;

__device__ __forceinline__ long long foot_offset(const ProlongArgs& a, const Box& x, int e) {
  const int nxy = x.ext[0] * x.ext[1];
  const int cz = e / nxy, r = e - cz * nxy, cy = r / x.ext[0], cx = r - cy * x.ext[0];
  return x.cbase + cx + (long long)cy * a.C.sy + (long long)cz * a.C.sz;
}

// loads of footprint elements e0 + u * blockDim.x, u < kU, into ld
__device__ __forceinline__ void foot_issue(const ProlongArgs& a, const Box& x, int e0,
                                           double (&ld)[kU][kMaxTimeLevels]) {
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int e = e0 + u * (int)blockDim.x;
    if (e < x.nfoot) {
      const long long o = foot_offset(a, x, e);
#pragma unroll
      for (int l = 0; l < kMaxTimeLevels; ++l)
        if (l < a.ntimes) ld[u][l] = a.yc[l][o];
    }
  }
}

// those elements, combined in time, into A
__device__ __forceinline__ void foot_store(const ProlongArgs& a, const Box& x, int e0,
                                           const double (&ld)[kU][kMaxTimeLevels], double* A) {
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int e = e0 + u * (int)blockDim.x;
    if (e < x.nfoot) {
      double val = 0.0;
#pragma unroll
      for (int l = 0; l < kMaxTimeLevels; ++l)
        if (l < a.ntimes) val += a.wt[l] * ld[u][l];
      A[e] = val;
    }
  }
}

// One workgroup per (box, grid function).  Workgroup b runs on XCD b % 8;
// xcd_tile gives each XCD a contiguous range of boxes, so that neighbouring
// boxes' shared footprint lines meet in one L2.
__global__ void __launch_bounds__(kProlongThreads) prolong_kernel(ProlongArgs a) {
  extern __shared__ double lds[];
  double* A = lds;
  double* B = lds + a.lds_b;
  const Geo& F = a.F;
  Box x;
  box_of(a, (int)blockIdx.y * a.boxes + xcd_tile((int)blockIdx.x, (int)gridDim.x), x);
  // (1) the footprint, combined in time
  const int step = kU * (int)blockDim.x;
  for (int e0 = (int)threadIdx.x; e0 < x.nfoot; e0 += step) {
    double ld[kU][kMaxTimeLevels];
    foot_issue(a, x, e0, ld);
    foot_store(a, x, e0, ld, A);
  }
  __syncthreads();
  // (2)-(4) one axis per pass: A -> B -> A -> fine block
  double* out = a.yf + F.off0 + (long long)x.v * F.sv + x.i0 + (long long)x.j0 * F.sy +
                (long long)x.k0 * F.sz;
  if (x.seg == 0)
    passes<2, 1, 0>(A, B, x.ext, x.w, x.q0, x.c0, out, F.sy, F.sz);
  else if (x.seg == 1)
    passes<1, 2, 0>(A, B, x.ext, x.w, x.q0, x.c0, out, F.sy, F.sz);
  else
    passes<0, 1, 2>(A, B, x.ext, x.w, x.q0, x.c0, out, F.sy, F.sz);
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

// LDS doubles of a box with the given fine extents and axis order: the
// footprint or the second pass's output (buffer A), the first pass's output
// (buffer B); footprints bounded by w / 2 + 7 coarse points per axis
static void box_lds(const int w[3], const int ord[3], int& na, int& nb) {
  int e[3] = {w[0] / 2 + 7, w[1] / 2 + 7, w[2] / 2 + 7};
  const int foot = e[0] * e[1] * e[2];
  e[ord[0]] = w[ord[0]];
  const int p1 = e[0] * e[1] * e[2];
  e[ord[1]] = w[ord[1]];
  const int p2 = e[0] * e[1] * e[2];
  na = std::max(na, std::max(foot, p2));
  nb = std::max(nb, p1);
}

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
  // box shapes: the largest of these whose LDS fits in 64 KiB
  const int shapes[3][3] = {{32, 32, 32}, {32, 16, 16}, {32, 8, 16}};
  int na = 0, nb = 0;
  for (const auto& sh : shapes) {
    na = nb = 0;
    const int ws[3] = {sh[0], sh[1], g}, os[3] = {2, 1, 0};
    const int wb[3] = {kBandX, g, sh[2]}, ob[3] = {1, 2, 0};
    const int wc[3] = {g, kBandY, sh[2]}, oc[3] = {0, 1, 2};
    box_lds(ws, os, na, nb);
    box_lds(wb, ob, na, nb);
    box_lds(wc, oc, na, nb);
    a.sbx = sh[0];
    a.sby = sh[1];
    a.zc = sh[2];
    if (8LL * (na + nb) <= 65536) break;
  }
  if (8LL * (na + nb) > 65536) return hipErrorInvalidValue;
  a.lds_b = na;
  a.sx = (ex + a.sbx - 1) / a.sbx;
  a.sy = (ey + a.sby - 1) / a.sby;
  a.bx = (ex + kBandX - 1) / kBandX;
  a.cy = (F.n[1] + kBandY - 1) / kBandY;
  a.nzc = (F.n[2] + a.zc - 1) / a.zc;
  const long long sa = 2LL * a.sx * a.sy;
  const long long sb = 2LL * a.bx * a.nzc;
  const long long sc = 2LL * a.cy * a.nzc;
  if ((sa + sb + sc) * nvar > 0x7fffffffLL || nvar > 65535) return hipErrorInvalidValue;
  a.blocks_a = (int)sa;
  a.blocks_b = (int)(sa + sb);
  a.boxes = (int)(sa + sb + sc);
  a.nvar = nvar;
  const dim3 grid((unsigned)a.boxes, (unsigned)nvar);
  hipLaunchKernelGGL(prolong_kernel, grid, dim3(kProlongThreads), (size_t)8 * (na + nb), s, a);
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
