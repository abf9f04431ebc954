// prolong_box.h -- prolongation of a fine block's ghost zones from the next
// coarser level (ratio 2) by boxes, shared by the standalone prolongation
// (amr.hip) and the batch's prolongation ghost items (batch_stage.h).
//
// Geometry is integer: with h_c = 2 h_f on every axis and the fine origin
// `off` fine spacings from the coarse origin (checked on the host), fine
// point i sits at fine-unit coordinate q = off + i from the coarse origin;
// q even coincides with coarse point q/2, q odd lies half-way between
// coarse points (q-1)/2 and (q+1)/2.  Per axis a fine value is the coarse
// value (coincident) or the degree-5 Lagrange interpolant through the six
// coarse points at offsets -2 .. 3 from the lower neighbour (half-way),
// weights (3, -25, 150, 150, -25, 3) / 256; the tensor product over the
// axes; up to three coarse time levels combined with Lagrange weights in
// time.
//
// A workgroup takes a box of fine ghost points and works through it axis by
// axis: (1) the coarse points of the box's footprint are loaded into LDS
// buffer A once, combined in time; (2)-(4) three passes each interpolate one
// axis from coarse to fine points, A -> B -> A -> the fine block.  The ghost
// shell is cut into boxes: the two z slabs in SX x SY columns of all g slab
// planes (pass order z, y, x: the thin axis first), the y bands of the
// interior planes in BX x g x ZC boxes (y, z, x) and the x bands of the
// interior rows in g x BY x ZC boxes (x, y, z).
#pragma once

#include <algorithm>

#include "internal.h"

namespace chemora {

// how a fine block's ghost shell is cut into boxes
struct BoxGrid {
  int sbx, sby, bandx, bandy, zc;  // slab column, y-band box x, x-band box y, band planes
  int sx, sy, bx, cy, nzc;         // boxes: slab columns along x, y; y-band boxes along x;
                                   // x-band boxes along y; z chunks of the bands
  int blocks_a, blocks_b, boxes;   // first box of the y bands, of the x bands; total
  int lds_a, lds_b;                // LDS doubles of buffers A and B
};

// Host: LDS doubles of a box with fine extents w and pass order ord: the
// footprint or the second pass's output (A), the first pass's output (B);
// footprints bounded by w / 2 + 7 coarse points per axis.
inline void box_lds(const int w[3], const int ord[3], int& na, int& nb) {
  int e[3] = {w[0] / 2 + 7, w[1] / 2 + 7, w[2] / 2 + 7};
  const int foot = e[0] * e[1] * e[2];
  e[ord[0]] = w[ord[0]];
  const int p1 = e[0] * e[1] * e[2];
  e[ord[1]] = w[ord[1]];
  const int p2 = e[0] * e[1] * e[2];
  na = std::max(na, std::max(foot, p2));
  nb = std::max(nb, p1);
}

// Host: the boxes of fine block F (interior n, ghost g) with slab columns
// sbx x sby, band boxes bandx / bandy wide and zc planes deep.
inline BoxGrid make_box_grid(const Geo& F, int sbx, int sby, int bandx, int bandy, int zc) {
  BoxGrid b{};
  const int g = F.g, ex = F.n[0] + 2 * g, ey = F.n[1] + 2 * g;
  b.sbx = sbx;
  b.sby = sby;
  b.bandx = bandx;
  b.bandy = bandy;
  b.zc = zc;
  b.sx = (ex + sbx - 1) / sbx;
  b.sy = (ey + sby - 1) / sby;
  b.bx = (ex + bandx - 1) / bandx;
  b.cy = (F.n[1] + bandy - 1) / bandy;
  b.nzc = (F.n[2] + zc - 1) / zc;
  const long long sa = 2LL * b.sx * b.sy, sb = 2LL * b.bx * b.nzc, sc = 2LL * b.cy * b.nzc;
  const long long tot = sa + sb + sc;
  b.blocks_a = (int)sa;
  b.blocks_b = (int)(sa + sb);
  b.boxes = tot > 0x7fffffffLL ? -1 : (int)tot;
  int na = 0, nb = 0;
  const int ws[3] = {sbx, sby, g}, os[3] = {2, 1, 0};
  const int wb[3] = {bandx, g, zc}, ob[3] = {1, 2, 0};
  const int wc[3] = {g, bandy, zc}, oc[3] = {0, 1, 2};
  box_lds(ws, os, na, nb);
  box_lds(wb, ob, na, nb);
  box_lds(wc, oc, na, nb);
  b.lds_a = na;
  b.lds_b = nb;
  return b;
}

constexpr double kProlongW[6] = {3.0 / 256, -25.0 / 256, 150.0 / 256, 150.0 / 256,
                                 -25.0 / 256, 3.0 / 256};

__device__ __forceinline__ int floor_half(int q) { return q >> 1; }  // floor(q / 2)

// Coarse window [lo, lo + cnt) that fine points q0 .. q1 (fine units) reach
// along an axis, clamped into the coarse extended range [-g, n + g): the
// host checks that every fine point's own stencil lies inside it, but the
// window of a box whose last point is coincident would reach one further.
__device__ __forceinline__ void footprint(int q0, int q1, int n, int g, int& lo, int& cnt) {
  lo = max(floor_half(q0) - 2, -g);
  cnt = min(floor_half(q1) + 3, n + g - 1) - lo + 1;
}

// Coordinates (x, y, z) of element e of a box with extents n0 x n1 x ...
// (x fastest) that a thread visits at e = threadIdx.x, then every
// blockDim.x elements.  The stride's own coordinates are computed once (the
// same for the whole workgroup); each step then adds them with one carry per
// axis instead of dividing e by the extents.
struct Walk {
  int x, y, z;     // coordinates of the current element
  int dx, dy, dz;  // coordinates of the stride blockDim.x
  int n0, n1;
  __device__ __forceinline__ Walk(int e0, int n0_, int n1_) : n0(n0_), n1(n1_) {
    const int s = (int)blockDim.x, r = e0 / n0, sr = s / n0;
    x = e0 - r * n0;
    y = r % n1;
    z = r / n1;
    dx = s - sr * n0;
    dy = sr % n1;
    dz = sr / n1;
  }
  // x + dx < 2 n0 and y + dy + 1 < 2 n1: one subtraction per axis suffices
  __device__ __forceinline__ void step() {
    x += dx;
    const int cx = x >= n0;
    x -= cx ? n0 : 0;
    y += dy + cx;
    const int cy = y >= n1;
    y -= cy ? n1 : 0;
    z += dz + cy;
  }
};

// One pass: interpolate axis D of src (extents ext[0..2], x fastest) from its
// coarse window (first coarse index c0[D]) to w[D] fine points starting at
// fine coordinate q0[D]; ext[D] becomes w[D].  Output to the LDS buffer dst
// (LDS = true), or to the fine block at out (strides 1, sy, sz).  A thread
// takes two neighbouring fine points along D at a time: one coincident (one
// coarse value) and one half-way (six), so that no lane of a wave waits on
// the other kind's path; a box with odd w[D] ends in a single point.  The
// half-way value sums the six weighted coarse values in order.
template <int D, bool LDS>
__device__ __forceinline__ void pass(const double* src, double* dst, int ext[3], const int w[3],
                                     const int q0[3], const int c0[3], double* out, long long sy,
                                     long long sz) {
  const int ne0 = D == 0 ? w[0] : ext[0], ne1 = D == 1 ? w[1] : ext[1];
  const int ne2 = D == 2 ? w[2] : ext[2];
  // pairs along D
  const int np0 = D == 0 ? (ne0 + 1) / 2 : ne0, np1 = D == 1 ? (ne1 + 1) / 2 : ne1;
  const int np2 = D == 2 ? (ne2 + 1) / 2 : ne2;
  const int total = np0 * np1 * np2;
  const int st1 = ext[0], st2 = ext[0] * ext[1];  // source strides
  const int sd = D == 0 ? 1 : (D == 1 ? st1 : st2);
  const int o1 = ne0, o2 = ne0 * ne1;             // LDS output strides
  const int od = D == 0 ? 1 : (D == 1 ? o1 : o2);
  const long long gd = D == 0 ? 1 : (D == 1 ? sy : sz);
  Walk p((int)threadIdx.x, np0, np1);
  for (int e = threadIdx.x; e < total; e += blockDim.x, p.step()) {
    const int i = 2 * (D == 0 ? p.x : (D == 1 ? p.y : p.z));  // first fine index along D
    const int x = D == 0 ? i : p.x, y = D == 1 ? i : p.y, z = D == 2 ? i : p.z;
    const double* s0 = src + (D == 0 ? 0 : x) + (D == 1 ? 0 : y) * st1 + (D == 2 ? 0 : z) * st2;
    const int q = q0[D] + i;
    const bool two = i + 1 < w[D];
    const int qe = q + (q & 1), qo = q + 1 - (q & 1);  // the coincident and half-way point
    // the coincident point lies inside the footprint even when it is past
    // the box's last (half-way) point; the half-way point's six do not
    const double ve = s0[(floor_half(qe) - c0[D]) * sd];
    double vo = 0.0;
    if ((q & 1) || two) {
      const double* s6 = s0 + (floor_half(qo) - 2 - c0[D]) * sd;
#pragma unroll
      for (int m = 0; m < 6; ++m) vo += kProlongW[m] * s6[m * sd];
    }
    const double v0 = (q & 1) ? vo : ve, v1 = (q & 1) ? ve : vo;
    if constexpr (LDS) {
      const int o = x + y * o1 + z * o2;
      dst[o] = v0;
      if (two) dst[o + od] = v1;
    } else {
      double* g = out + x + y * sy + z * sz;
      g[0] = v0;
      if (two) g[gd] = v1;
    }
  }
  ext[D] = w[D];
}

// the three passes of a box in axis order D0, D1, D2: A -> B -> A -> fine block
template <int D0, int D1, int D2>
__device__ __forceinline__ void passes(double* A, double* B, int ext[3], const int w[3],
                                       const int q0[3], const int c0[3], double* out,
                                       long long sy, long long sz) {
  pass<D0, true>(A, B, ext, w, q0, c0, nullptr, 0, 0);
  __syncthreads();
  pass<D1, true>(B, A, ext, w, q0, c0, nullptr, 0, 0);
  __syncthreads();
  pass<D2, false>(A, nullptr, ext, w, q0, c0, out, sy, sz);
}

// One box of fine ghost points: fine corner, extents, the segment it belongs
// to (its pass order), and its coarse footprint.
struct Box {
  int i0, j0, k0;
  int seg;  // 0 z slab (pass order z, y, x), 1 y band (y, z, x), 2 x band (x, y, z)
  int w[3], q0[3], c0[3], ext[3];
  int nfoot;
};

// box b (0 <= b < bg.boxes) of fine block F, coarse block C, offset off
__device__ __forceinline__ void box_geometry(const BoxGrid& bg, const Geo& C, const Geo& F,
                                             const int off[3], int b, Box& x) {
  const int g = F.g;
  if (b < bg.blocks_a) {  // z slabs: an SX x SY column of all g slab planes
    const int per = bg.sx * bg.sy;
    const int s = b / per, r = b - s * per, tx = r % bg.sx, ty = r / bg.sx;
    x.k0 = s == 0 ? -g : F.n[2];
    x.i0 = -g + tx * bg.sbx;
    x.j0 = -g + ty * bg.sby;
    x.w[0] = min(bg.sbx, F.n[0] + g - x.i0);
    x.w[1] = min(bg.sby, F.n[1] + g - x.j0);
    x.w[2] = g;
    x.seg = 0;
  } else if (b < bg.blocks_b) {  // y bands of the interior planes
    b -= bg.blocks_a;
    const int zc = b / (2 * bg.bx), r = b - zc * 2 * bg.bx, band = r / bg.bx, tx = r % bg.bx;
    x.k0 = zc * bg.zc;
    x.i0 = -g + tx * bg.bandx;
    x.j0 = band == 0 ? -g : F.n[1];
    x.w[0] = min(bg.bandx, F.n[0] + g - x.i0);
    x.w[1] = g;
    x.w[2] = min(bg.zc, F.n[2] - x.k0);
    x.seg = 1;
  } else {  // x bands of the interior rows
    b -= bg.blocks_b;
    const int zc = b / (2 * bg.cy), r = b - zc * 2 * bg.cy, band = r / bg.cy, ty = r % bg.cy;
    x.k0 = zc * bg.zc;
    x.i0 = band == 0 ? -g : F.n[0];
    x.j0 = ty * bg.bandy;
    x.w[0] = g;
    x.w[1] = min(bg.bandy, F.n[1] - x.j0);
    x.w[2] = min(bg.zc, F.n[2] - x.k0);
    x.seg = 2;
  }
  x.q0[0] = off[0] + x.i0;
  x.q0[1] = off[1] + x.j0;
  x.q0[2] = off[2] + x.k0;
  for (int d = 0; d < 3; ++d)
    footprint(x.q0[d], x.q0[d] + x.w[d] - 1, C.n[d], C.g, x.c0[d], x.ext[d]);
  x.nfoot = x.ext[0] * x.ext[1] * x.ext[2];
}

// kU footprint elements per thread and round, all their loads issued before
// the first is used (one memory latency per round, not per element)
constexpr int kProlongU = 8;

// Footprint of box x of one grid function into A, combined in time: lev[l]
// points at that grid function's coarse element (0,0,0) of time level l.
__device__ __forceinline__ void box_footprint(const Box& x, const Geo& C,
                                              const double* const* lev, const double* wt,
                                              int ntimes, double* A) {
  const long long corner = C.off0 + x.c0[0] + (long long)x.c0[1] * C.sy +
                           (long long)x.c0[2] * C.sz;
  const int step = kProlongU * (int)blockDim.x;
  Walk p((int)threadIdx.x, x.ext[0], x.ext[1]);
  for (int e0 = (int)threadIdx.x; e0 < x.nfoot; e0 += step) {
    double ld[kProlongU][kMaxTimeLevels];
#pragma unroll
    for (int u = 0; u < kProlongU; ++u) {
      const int e = e0 + u * (int)blockDim.x;
      if (e < x.nfoot) {
        const long long o = corner + p.x + (long long)p.y * C.sy + (long long)p.z * C.sz;
#pragma unroll
        for (int l = 0; l < kMaxTimeLevels; ++l)
          if (l < ntimes) ld[u][l] = lev[l][o];
      }
      p.step();
    }
#pragma unroll
    for (int u = 0; u < kProlongU; ++u) {
      const int e = e0 + u * (int)blockDim.x;
      if (e < x.nfoot) {
        double val = 0.0;
#pragma unroll
        for (int l = 0; l < kMaxTimeLevels; ++l)
          if (l < ntimes) val += wt[l] * ld[u][l];
        A[e] = val;
      }
    }
  }
}

// One grid function of box x: footprint into A, three passes, stored into
// the fine grid function whose element (0,0,0) is yf0 (strides F.sy, F.sz).
// Ends with the last pass's stores (no barrier after it).
__device__ __forceinline__ void prolong_box(const Box& x, const Geo& C, const Geo& F,
                                            const double* const* lev, const double* wt,
                                            int ntimes, double* yf0, double* A, double* B) {
  box_footprint(x, C, lev, wt, ntimes, A);
  __syncthreads();
  double* out = yf0 + x.i0 + (long long)x.j0 * F.sy + (long long)x.k0 * F.sz;
  int ext[3] = {x.ext[0], x.ext[1], x.ext[2]};
  if (x.seg == 0)
    passes<2, 1, 0>(A, B, ext, x.w, x.q0, x.c0, out, F.sy, F.sz);
  else if (x.seg == 1)
    passes<1, 2, 0>(A, B, ext, x.w, x.q0, x.c0, out, F.sy, F.sz);
  else
    passes<0, 1, 2>(A, B, ext, x.w, x.q0, x.c0, out, F.sy, F.sz);
}

// Lagrange weights in time at t of ntimes (<= kMaxTimeLevels) levels at
// times T; entries from ntimes on are left alone
__host__ __device__ __forceinline__ void time_weights(const double* T, int ntimes, double t,
                                                      double* wt) {
#pragma unroll
  for (int l = 0; l < kMaxTimeLevels; ++l) {
    if (l >= ntimes) continue;
    double w = 1.0;
#pragma unroll
    for (int m = 0; m < kMaxTimeLevels; ++m)
      if (m < ntimes && m != l) w *= (t - T[m]) / (T[l] - T[m]);
    wt[l] = w;
  }
}

}  // namespace chemora
