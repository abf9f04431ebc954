// internal.h -- shared definitions of libchemora's HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "chemora.h"

namespace chemora {

constexpr int kAlign = 16;  // interior x = 0 starts on a 16-double (128 B) boundary
constexpr int kMaxGhost = 8;
constexpr int kMaxTimeLevels = 3;  // coarse time levels a prolongation may combine
constexpr int kNumXcd = 8;  // MI355X: 8 accelerator complex dies, each with its own L2

// Device view of one block's geometry (element strides, x fastest).
struct Geo {
  int n[3];
  int g;
  int sy, sz;      // strides of y and z within one grid function
  long long sv;    // stride between grid functions
  long long off0;  // element index of interior point (0,0,0) of variable 0
};

// Run-time parameters of the BSSN system and its analytic boundary.
struct BssnPar {
  double h[3];
  double origin[3];
  int slicing;  // 0: 1+log, 1: harmonic
  int shift;    // 0: frozen, 1: Gamma-driver
  double F, eta;
  double gw_A, gw_d;
  int gw_axis;
  int enforce;      // det gt = 1, tr At = 0 after every RK substage
  double ko_sigma;  // Kreiss-Oliger dissipation strength (0: none)
  int fd_order;     // finite-difference order: 4, 6 or 8
};

// The four classical RK4 substages fused with the right-hand side.  Stage 0
// means "right-hand side only".  With k_s the right-hand side of stage s:
//   s1: acc = k1;            out = y0 + dt/2 k1
//   s2: acc = acc + 2 k2;    out = y0 + dt/2 k2
//   s3: acc = acc + 2 k3;    out = y0 + dt k3
//   s4:                      out = y0 + dt/6 (acc + k4)   (out == y0)
struct StageIO {
  const double* yin;  // stencil source (valid ghosts)
  const double* y0;   // y_n (pointwise)
  double* acc;        // accumulator (pointwise)
  double* out;        // stage output, or the rhs for stage 0
  double cdt;         // dt/2, dt/2, dt, dt/6 for stages 1..4
  // Split kernels only: a state-sized buffer whose interior holds the
  // first kernel's per-point intermediates until the second kernel reads
  // them (each point's own values, read before that point is written).
  // nullptr: out serves (it may not when out aliases y0, the last stage).
  double* tmp = nullptr;
};

// Hardware places workgroup b on XCD b % 8.  Give each XCD a contiguous range
// of tiles so that halo re-reads of neighbouring tiles hit the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb / kNumXcd, r = nb % kNumXcd;
  const int x = b % kNumXcd, l = b / kNumXcd;
  return x * q + (x < r ? x : r) + l;
}

// XCD column walk for single-plane tiles.  The xy tile grid is cut into
// cx x cy columns (cx * cy == kNumXcd, cx <= tiles[0], cy <= tiles[1]); the
// workgroups that land on XCD x (b % 8 == x) take column x's tiles plane by
// plane, so that the planes just below and above those in flight are still
// in that XCD's L2 when the next planes need them (z stencils reach 3
// planes each way).  A grid of 8 x (largest column) x tiles[2] blocks;
// blocks past the end of a smaller column get no tile (returns false).
__host__ __device__ __forceinline__ bool column_tile(int b, const int tiles[3], int cx, int cy, int& bx,
                                            int& by, int& bz) {
  const int x = b % kNumXcd, l = b / kNumXcd;
  const int ux = x % cx, uy = x / cx;
  const int xlo = ux * tiles[0] / cx, xhi = (ux + 1) * tiles[0] / cx;
  const int ylo = uy * tiles[1] / cy, yhi = (uy + 1) * tiles[1] / cy;
  const int wx = xhi - xlo, ncol = wx * (yhi - ylo);
  bz = l / ncol;
  if (bz >= tiles[2]) return false;
  const int r = l - bz * ncol;
  bx = xlo + r % wx;
  by = ylo + r / wx;
  return true;
}

// Host: the column split for a tiles[0] x tiles[1] plane of ltx x lty tiles
// (the smallest largest column, then the smallest column perimeter), or
// {0, 0} when the plane has too few tiles for eight columns.
struct ColumnSplit {
  int cx, cy;
  long long blocks_per_plane;  // 8 x the largest column
};
inline ColumnSplit column_split(const int tiles[2], int ltx, int lty) {
  ColumnSplit best{0, 0, 0};
  long long best_max = 0, best_per = 0;
  for (int cx = 1; cx <= kNumXcd; cx *= 2) {
    const int cy = kNumXcd / cx;
    if (cx > tiles[0] || cy > tiles[1]) continue;
    const long long mx = (tiles[0] + cx - 1) / cx, my = (tiles[1] + cy - 1) / cy;
    const long long m = mx * my, per = mx * ltx + my * lty;
    if (best.cx == 0 || m < best_max || (m == best_max && per < best_per)) {
      best = {cx, cy, kNumXcd * m};
      best_max = m;
      best_per = per;
    }
  }
  return best;
}

// Periodic write-through: store v at interior point (i,j,k) of one grid
// function and at every periodic image of it that lies in the ghost zones.
__device__ __forceinline__ void store_with_images(double* f, const Geo& G, int i, int j, int k,
                                                  double v, bool images) {
  f[i + (long long)j * G.sy + (long long)k * G.sz] = v;
  if (!images) return;
  int ii[3], jj[3], kk[3];
  int ci = 1, cj = 1, ck = 1;
  ii[0] = i;
  jj[0] = j;
  kk[0] = k;
  if (i < G.g) ii[ci++] = i + G.n[0];
  if (i >= G.n[0] - G.g) ii[ci++] = i - G.n[0];
  if (j < G.g) jj[cj++] = j + G.n[1];
  if (j >= G.n[1] - G.g) jj[cj++] = j - G.n[1];
  if (k < G.g) kk[ck++] = k + G.n[2];
  if (k >= G.n[2] - G.g) kk[ck++] = k - G.n[2];
  if (ci == 1 && cj == 1 && ck == 1) return;
  for (int c = 0; c < ck; ++c)
    for (int b = 0; b < cj; ++b)
      for (int a = 0; a < ci; ++a)
        if (a | b | c) f[ii[a] + (long long)jj[b] * G.sy + (long long)kk[c] * G.sz] = v;
}

// ---- launchers (host) -----------------------------------------------------
hipError_t launch_fill_periodic(const Geo& G, int nvar, double* state, hipStream_t s);
hipError_t launch_fill_gaugewave(const Geo& G, const BssnPar& P, double t, double* state,
                                 hipStream_t s);
hipError_t launch_wave_stage(const Geo& G, const double h[3], int stage, int precision,
                             bool images, const StageIO& io, hipStream_t s);
hipError_t launch_wave5_stage(const Geo& G, const double h[3], int stage, int precision,
                              bool images, const StageIO& io, hipStream_t s);
long long energy_partial_count(const Geo& G);
hipError_t launch_wave5_energy(const Geo& G, const double h[3], const double* y, double* eps,
                               double* total, double* partial, hipStream_t s);
hipError_t launch_bssn_stage(const Geo& G, const BssnPar& P, int stage, int precision,
                             bool images, const StageIO& io, hipStream_t s);
hipError_t launch_bssn_constraints(const Geo& G, const BssnPar& P, const double* y,
                                   double* hm, double* norms, double* partial,
                                   hipStream_t s);
long long constraints_partial_count(const Geo& G, int order);
hipError_t launch_probe_copy(void* dst, const void* src, long long nbytes, hipStream_t s);
hipError_t launch_prolong(const Geo& C, const double* const* yc, const double* wt, int ntimes,
                          const Geo& F, const int off[3], int nvar, double* yf, hipStream_t s);
hipError_t launch_restrict(const Geo& C, double* yc, const Geo& F, const double* yf,
                           const int off[3], const int lo[3], const int cnt[3], int nvar,
                           hipStream_t s);

}  // namespace chemora
