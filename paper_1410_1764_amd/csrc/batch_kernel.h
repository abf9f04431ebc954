// batch_kernel.h -- data structures and device helpers of the batched patch
// path (batch.hip), shared by its host code and by the translation units
// that instantiate the stage kernel (batch_stage.h, one unit per
// kernel kind, so that they compile in parallel).
#pragma once

#include "bssn_lds.h"
#include "prolong_box.h"

namespace chemora {

constexpr int kThreads = 256;
// staging buffers of the LDS-staged kinds (three: two workgroups per CU fit)
constexpr int kBatchBufs = 3;
constexpr int kGhostChunk = 1024;  // ghost points per ghost item
constexpr int kMaxPatches = 4096;

struct PatchDesc {
  Geo G;
  BssnPar P;
  Weights W;
  long long state_off;  // byte offset of the patch's state from Batch::base
  long long ws_off;     // same for its workspace: B1 | B2 | acc, each E doubles
  long long E;        // elements of one state
  long long ghosts;   // ghost points of one grid function
  int ltx, lty, tz;   // tile: ltx * lty threads, tz planes each
  int tiles[3];
  int cols[2];        // column split of the xy tile grid (work-list order), 1 x 1: none
  // Ghosts prolongated from a coarse parent (parent != 0) instead of the
  // analytic gauge wave: the parent's geometry, the fine offset, the boxes
  // of the ghost shell (one ghost item each, all grid functions), the byte
  // offsets of the parent's time levels from Batch::base and their times.
  int parent;
  int poff[3];
  int pntimes;
  Geo PC;
  BoxGrid pb;
  long long plev[kMaxTimeLevels];
  double ptimes[kMaxTimeLevels];
};

// Prolongation ghost boxes of the batch: 16 x 16 slab columns, 16-point band
// boxes 16 planes deep; both LDS buffers within kBatchProlongLds doubles for
// ghost widths up to 5 (checked on the host per patch).
constexpr int kBatchProlongBox = 16;
constexpr int kBatchProlongLds = 2048;

// Device plan buffer: patch descriptors, prefix sums of interior and ghost
// items per patch (in work-list order), the clock.
struct MetaLayout {
  static long long desc_off() { return 0; }
  static long long prefix_off(int np) { return ((long long)sizeof(PatchDesc) * np + 255) / 256 * 256; }
  static long long gprefix_off(int np) { return prefix_off(np) + 8LL * (np + 1); }
  static long long clock_off(int np) { return gprefix_off(np) + 8LL * (np + 1); }
  static long long bytes(int np) { return (clock_off(np) + 8 + 255) / 256 * 256; }
};

struct Batch {
  // Every patch pointer is base + a byte offset: derived from a kernel
  // argument, the compiler knows it is global memory and uses global loads
  // and stores (a pointer read from the descriptor would be generic, and
  // its accesses FLAT instructions, which also count in the LDS wait counter
  // and stall the LDS-staged kernels).
  char* base;
  const PatchDesc* pd;
  const long long* prefix;   // interior items before patch q (work-list order)
  const long long* gprefix;  // ghost items before patch q
  double* clock;
  int np;
  long long n_interior, n_total;
  double dt;
  double t_out;   // stage-output time offset in units of dt (0.5, 0.5, 1, 1)
  int stage_io;   // 1..4, or 0 (right-hand side only, into B1)
};

// Tile of a patch's l-th interior item.  A patch's items are listed column
// by column (cols[0] x cols[1] columns of the xy tile grid), each column
// plane by plane: cut into eight contiguous shares, one per XCD, the list
// makes every XCD walk columns along z (as column_tile does for one block),
// so the planes above and below the ones in flight stay in its L2.
__host__ __device__ __forceinline__ void patch_tile(const PatchDesc& p, long long l, int& bx, int& by,
                                           int& bz) {
  const int cx = p.cols[0], cy = p.cols[1];
  long long base = 0;
  for (int c = 0; c < cx * cy; ++c) {
    const int ux = c % cx, uy = c / cx;
    const int xlo = ux * p.tiles[0] / cx, xhi = (ux + 1) * p.tiles[0] / cx;
    const int ylo = uy * p.tiles[1] / cy, yhi = (uy + 1) * p.tiles[1] / cy;
    const int wx = xhi - xlo;
    const long long per = (long long)wx * (yhi - ylo), n = per * p.tiles[2];
    if (l < base + n || c == cx * cy - 1) {
      const long long r = l - base;
      bz = (int)(r / per);
      const int t = (int)(r - bz * per);
      bx = xlo + t % wx;
      by = ylo + t / wx;
      return;
    }
    base += n;
  }
}

__device__ __forceinline__ int find_patch(const long long* prefix, int np, long long item) {
  int lo = 0, hi = np - 1;  // last q with prefix[q] <= item
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ghost point t of a patch (same enumeration as the single-grid fill)
__device__ __forceinline__ void ghost_ijk(const Geo& G, long long t, int ijk[3]) {
  const int g = G.g, e0 = G.n[0] + 2 * g, e1 = G.n[1] + 2 * g;
  const long long cz = 2LL * g * e1 * e0;
  const long long cy = (long long)G.n[2] * 2 * g * e0;
  if (t < cz) {
    ijk[0] = (int)(t % e0) - g;
    const long long r = t / e0;
    ijk[1] = (int)(r % e1) - g;
    const int p = (int)(r / e1);
    ijk[2] = p < g ? p - g : G.n[2] + (p - g);
  } else if (t < cz + cy) {
    t -= cz;
    ijk[0] = (int)(t % e0) - g;
    const long long r = t / e0;
    const int p = (int)(r % (2 * g));
    ijk[1] = p < g ? p - g : G.n[1] + (p - g);
    ijk[2] = (int)(r / (2 * g));
  } else {
    t -= cz + cy;
    const int p = (int)(t % (2 * g));
    ijk[0] = p < g ? p - g : G.n[0] + (p - g);
    const long long r = t / (2 * g);
    ijk[1] = (int)(r % G.n[1]);
    ijk[2] = (int)(r / G.n[1]);
  }
}

// gauge wave (zero shift; exact under harmonic slicing): chi = H^-1/3,
// gt_aa = H^2/3, gt_bb = H^-1/3, K = -(pi A/d) cos H^-3/2,
// At_aa = -(2 pi A/3d) cos H^-5/6, At_bb = (pi A/3d) cos H^-11/6,
// Gamt^a = -(4 pi A/3d) cos H^-5/3, alpha = sqrt(H)
__device__ __forceinline__ void gw_store(const BssnPar& P, double xa, double t, double* f,
                                         long long sv) {
  const double pi = 3.141592653589793;
  const double A = P.gw_A, d = P.gw_d;
  const int a = P.gw_axis;
  double s, c;
  sincos(2.0 * pi * (xa - t) / d, &s, &c);
  const double H = 1.0 - A * s;
  const double L = log(H);
  const double Hm13 = exp(-L / 3.0);
  double v[V_N];
#pragma unroll
  for (int q = 0; q < V_N; ++q) v[q] = 0.0;
  v[V_CHI] = Hm13;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int q = sidx(b, b);
    if (b == a) {
      v[V_GT + q] = exp(2.0 * L / 3.0);
      v[V_AT + q] = -(2.0 * pi * A / (3.0 * d)) * c * exp(-5.0 * L / 6.0);
    } else {
      v[V_GT + q] = Hm13;
      v[V_AT + q] = (pi * A / (3.0 * d)) * c * exp(-11.0 * L / 6.0);
    }
  }
  v[V_TRK] = -(pi * A / d) * c * exp(-1.5 * L);
  const double gam = -(4.0 * pi * A / (3.0 * d)) * c * exp(-5.0 * L / 3.0);
#pragma unroll
  for (int b = 0; b < 3; ++b) v[V_GAM + b] = b == a ? gam : 0.0;  // constant indices
  v[V_ALP] = sqrt(H);
#pragma unroll
  for (int q = 0; q < V_N; ++q) f[q * sv] = v[q];
}

__device__ __forceinline__ double* patch_state(const Batch& B, const PatchDesc& p) {
  return reinterpret_cast<double*>(B.base + p.state_off);
}

__device__ __forceinline__ void stage_buffers(const Batch& B, const PatchDesc& p, int io,
                                              StageIO& s, double dt) {
  double* const state = patch_state(B, p);
  double* const ws = reinterpret_cast<double*>(B.base + p.ws_off);
  double* B1 = ws;
  double* B2 = ws + p.E;
  double* acc = ws + 2 * p.E;
  s.y0 = state;
  s.acc = acc;
  switch (io) {
    case 0: s.yin = state; s.out = B1; s.cdt = 0.0; break;
    case 1: s.yin = state; s.out = B1; s.cdt = 0.5 * dt; break;
    case 2: s.yin = B1; s.out = B2; s.cdt = 0.5 * dt; break;
    case 3: s.yin = B2; s.out = B1; s.cdt = dt; break;
    default: s.yin = B1; s.out = state; s.cdt = dt / 6.0; break;
  }
}


// ---- kernel instances, one translation unit each ------------------------------
//   kind 0: stencil neighbours through the caches, tile per patch (tz planes)
//   kinds 1 / 2: LDS-staged 4th order, 32x8 / 16x16 single-plane tiles
//   kinds 3 / 5: LDS-staged 6th order, 32x8 / 16x16
//   kinds 4 / 6: LDS-staged 8th order, 32x8 / 16x16
//   kind 7: LDS-staged 4th order, z-blocked 32x8x2 tiles (mixed precision,
//     no dissipation)
// launch_batch_kind<K>: one substage (0 = right-hand side only, 1..4) over
// the work list of b on grid workgroups, the instance with prolongation
// ghost items when par; batch_per_cu<K>: resident workgroups per CU of that
// instance (its registers and LDS decide).
constexpr int kNumKinds = 8;
// host side of batch_persistent (batch_stage.h): FP64 kinds 0-2 stride
// their share with a resident grid, every other instance takes one item per
// workgroup
inline bool batch_persistent_host(int precision, int kind) {
  return precision == CHEMORA_FP64 && kind <= 2;
}
template <int K>
hipError_t launch_batch_kind(int precision, bool ko, bool par, int stage, const Batch& b,
                             unsigned grid, hipStream_t s);
template <int K>
int batch_per_cu(int precision, bool ko, bool par);
#define CHEMORA_BATCH_KIND_DECL(K)                                                            \
  template <>                                                                                 \
  hipError_t launch_batch_kind<K>(int precision, bool ko, bool par, int stage, const Batch& b, \
                                  unsigned grid, hipStream_t s);                              \
  template <>                                                                                 \
  int batch_per_cu<K>(int precision, bool ko, bool par);
CHEMORA_BATCH_KIND_DECL(0)
CHEMORA_BATCH_KIND_DECL(1)
CHEMORA_BATCH_KIND_DECL(2)
CHEMORA_BATCH_KIND_DECL(3)
CHEMORA_BATCH_KIND_DECL(4)
CHEMORA_BATCH_KIND_DECL(5)
CHEMORA_BATCH_KIND_DECL(6)
CHEMORA_BATCH_KIND_DECL(7)
#undef CHEMORA_BATCH_KIND_DECL

}  // namespace chemora
