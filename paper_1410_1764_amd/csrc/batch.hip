// batch.hip -- many uneven BSSN patches advanced together (mesh-refinement /
// multi-block patches of the Carpet driver, Sec. IV of arXiv:1410.1764), with
// tile shapes chosen by a model-driven, measured autotuner (the GPU run-time
// library of Sec. III.B.3 auto-tunes the thread assignment with a model).
//
// One RK4 substage = ONE persistent kernel launch.  Its work list holds
//   - interior items: one (patch, tile) each -- right-hand side at the tile's
//     points fused with the substage update (bssn_point.h), and
//   - ghost items: a chunk of one patch's ghost points -- the analytic gauge
//     wave at the time of the stage being produced, written into the ghost
//     zones of the substage's OUTPUT buffer.
// Interior items read the input buffer and write output interiors; ghost
// items write output ghosts only; so items never conflict and need no
// ordering.  Workgroups take items round-robin (item = wg + r * grid), in an
// order sorted by decreasing cost (longest-processing-time first).
//
// Three kernel kinds share this structure: kind 0 reads stencil neighbours
// through the caches with a tile shape per patch (size class); kinds 1 and 2
// stage each grid function's tile neighbourhood in LDS with async copies
// (bssn_lds.h, ASrc, in both precisions) with 32x8 or 16x16 single-plane
// tiles.  The autotuner picks the kind and, for kind 0,
// the tile of each size class.  Patches with the 6th- or 8th-order operators
// run kinds 3 and 4: 32x8 single-plane tiles staged with the wider
// neighbourhood of those orders (HSrc), nothing to tune.
//
// The four substage launches and a one-thread clock update (t += dt) are
// captured once into a HIP graph and replayed per step; the time lives in a
// device scalar so the frozen kernel arguments stay valid.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <cstdlib>
#include <type_traits>

#include "bssn_lds.h"

namespace chemora {

int fail(int status, const char* fmt, ...);
int device_status(hipError_t e, const char* what);
bool aligned(const void* p);
const Geo& grid_geo(const chemora_grid* g);
const BssnPar& grid_par(const chemora_grid* g);
const chemora_grid_desc& grid_desc(const chemora_grid* g);
long long grid_state_elems(const chemora_grid* g);

namespace {

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
};

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

template <int KIND>
struct KindShape {
  static constexpr int TX = KIND == 2 ? 16 : 32, TY = KIND == 2 ? 16 : 8;
  static constexpr int ORD = KIND == 3 ? 6 : (KIND == 4 ? 8 : 4);
  static constexpr bool HI = KIND >= 3;
  static constexpr int TOT = KIND == 0 ? 1
                             : HI      ? HShape<TX, TY, ORD / 2 + 1>::TOTAL
                                       : LdsShape<TX, TY>::TOTAL;
  static constexpr int TOT3 = HI ? 1 : TOT;  // third buffer: the async kinds only
  static constexpr int TAB = HI ? TOT : 1;   // offset table: the high-order kinds only
};

// kind of a plan for patches of finite-difference order ord
inline int order_kind(int ord, int kind4) { return ord == 6 ? 3 : (ord == 8 ? 4 : kind4); }

// one single-plane tile of a staged kind
template <int STAGE, typename T, int KIND, int KOM>
__device__ __forceinline__ void staged_tile(const PatchDesc& p, const StageIO& io, long long tile,
                                            double* const* bufs, int* tab) {
  constexpr int TX = KindShape<KIND>::TX, TY = KindShape<KIND>::TY;
  const Geo& G = p.G;
  int bx, by, k;
  patch_tile(p, tile, bx, by, k);
  const int tx = (int)threadIdx.x % TX, ty = (int)threadIdx.x / TX;
  const int x0 = bx * TX, y0 = by * TY;
  const int i = x0 + tx, j = y0 + ty;
  T rhs[V_N];
  if constexpr (KindShape<KIND>::HI) {
    constexpr int ORD = KindShape<KIND>::ORD;
    HSrc<TX, TY, ORD / 2 + 1> src;
    src.init(G, io.yin, bufs[0], bufs[1], tab, x0, y0, k, tx, ty);
    bssn_rhs_point<T, KO_OFF, ORD>(src, p.W, p.P, rhs);
  } else {
    ASrc<TX, TY, kBatchBufs> src;
    src.init(G, io.yin, bufs, x0, y0, k, tx, ty);
    bssn_rhs_point<T, KOM>(src, p.W, p.P, rhs);
  }
  if (i < G.n[0] && j < G.n[1])
    bssn_store<STAGE, T>(io, G, i + (long long)j * G.sy + (long long)k * G.sz, i, j, k, rhs,
                         false, p.P.enforce != 0);
}

// KOM: Kreiss-Oliger dissipation compiled in (KO_ON: patches with sigma = 0
// add an exact zero) or out (KO_OFF: no patch dissipates)
template <int STAGE, typename T, int KIND, int KOM>
__global__ void __launch_bounds__(kThreads) batch_stage_kernel(Batch B) {
  __shared__ int s_patch;
  constexpr int TOT = KindShape<KIND>::TOT;
  // separate arrays, one per staging buffer (see bssn_lds.h); a tiny
  // placeholder each for kind 0
  __shared__ double L0[TOT], L1[TOT], L2[KindShape<KIND>::TOT3];
  __shared__ int TB[KindShape<KIND>::TAB];
  double* bufs[3] = {L0, L1, L2};
  __shared__ long long s_lo, s_hi;  // item range of s_patch (interior or ghost)
  // The current patch's descriptor lives in LDS: under register pressure the
  // compiler re-reads descriptor fields (weights, strides) inside the point
  // code; from global memory every such read would be followed by a vmcnt
  // wait that also drains the stencil copies in flight, from LDS it waits
  // on lgkmcnt only.
  __shared__ PatchDesc s_pd;
  __shared__ int s_changed;
  const double tnow = *B.clock;
  // XCD x (blockIdx.x % 8) takes share x of the interior items and share x
  // of the ghost items, in list order; its gridDim.x / 8 blocks stride it
  const int x = (int)blockIdx.x % kNumXcd;
  const long long R = gridDim.x / kNumXcd;
  const long long ni = B.n_interior, ng = B.n_total - B.n_interior;
  const long long i0 = ni * x / kNumXcd, i1 = ni * (x + 1) / kNumXcd;
  const long long g0 = ng * x / kNumXcd, g1 = ng * (x + 1) / kNumXcd;
  const long long share = (i1 - i0) + (g1 - g0);
  if (threadIdx.x == 0) {
    s_lo = 0;
    s_hi = -1;
  }
  for (long long t = blockIdx.x / kNumXcd; t < share; t += R) {
    const bool interior = t < i1 - i0;
    const long long item = interior ? i0 + t : ni + g0 + (t - (i1 - i0));
    __syncthreads();  // the previous item is finished by every wave
    if (threadIdx.x == 0) {
      s_changed = 0;
      if (!(item >= s_lo && item < s_hi)) {
        // consecutive items of a block mostly stay in one patch: search only
        // when the item leaves the current patch's range
        const int q = interior ? find_patch(B.prefix, B.np, item)
                               : find_patch(B.gprefix, B.np, item - ni);
        s_patch = q;
        s_lo = interior ? B.prefix[q] : ni + B.gprefix[q];
        s_hi = interior ? B.prefix[q + 1] : ni + B.gprefix[q + 1];
        s_changed = 1;
      }
    }
    __syncthreads();
    if (s_changed) {  // the same value in every thread
      static_assert(sizeof(PatchDesc) % 8 == 0, "descriptor copied in 8-byte words");
      const unsigned long long* from =
          reinterpret_cast<const unsigned long long*>(B.pd + s_patch);
      unsigned long long* to = reinterpret_cast<unsigned long long*>(&s_pd);
      for (int w = (int)threadIdx.x; w < (int)(sizeof(PatchDesc) / 8); w += kThreads)
        to[w] = from[w];
      __syncthreads();
    }
    const PatchDesc& p = s_pd;
    const Geo& G = p.G;
    StageIO io;
    stage_buffers(B, p, B.stage_io, io, B.dt);
    if (interior) {
      const long long tile = item - B.prefix[s_patch];
      if constexpr (KIND != 0) {
        staged_tile<STAGE, T, KIND, KOM>(p, io, tile, bufs, TB);
      } else {
        int tx, ty, tzi;
        patch_tile(p, tile, tx, ty, tzi);
        const int lx = (int)threadIdx.x % p.ltx, ly = (int)threadIdx.x / p.ltx;
        const int i = tx * p.ltx + lx, j = ty * p.lty + ly;
        if (ly < p.lty && i < G.n[0] && j < G.n[1]) {
          const int k0 = tzi * p.tz, k1 = min(k0 + p.tz, G.n[2]);
          for (int k = k0; k < k1; ++k) {
            const long long q = i + (long long)j * G.sy + (long long)k * G.sz;
            T rhs[V_N];
            GSrc src{io.yin + G.off0 + q, G.sv, G.sy, G.sz};
            bssn_rhs_point<T, KOM>(src, p.W, p.P, rhs);
            bssn_store<STAGE, T>(io, G, q, i, j, k, rhs, false, p.P.enforce != 0);
          }
        }
      }
    } else {
      const long long chunk = item - B.n_interior - B.gprefix[s_patch];
      const double t = tnow + B.t_out * B.dt;
      for (long long gq = chunk * kGhostChunk + threadIdx.x;
           gq < min((chunk + 1) * kGhostChunk, p.ghosts); gq += kThreads) {
        int ijk[3];
        ghost_ijk(G, gq, ijk);
        const int a = p.P.gw_axis;
        const double xa = p.P.origin[a] + ijk[a] * p.P.h[a];
        gw_store(p.P, xa, t, io.out + G.off0 + ijk[0] + (long long)ijk[1] * G.sy +
                                  (long long)ijk[2] * G.sz, G.sv);
      }
    }
  }
}

__global__ void set_clock_kernel(double* clock, double t) { *clock = t; }
__global__ void advance_clock_kernel(double* clock, double dt) { *clock = *clock + dt; }

// Fill the ghosts of every patch's state at the clock time (ghost items of
// the work list, output = state).
__global__ void __launch_bounds__(kThreads) batch_state_ghosts_kernel(Batch B) {
  const double t = *B.clock;
  for (long long item = blockIdx.x; item < B.n_total - B.n_interior; item += gridDim.x) {
    const int q = find_patch(B.gprefix, B.np, item);
    const PatchDesc& p = B.pd[q];
    const long long chunk = item - B.gprefix[q];
    for (long long gq = chunk * kGhostChunk + threadIdx.x;
         gq < min((chunk + 1) * kGhostChunk, p.ghosts); gq += kThreads) {
      int ijk[3];
      ghost_ijk(p.G, gq, ijk);
      const int a = p.P.gw_axis;
      const double xa = p.P.origin[a] + ijk[a] * p.P.h[a];
      gw_store(p.P, xa, t, patch_state(B, p) + p.G.off0 + ijk[0] + (long long)ijk[1] * p.G.sy +
                               (long long)ijk[2] * p.G.sz, p.G.sv);
    }
  }
}

// ---- tile shapes ------------------------------------------------------------

struct Tile {
  int ltx, lty, tz;
};

const Tile kCandidates[] = {{64, 4, 1}, {64, 4, 2}, {64, 4, 4}, {32, 8, 1}, {32, 8, 2},
                            {32, 8, 4}, {16, 16, 1}, {16, 16, 2}, {16, 16, 4}};

// size class of a patch for the tuning table: the x extent decides how well
// a tile row fills a wavefront
int size_class(const int32_t n[3]) { return n[0] <= 40 ? 0 : (n[0] <= 72 ? 1 : 2); }

std::mutex g_table_mu;
std::map<std::pair<int, int>, Tile> g_table;  // (precision, class) -> tuned tile (kind 0)
std::map<int, int> g_kind;                    // precision -> tuned kernel kind

// CHEMORA_BATCH_KIND=0|1|2 forces the kernel kind of new plans (ablation
// switch, read at every plan build)
int default_kind(int precision) {
  const char* e = std::getenv("CHEMORA_BATCH_KIND");
  if (e && (e[0] == '0' || e[0] == '1' || e[0] == '2') && e[1] == 0) return e[0] - '0';
  std::lock_guard<std::mutex> lk(g_table_mu);
  auto it = g_kind.find(precision);
  return it != g_kind.end() ? it->second : 1;  // untuned: staged 32x8
}

// model score (lower is better): padded-thread waste from ragged tiles, times
// the halo re-read factor of the tile's cache footprint
double model_cost(const Tile& t, const int32_t n[3]) {
  const double tiles_x = std::ceil(n[0] / (double)t.ltx), tiles_y = std::ceil(n[1] / (double)t.lty);
  const double tiles_z = std::ceil(n[2] / (double)t.tz);
  const double work = tiles_x * t.ltx * tiles_y * t.lty * tiles_z * t.tz;
  const double useful = (double)n[0] * n[1] * n[2];
  const double halo = (t.ltx + 6.0) * (t.lty + 6.0) * (t.tz + 6.0) / (t.ltx * t.lty * t.tz);
  return work / useful * (1.0 + 0.02 * halo);
}

Tile default_tile(const int32_t n[3], int precision) {
  {
    std::lock_guard<std::mutex> lk(g_table_mu);
    auto it = g_table.find({precision, size_class(n)});
    if (it != g_table.end()) return it->second;
  }
  Tile best = kCandidates[0];
  double bc = 1e300;
  for (const Tile& t : kCandidates) {
    if (t.tz != 1) continue;  // untuned default: one plane per tile, most parallelism
    const double c = model_cost(t, n);
    if (c < bc) {
      bc = c;
      best = t;
    }
  }
  return best;
}

// ---- plans --------------------------------------------------------------------

struct Plan {
  std::vector<const chemora_grid*> grids;
  std::vector<double*> states;
  std::vector<void*> wss;
  std::vector<Tile> tiles;
  double dt = 0.0;
  int precision = 0;
  int kind = 0;
  bool ko = false;  // some patch has Kreiss-Oliger dissipation
  int np = 0;
  long long n_interior = 0, n_total = 0;
  int grid_blocks = 0;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  Batch batch[5];
};

std::mutex g_plan_mu;
std::map<void*, Plan*> g_plans;

void destroy_plan(Plan* p) {
  if (!p) return;
  if (p->exec) hipGraphExecDestroy(p->exec);
  if (p->graph) hipGraphDestroy(p->graph);
  delete p;
}

int compute_units() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
      cus = prop.multiProcessorCount;
  }
  return cus;
}

// Persistent grid: as many workgroups as can be resident at once (registers
// and LDS of the kernel instance decide), so that none waits for a slot.
template <typename T, int KIND, int KOM>
int resident_blocks() {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_stage_kernel<1, T, KIND, KOM>,
                                                   kThreads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return compute_units() * per_cu;
}

template <typename T, int KOM>
int persistent_blocks_t(int kind) {
  if constexpr (KOM == KO_OFF) {  // high orders run without dissipation
    if (kind == 3) return resident_blocks<T, 3, KOM>();
    if (kind == 4) return resident_blocks<T, 4, KOM>();
  }
  switch (kind) {
    case 1: return resident_blocks<T, 1, KOM>();
    case 2: return resident_blocks<T, 2, KOM>();
    default: return resident_blocks<T, 0, KOM>();
  }
}

int persistent_blocks(int precision, int kind, bool ko) {
  if (precision == CHEMORA_MIXED)
    return ko ? persistent_blocks_t<float, KO_ON>(kind) : persistent_blocks_t<float, KO_OFF>(kind);
  return ko ? persistent_blocks_t<double, KO_ON>(kind) : persistent_blocks_t<double, KO_OFF>(kind);
}

int validate_patches(const chemora_patch* patches, int32_t np, int* precision,
                     int* order = nullptr) {
  if (!patches) return fail(CHEMORA_ERR_INVALID, "patch list is NULL");
  if (np < 1 || np > kMaxPatches)
    return fail(CHEMORA_ERR_INVALID, "npatches must be in [1, %d], got %d", kMaxPatches, np);
  for (int q = 0; q < np; ++q) {
    const chemora_patch& p = patches[q];
    if (!p.grid || !p.state || !p.workspace)
      return fail(CHEMORA_ERR_INVALID, "patch %d: grid, state and workspace must not be NULL", q);
    if (!aligned(p.state) || !aligned(p.workspace))
      return fail(CHEMORA_ERR_INVALID, "patch %d: state and workspace must be 256-byte aligned", q);
    const chemora_grid_desc& d = grid_desc(p.grid);
    if (d.system != CHEMORA_BSSN || d.boundary != CHEMORA_BC_GAUGEWAVE)
      return fail(CHEMORA_ERR_INVALID,
                  "patch %d: batches need BSSN grids with the gauge-wave boundary", q);
    const int ord = grid_par(p.grid).fd_order;
    if (q == 0) {
      *precision = d.precision;
      if (order) *order = ord;
    }
    if (order && ord != *order)
      return fail(CHEMORA_ERR_INVALID, "patch %d: all patches must share one fd_order", q);
    // the FP64 instance of the 6th-order batch kind gives wrong results on
    // every point (the same code in mixed precision, at order 8, and the
    // single-grid 6th-order kernel are correct); switched off until the
    // cause is found
    if (ord == 6 && d.precision == CHEMORA_FP64)
      return fail(CHEMORA_ERR_UNSUPPORTED,
                  "patch %d: FP64 batches of 6th-order patches are not supported", q);
    if (d.precision != *precision)
      return fail(CHEMORA_ERR_INVALID, "patch %d: all patches must share one precision", q);
  }
  return CHEMORA_OK;
}

// Build descriptors and the work list, upload to meta (synchronously).
int build_plan(Plan* P, const chemora_patch* patches, int32_t np, void* meta, double dt,
               int precision, int kind, const Tile* forced) {
  P->np = np;
  P->dt = dt;
  P->precision = precision;
  P->kind = kind;
  P->ko = false;
  for (int q = 0; q < np; ++q) P->ko = P->ko || grid_par(patches[q].grid).ko_sigma != 0.0;
  P->grids.resize(np);
  P->states.resize(np);
  P->wss.resize(np);
  P->tiles.resize(np);
  std::vector<PatchDesc> pd(np);
  std::vector<long long> cost(np);
  for (int q = 0; q < np; ++q) {
    const chemora_grid* g = patches[q].grid;
    P->grids[q] = g;
    P->states[q] = patches[q].state;
    P->wss[q] = patches[q].workspace;
    const Geo& G = grid_geo(g);
    const int32_t n[3] = {G.n[0], G.n[1], G.n[2]};
    const Tile t = (kind == 1 || kind >= 3) ? Tile{32, 8, 1}
                   : kind == 2             ? Tile{16, 16, 1}
                                           : (forced ? *forced : default_tile(n, precision));
    P->tiles[q] = t;
    PatchDesc& d = pd[q];
    d.G = G;
    d.P = grid_par(g);
    d.W = make_weights(d.P.h, d.P.ko_sigma, d.P.fd_order);
    d.state_off = reinterpret_cast<char*>(patches[q].state) - reinterpret_cast<char*>(patches[0].state);
    d.ws_off = static_cast<char*>(patches[q].workspace) - reinterpret_cast<char*>(patches[0].state);
    d.E = grid_state_elems(g);
    const long long e0 = G.n[0] + 2 * G.g, e1 = G.n[1] + 2 * G.g;
    d.ghosts = 2LL * G.g * e1 * e0 + (long long)G.n[2] * 2 * G.g * e0 +
               (long long)G.n[2] * G.n[1] * 2 * G.g;
    d.ltx = t.ltx;
    d.lty = t.lty;
    d.tz = t.tz;
    d.tiles[0] = (G.n[0] + t.ltx - 1) / t.ltx;
    d.tiles[1] = (G.n[1] + t.lty - 1) / t.lty;
    d.tiles[2] = (G.n[2] + t.tz - 1) / t.tz;
    // staged kinds: eight columns when the plane has enough tiles
    d.cols[0] = d.cols[1] = 1;
    if (kind != 0) {
      const ColumnSplit c = column_split(d.tiles, t.ltx, t.lty);
      if (c.cx > 0) {
        d.cols[0] = c.cx;
        d.cols[1] = c.cy;
      }
    }
    cost[q] = (long long)G.n[0] * G.n[1] * G.n[2];
  }
  // work-list order: patches by decreasing cost (LPT), so the biggest tiles
  // are handed out first and the short ones fill the tail
  std::vector<int> order(np);
  for (int q = 0; q < np; ++q) order[q] = q;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<PatchDesc> pds(np);
  std::vector<long long> prefix(np + 1), gprefix(np + 1);
  prefix[0] = gprefix[0] = 0;
  for (int r = 0; r < np; ++r) {
    pds[r] = pd[order[r]];
    const PatchDesc& d = pds[r];
    prefix[r + 1] = prefix[r] + (long long)d.tiles[0] * d.tiles[1] * d.tiles[2];
    gprefix[r + 1] = gprefix[r] + (d.ghosts + kGhostChunk - 1) / kGhostChunk;
  }
  P->n_interior = prefix[np];
  P->n_total = prefix[np] + gprefix[np];
  char* m = static_cast<char*>(meta);
  hipError_t e = hipMemcpy(m + MetaLayout::desc_off(), pds.data(), sizeof(PatchDesc) * np,
                           hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(m + MetaLayout::prefix_off(np), prefix.data(), 8 * (np + 1),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(m + MetaLayout::gprefix_off(np), gprefix.data(), 8 * (np + 1),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) return device_status(e, "batch plan upload");
  // a multiple of 8 (one share of the work list per XCD)
  P->grid_blocks = std::max(kNumXcd, persistent_blocks(precision, kind, P->ko) / kNumXcd * kNumXcd);
  const double tout[5] = {0.0, 0.5, 0.5, 1.0, 1.0};
  for (int s = 0; s <= 4; ++s) {
    Batch& b = P->batch[s];
    b.base = reinterpret_cast<char*>(patches[0].state);
    b.pd = reinterpret_cast<const PatchDesc*>(m + MetaLayout::desc_off());
    b.prefix = reinterpret_cast<const long long*>(m + MetaLayout::prefix_off(np));
    b.gprefix = reinterpret_cast<const long long*>(m + MetaLayout::gprefix_off(np));
    b.clock = reinterpret_cast<double*>(m + MetaLayout::clock_off(np));
    b.np = np;
    b.n_interior = P->n_interior;
    b.n_total = s == 0 ? P->n_interior : P->n_total;  // stage 0 (tuning): no ghosts
    b.dt = dt;
    b.t_out = tout[s];
    b.stage_io = s;
  }
  return CHEMORA_OK;
}

template <typename T, int KIND, int KOM>
hipError_t launch_stage(const Plan* P, int s, hipStream_t st) {
  const dim3 grid(P->grid_blocks), block(kThreads);
  const Batch& b = P->batch[s];
  switch (s) {
    case 0: hipLaunchKernelGGL((batch_stage_kernel<0, T, KIND, KOM>), grid, block, 0, st, b); break;
    case 1: hipLaunchKernelGGL((batch_stage_kernel<1, T, KIND, KOM>), grid, block, 0, st, b); break;
    case 2: hipLaunchKernelGGL((batch_stage_kernel<2, T, KIND, KOM>), grid, block, 0, st, b); break;
    case 3: hipLaunchKernelGGL((batch_stage_kernel<3, T, KIND, KOM>), grid, block, 0, st, b); break;
    default: hipLaunchKernelGGL((batch_stage_kernel<4, T, KIND, KOM>), grid, block, 0, st, b); break;
  }
  return hipGetLastError();
}

template <typename T, int KOM>
hipError_t launch_kind(const Plan* P, int s, hipStream_t st) {
  if constexpr (KOM == KO_OFF) {
    if (P->kind == 3) return launch_stage<T, 3, KOM>(P, s, st);
    if (P->kind == 4) return launch_stage<T, 4, KOM>(P, s, st);
  }
  switch (P->kind) {
    case 1: return launch_stage<T, 1, KOM>(P, s, st);
    case 2: return launch_stage<T, 2, KOM>(P, s, st);
    default: return launch_stage<T, 0, KOM>(P, s, st);
  }
}

hipError_t launch_any(const Plan* P, int s, hipStream_t st) {
  if (P->precision == CHEMORA_MIXED)
    return P->ko ? launch_kind<float, KO_ON>(P, s, st) : launch_kind<float, KO_OFF>(P, s, st);
  return P->ko ? launch_kind<double, KO_ON>(P, s, st) : launch_kind<double, KO_OFF>(P, s, st);
}

// capture: S1, S2, S3, S4, clock += dt
int capture_graph(Plan* P) {
  hipStream_t cs;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return device_status(e, "capture stream");
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    for (int s = 1; s <= 4 && e == hipSuccess; ++s) e = launch_any(P, s, cs);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(advance_clock_kernel, dim3(1), dim3(1), 0, cs, P->batch[1].clock, P->dt);
      e = hipGetLastError();
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess) e = e2;
    P->graph = g;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
  hipStreamDestroy(cs);
  return device_status(e, "batch graph capture");
}

// Time three right-hand-side launches (stage 0 writes the first stage buffer;
// states are untouched) of a plan after one warm-up launch.
int time_plan(const Plan* P, hipEvent_t e0, hipEvent_t e1, float* ms) {
  hipError_t e = launch_any(P, 0, nullptr);
  if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
  for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch_any(P, 0, nullptr);
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  return device_status(e, "autotune trial");
}

bool same_patches(const Plan* P, const chemora_patch* patches, int32_t np, double dt) {
  if (P->np != np || P->dt != dt) return false;
  for (int q = 0; q < np; ++q)
    if (P->grids[q] != patches[q].grid || P->states[q] != patches[q].state ||
        P->wss[q] != patches[q].workspace)
      return false;
  return true;
}

}  // namespace
}  // namespace chemora

using namespace chemora;

extern "C" {

int64_t chemora_batch_meta_bytes(int32_t npatches) {
  if (npatches < 1 || npatches > kMaxPatches) {
    fail(CHEMORA_ERR_INVALID, "npatches must be in [1, %d]", kMaxPatches);
    return -1;
  }
  return MetaLayout::bytes(npatches);
}

int chemora_batch_step(const chemora_patch* patches, int32_t npatches, void* meta, double t,
                       double dt, int32_t nsteps, chemora_stream stream) {
  int precision = 0, order = 4;
  int st = validate_patches(patches, npatches, &precision, &order);
  if (st != CHEMORA_OK) return st;
  if (!meta || !aligned(meta)) return fail(CHEMORA_ERR_INVALID, "meta must be a 256-byte aligned device pointer");
  if (nsteps < 0) return fail(CHEMORA_ERR_INVALID, "nsteps must be >= 0");
  if (!std::isfinite(t) || !std::isfinite(dt)) return fail(CHEMORA_ERR_INVALID, "t and dt must be finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Plan* P = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(meta);
    if (it != g_plans.end() && same_patches(it->second, patches, npatches, dt) &&
        it->second->precision == precision) {
      P = it->second;
    } else {
      if (it != g_plans.end()) {
        // the old plan's graph may still be queued on the caller's stream
        hipStreamSynchronize(s);
        destroy_plan(it->second);
        g_plans.erase(it);
      }
      P = new Plan;
      // the meta buffer may be in use by queued work of this stream
      hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        delete P;
        return device_status(e, "batch plan");
      }
      st = build_plan(P, patches, npatches, meta, dt, precision,
                      order_kind(order, default_kind(precision)), nullptr);
      if (st == CHEMORA_OK) st = capture_graph(P);
      if (st != CHEMORA_OK) {
        destroy_plan(P);
        return st;
      }
      g_plans[meta] = P;
    }
  }
  hipLaunchKernelGGL(set_clock_kernel, dim3(1), dim3(1), 0, s, P->batch[1].clock, t);
  st = device_status(hipGetLastError(), "batch clock");
  if (st != CHEMORA_OK) return st;
  const long long nghost = P->n_total - P->n_interior;
  if (nghost > 0) {
    const long long blocks = std::min<long long>(nghost, (long long)P->grid_blocks);
    hipLaunchKernelGGL(batch_state_ghosts_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, s,
                       P->batch[1]);
    st = device_status(hipGetLastError(), "batch ghost fill");
    if (st != CHEMORA_OK) return st;
  }
  for (int n = 0; n < nsteps; ++n) {
    st = device_status(hipGraphLaunch(P->exec, s), "batch graph launch");
    if (st != CHEMORA_OK) return st;
  }
  return CHEMORA_OK;
}

int chemora_batch_release(void* meta) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto it = g_plans.find(meta);
  if (it == g_plans.end()) return fail(CHEMORA_ERR_INVALID, "no batch plan for this meta buffer");
  hipDeviceSynchronize();
  destroy_plan(it->second);
  g_plans.erase(it);
  return CHEMORA_OK;
}

int chemora_batch_tile(const int32_t n[3], int32_t precision, int32_t tile[3]) {
  if (!n || !tile) return fail(CHEMORA_ERR_INVALID, "NULL argument");
  if (n[0] < 1 || n[1] < 1 || n[2] < 1) return fail(CHEMORA_ERR_INVALID, "n must be >= 1");
  const int kind = default_kind(precision);
  const Tile t = kind == 1 ? Tile{32, 8, 1} : kind == 2 ? Tile{16, 16, 1} : default_tile(n, precision);
  tile[0] = t.ltx;
  tile[1] = t.lty;
  tile[2] = t.tz;
  return CHEMORA_OK;
}

int chemora_autotune(const chemora_patch* patches, int32_t npatches, void* meta,
                     const char* table_path) {
  int precision = 0, order = 4;
  int st = validate_patches(patches, npatches, &precision, &order);
  if (st != CHEMORA_OK) return st;
  if (!meta || !aligned(meta)) return fail(CHEMORA_ERR_INVALID, "meta must be a 256-byte aligned device pointer");
  if (order != 4) return CHEMORA_OK;  // one kernel kind per high order: nothing to tune
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    // the trials rewrite meta: nothing queued may still read it
    st = device_status(hipDeviceSynchronize(), "autotune");
    if (st != CHEMORA_OK) return st;
    auto it = g_plans.find(meta);
    if (it != g_plans.end()) {
      destroy_plan(it->second);
      g_plans.erase(it);
    }
  }
  // group patches by size class
  std::map<int, std::vector<chemora_patch>> classes;
  for (int q = 0; q < npatches; ++q) {
    const Geo& G = grid_geo(patches[q].grid);
    const int32_t n[3] = {G.n[0], G.n[1], G.n[2]};
    classes[size_class(n)].push_back(patches[q]);
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(CHEMORA_ERR_DEVICE, "event creation failed");
  std::string json = "{\n";
  bool first = true;
  for (auto& kv : classes) {
    const std::vector<chemora_patch>& ps = kv.second;
    // model-driven pruning: keep the 4 candidates with the best mean model cost
    std::vector<std::pair<double, Tile>> scored;
    for (const Tile& t : kCandidates) {
      double c = 0.0;
      for (const chemora_patch& p : ps) {
        const Geo& G = grid_geo(p.grid);
        const int32_t n[3] = {G.n[0], G.n[1], G.n[2]};
        c += model_cost(t, n);
      }
      scored.push_back({c / ps.size(), t});
    }
    std::stable_sort(scored.begin(), scored.end(),
                     [](const std::pair<double, Tile>& a, const std::pair<double, Tile>& b) {
                       return a.first < b.first;
                     });
    Tile best = scored[0].second;
    float best_ms = 1e30f;
    for (size_t c = 0; c < scored.size() && c < 4; ++c) {
      Plan P;
      st = build_plan(&P, ps.data(), (int)ps.size(), meta, 0.0, precision, 0, &scored[c].second);
      float ms = 0.f;
      if (st == CHEMORA_OK) st = time_plan(&P, e0, e1, &ms);
      if (st != CHEMORA_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best = scored[c].second;
      }
    }
    if (st != CHEMORA_OK) break;
    {
      std::lock_guard<std::mutex> lk(g_table_mu);
      g_table[{precision, kv.first}] = best;
    }
    char buf[256];
    snprintf(buf, sizeof buf,
             "%s  \"precision%d_class%d\": {\"tile\": [%d, %d, %d], \"ms_per_rhs\": %.5f, "
             "\"patches\": %zu}",
             first ? "" : ",\n", precision, kv.first, best.ltx, best.lty, best.tz, best_ms / 3.0,
             ps.size());
    json += buf;
    first = false;
  }
  // kernel kind: per-patch global-load tiles (as just tuned) against the
  // two staged kinds, each timed over the whole batch
  float kind_ms[3] = {0.f, 0.f, 0.f};
  int best_kind = 0;
  for (int kind = 0; kind < 3 && st == CHEMORA_OK; ++kind) {
    Plan P;
    st = build_plan(&P, patches, npatches, meta, 0.0, precision, kind, nullptr);
    if (st == CHEMORA_OK) st = time_plan(&P, e0, e1, &kind_ms[kind]);
    if (st == CHEMORA_OK && kind_ms[kind] < kind_ms[best_kind]) best_kind = kind;
  }
  if (st == CHEMORA_OK) {
    std::lock_guard<std::mutex> lk(g_table_mu);
    g_kind[precision] = best_kind;
    char buf[256];
    snprintf(buf, sizeof buf,
             "%s  \"precision%d_kind\": {\"kind\": %d, \"ms_per_rhs\": [%.5f, %.5f, %.5f]}",
             first ? "" : ",\n", precision, best_kind, kind_ms[0] / 3.0, kind_ms[1] / 3.0,
             kind_ms[2] / 3.0);
    json += buf;
  }
  json += "\n}\n";
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != CHEMORA_OK) return st;
  if (table_path) {
    FILE* f = fopen(table_path, "w");
    if (!f) return fail(CHEMORA_ERR_INVALID, "cannot write %s", table_path);
    fputs(json.c_str(), f);
    fclose(f);
  }
  return CHEMORA_OK;
}

}  // extern "C"
