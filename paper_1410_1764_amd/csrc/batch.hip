// batch.hip -- many uneven BSSN patches advanced together (mesh-refinement /
// multi-block patches of the Carpet driver, Sec. IV of arXiv:1410.1764), with
// tile shapes chosen by a model-driven, measured autotuner (the GPU run-time
// library of Sec. III.B.3 auto-tunes the thread assignment with a model).
//
// One RK4 substage = ONE kernel launch (batch_stage.h).  Its work
// list holds
//   - interior items: one (patch, tile) each -- right-hand side at the tile's
//     points fused with the substage update (bssn_point.h), and
//   - ghost items: a chunk of one patch's ghost points -- the analytic gauge
//     wave at the time of the stage being produced, written into the ghost
//     zones of the substage's OUTPUT buffer.
// Interior items read the input buffer and write output interiors; ghost
// items write output ghosts only; so items never conflict and need no
// ordering.  The list is sorted by decreasing patch size (longest-
// processing-time first) and cut into one share per XCD.  FP64 4th-order
// instances run a resident grid whose workgroups stride their XCD's share;
// every other instance gets one workgroup per item and the hardware hands
// them out in order (a loop of one iteration, so the compiler does not hold
// loop-invariant values through the point code: that cost mixed batches a
// wave per SIMD and spilled the high-order instances).
//
// Kernel instances ("kinds", one translation unit each): kind 0 reads
// stencil neighbours through the caches, with a tile of 1..4 planes per
// patch; the staged kinds stage each grid function's tile neighbourhood in
// LDS (bssn_lds.h: ASrc for 4th order, HSrc for the wider neighbourhood of
// 6th and 8th order) with one single-plane tile shape each: 32x8 (kinds 1,
// 3, 4 for orders 4, 6, 8) or 16x16 (kinds 2, 5, 6); kind 7 stages 4th
// order in z-blocked 32x8x2 tiles (bssn_zsrc.h; mixed precision without
// dissipation, where the point code fits two waves per SIMD).  The autotuner
// (chemora_autotune) picks the tile of kind 0 per size class of patches,
// pruning the candidates with a performance model (model_time) and timing
// the survivors, then times the candidate kinds of the batch's order over
// the whole batch and keeps the fastest.
//
// The four substage launches and a one-thread clock update (t += dt) are
// captured once into a HIP graph and replayed per step; the time lives in a
// device scalar so the frozen kernel arguments stay valid.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "batch_kernel.h"

namespace chemora {

int fail(int status, const char* fmt, ...);
int device_status(hipError_t e, const char* what);
bool aligned(const void* p);
const Geo& grid_geo(const chemora_grid* g);
const BssnPar& grid_par(const chemora_grid* g);
const chemora_grid_desc& grid_desc(const chemora_grid* g);
long long grid_state_elems(const chemora_grid* g);
int grid_nvars(const chemora_grid* g);
int check_prolong_source(const chemora_grid* coarse, const chemora_grid* fine,
                         const double* const* levels, const double* times, int ntimes,
                         const void* avoid, long long avoid_bytes, int off[3]);
hipError_t launch_prolong(const Geo& C, const double* const* yc, const double* wt, int ntimes,
                          const Geo& F, const int off[3], int nvar, double* yf, hipStream_t s);

namespace {

__global__ void set_clock_kernel(double* clock, double t) { *clock = t; }
__global__ void advance_clock_kernel(double* clock, double dt) { *clock = *clock + dt; }

// Fill the ghosts of every patch's state at the clock time (ghost items of
// the work list, output = state).
__global__ void __launch_bounds__(kThreads) batch_state_ghosts_kernel(Batch B) {
  const double t = *B.clock;
  for (long long item = blockIdx.x; item < B.n_total - B.n_interior; item += gridDim.x) {
    const int q = find_patch(B.gprefix, B.np, item);
    const PatchDesc& p = B.pd[q];
    if (p.parent) continue;  // prolongated on the host side of the call
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


// ---- tile shapes and the performance model -------------------------------------

struct Tile {
  int ltx, lty, tz;
};

// kind 0 candidates: 256 threads, 1, 2 or 4 planes per item
const Tile kCandidates[] = {{64, 4, 1}, {64, 4, 2}, {64, 4, 4}, {32, 8, 1}, {32, 8, 2},
                            {32, 8, 4}, {16, 16, 1}, {16, 16, 2}, {16, 16, 4}};
// size class of a patch for the tuning table: the x extent decides how well
// a tile row fills a wavefront
int size_class(const int32_t n[3]) { return n[0] <= 40 ? 0 : (n[0] <= 72 ? 1 : 2); }

// staged kinds of a finite-difference order: {32x8, 16x16}
int staged_kind(int order, bool square) {
  if (order == 6) return square ? 5 : 3;
  if (order == 8) return square ? 6 : 4;
  return square ? 2 : 1;
}

Tile kind_shape(int kind) {
  if (kind == 7) return Tile{32, 8, 2};
  return (kind == 2 || kind == 5 || kind == 6) ? Tile{16, 16, 1} : Tile{32, 8, 1};
}

// the z-blocked kind runs mixed-precision 4th-order batches without dissipation
bool zblocked_ok(int precision, int order, bool ko) {
  return precision == CHEMORA_MIXED && order == 4 && !ko;
}

std::mutex g_table_mu;
// (precision, size class) -> tuned kind 0 tile
std::map<std::pair<int, int>, Tile> g_table;
// (precision, order) -> tuned kernel kind
std::map<std::pair<int, int>, int> g_kind;

// Kernel kind of a new plan.  CHEMORA_BATCH_KIND (ablation switch, read at
// every plan build): 0 = kind 0 (4th order; other orders: 32x8 staged),
// 1 = the 32x8 staged kind of the order, 2 = its 16x16 staged kind, 3 = the
// z-blocked kind where it applies (else 32x8 staged).  Otherwise the tuned
// kind, else the 32x8 staged kind.
int plan_kind(int precision, int order, bool ko) {
  const char* e = std::getenv("CHEMORA_BATCH_KIND");
  if (e && e[0] >= '0' && e[0] <= '3' && e[1] == 0) {
    if (e[0] == '0') return order == 4 ? 0 : staged_kind(order, false);
    if (e[0] == '3') return zblocked_ok(precision, order, ko) ? 7 : staged_kind(order, false);
    return staged_kind(order, e[0] == '2');
  }
  std::lock_guard<std::mutex> lk(g_table_mu);
  auto it = g_kind.find({precision, order});
  if (it != g_kind.end() && (it->second != 7 || zblocked_ok(precision, order, ko)))
    return it->second;
  return staged_kind(order, false);
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

// resident workgroups per CU of a kernel instance (its registers and LDS)
int per_cu(int precision, int kind, bool ko, bool par = false) {
  switch (kind) {
    case 0: return batch_per_cu<0>(precision, ko, par);
    case 2: return batch_per_cu<2>(precision, ko, par);
    case 3: return batch_per_cu<3>(precision, ko, par);
    case 4: return batch_per_cu<4>(precision, ko, par);
    case 5: return batch_per_cu<5>(precision, ko, par);
    case 6: return batch_per_cu<6>(precision, ko, par);
    case 7: return batch_per_cu<7>(precision, ko, par);
    default: return batch_per_cu<1>(precision, ko, par);
  }
}

// Persistent grid: as many workgroups as can be resident at once, so that
// none waits for a slot; a multiple of 8 (one share of the list per XCD).
int persistent_blocks(int precision, int kind, bool ko, bool par = false) {
  const int b = compute_units() * per_cu(precision, kind, ko, par);
  return std::max(kNumXcd, b / kNumXcd * kNumXcd);
}

// Performance model: predicted duration of one substage launch, in units of
// one wavefront evaluating the right-hand side on one plane of its lanes.
//  * Interior item (a tile of ltx * lty threads over tz planes):
//    ceil(ltx * lty / 64) waves x tz planes -- a ragged tile costs its whole
//    waves (wave quantisation) -- times a halo factor 1 + w x (points the
//    item reads per point it computes: its stencil neighbourhood), w = 0.02
//    for the staged kinds (every neighbourhood point is an HBM or L2 read
//    and an LDS store) and 0.005 for kind 0 (neighbours mostly hit L1/L2),
//    times a per-point cost of the kind: 2.6 for kind 0 (its point code,
//    fed from the caches, measured 2.6-3.6x slower than the staged one),
//    1 for the staged kinds.
//  * Ghost item: its points / 64 waves x 0.25 (closed-form evaluation and
//    stores, no stencils).
//  * Schedule: XCD x takes share x of the interior items and of the ghost
//    items, in list order.  Persistent instances: its grid / 8 workgroups
//    take every (grid / 8)-th item of the share (static).  One item per
//    workgroup: the hardware hands the share's items, in order, to
//    whichever of the XCD's grid / 8 resident slots frees first (greedy
//    list scheduling).
//  * Occupancy: grid = resident workgroups per CU (k) x CUs; the k
//    workgroups of a CU share it, so a launch lasts the largest
//    per-workgroup load x k / min(w, 2), w = k x (waves per SIMD of one
//    workgroup: 1 for 256 threads, 2 for the z-blocked kind's 512) --
//    latency hiding saturates at two waves per SIMD.
// halo factor times the kind's per-point cost
double halo_factor(int kind, const Tile& t, int order) {
  const double pts = (double)t.ltx * t.lty * t.tz;
  const int r = order / 2 + 1;  // reach of the lopsided advection stencils
  double reads;
  if (kind == 0)
    reads = (t.ltx + 2.0 * r) * (t.lty + 2.0 * r) * (t.tz + 2.0 * r);
  else if (kind == 7)  // planes -2 .. tz+1 with halo, the two outer planes without
    reads = (t.tz + 4.0) * (t.ltx + 2.0 * r) * (t.lty + 2.0 * r) + 2.0 * t.ltx * t.lty;
  else
    reads = (t.ltx + 2.0 * r) * (t.lty + 2.0 * r) + 2.0 * (r - 1) * (t.ltx + 2.0 * r - 2) *
            (t.lty + 2.0 * r - 2) + 2.0 * t.ltx * t.lty;
  return kind == 0 ? 2.6 * (1.0 + 0.005 * reads / pts) : 1.0 + 0.02 * reads / pts;
}

struct ModelPatch {
  int32_t n[3];
  long long ghosts;
};

long long ghost_points(const Geo& G) {
  const long long e0 = G.n[0] + 2 * G.g, e1 = G.n[1] + 2 * G.g;
  return 2LL * G.g * e1 * e0 + (long long)G.n[2] * 2 * G.g * e0 +
         (long long)G.n[2] * G.n[1] * 2 * G.g;
}

// work-list order of patches: decreasing size (LPT), stable
std::vector<int> list_order(const std::vector<ModelPatch>& ps) {
  std::vector<int> order(ps.size());
  for (size_t q = 0; q < ps.size(); ++q) order[q] = (int)q;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (long long)ps[a].n[0] * ps[a].n[1] * ps[a].n[2] >
           (long long)ps[b].n[0] * ps[b].n[1] * ps[b].n[2];
  });
  return order;
}

double model_time(const std::vector<ModelPatch>& ps, const std::vector<Tile>& tiles, int kind,
                  int order, int k_per_cu, int grid, bool ghosts, bool dynamic) {
  std::vector<double> items, gitems;
  for (int q : list_order(ps)) {
    const Tile& t = tiles[q];
    const long long nt = (long long)((ps[q].n[0] + t.ltx - 1) / t.ltx) *
                         ((ps[q].n[1] + t.lty - 1) / t.lty) * ((ps[q].n[2] + t.tz - 1) / t.tz);
    const double c = std::ceil(t.ltx * t.lty / 64.0) * t.tz * halo_factor(kind, t, order);
    items.insert(items.end(), (size_t)nt, c);
    if (ghosts)
      for (long long g = 0; g < ps[q].ghosts; g += kGhostChunk)
        gitems.push_back(0.25 * std::min<long long>(kGhostChunk, ps[q].ghosts - g) / 64.0);
  }
  const long long ni = (long long)items.size(), ng = (long long)gitems.size();
  const int R = std::max(1, grid / kNumXcd);
  double worst = 0.0;
  std::vector<double> load(R);
  for (int x = 0; x < kNumXcd; ++x) {
    std::fill(load.begin(), load.end(), 0.0);
    const long long i0 = ni * x / kNumXcd, i1 = ni * (x + 1) / kNumXcd;
    const long long g0 = ng * x / kNumXcd, g1 = ng * (x + 1) / kNumXcd;
    const long long share = (i1 - i0) + (g1 - g0);
    for (long long t = 0; t < share; ++t) {
      const double c = t < i1 - i0 ? items[i0 + t] : gitems[g0 + t - (i1 - i0)];
      if (dynamic)  // the slot that frees first takes the next item
        *std::min_element(load.begin(), load.end()) += c;
      else
        load[t % R] += c;
    }
    for (double l : load) worst = std::max(worst, l);
  }
  const double w = k_per_cu * (kind == 7 ? 2.0 : 1.0);
  return worst * k_per_cu / std::min(w, 2.0);
}

// model-best kind 0 tile of one patch with one plane per item (untuned
// default: the most parallelism)
Tile model_tile(const int32_t n[3]) {
  Tile best = kCandidates[0];
  double bc = 1e300;
  for (const Tile& t : kCandidates) {
    if (t.tz != 1) continue;
    const double c = std::ceil(n[0] / (double)t.ltx) * t.ltx * std::ceil(n[1] / (double)t.lty) *
                     t.lty * halo_factor(0, t, 4);
    if (c < bc) {
      bc = c;
      best = t;
    }
  }
  return best;
}

// tile of one patch in a plan of the given kind
Tile kind_tile(int kind, int precision, const int32_t n[3]) {
  if (kind != 0) return kind_shape(kind);
  {
    std::lock_guard<std::mutex> lk(g_table_mu);
    auto it = g_table.find({precision, size_class(n)});
    if (it != g_table.end()) return it->second;
  }
  return model_tile(n);
}

// ---- plans --------------------------------------------------------------------

struct Plan {
  std::vector<chemora_parent> parents;  // one per patch (coarse NULL: analytic ghosts)
  std::vector<int> poff;                // 3 per patch: fine offset in its parent
  std::vector<const chemora_grid*> grids;
  std::vector<double*> states;
  std::vector<void*> wss;
  std::vector<Tile> tiles;
  double dt = 0.0;
  int precision = 0;
  int kind = 0;
  bool ko = false;  // some patch has Kreiss-Oliger dissipation
  bool has_parents = false;  // some patch's ghosts are prolongated from a parent
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

// Build descriptors and the work list with the given tile per patch, upload
// to meta (synchronously).
int build_plan(Plan* P, const chemora_patch* patches, int32_t np, void* meta, double dt,
               int precision, int kind, const std::vector<Tile>& tiles,
               const chemora_parent* parents = nullptr, const int* poff = nullptr) {
  P->np = np;
  P->parents.assign(np, chemora_parent{});
  P->poff.assign(3 * (size_t)np, 0);
  P->has_parents = false;
  if (parents)
    for (int q = 0; q < np; ++q) {
      P->parents[q] = parents[q];
      P->has_parents = P->has_parents || parents[q].coarse;
      for (int d = 0; d < 3; ++d) P->poff[3 * q + d] = poff[3 * q + d];
    }
  P->dt = dt;
  P->precision = precision;
  P->kind = kind;
  P->ko = false;
  for (int q = 0; q < np; ++q) P->ko = P->ko || grid_par(patches[q].grid).ko_sigma != 0.0;
  P->grids.resize(np);
  P->states.resize(np);
  P->wss.resize(np);
  P->tiles = tiles;
  std::vector<PatchDesc> pd(np);
  std::vector<ModelPatch> mp(np);
  for (int q = 0; q < np; ++q) {
    const chemora_grid* g = patches[q].grid;
    P->grids[q] = g;
    P->states[q] = patches[q].state;
    P->wss[q] = patches[q].workspace;
    const Geo& G = grid_geo(g);
    const Tile t = tiles[q];
    PatchDesc& d = pd[q];
    d.G = G;
    d.P = grid_par(g);
    d.W = make_weights(d.P.h, d.P.ko_sigma, d.P.fd_order);
    d.state_off = reinterpret_cast<char*>(patches[q].state) - reinterpret_cast<char*>(patches[0].state);
    d.ws_off = static_cast<char*>(patches[q].workspace) - reinterpret_cast<char*>(patches[0].state);
    d.E = grid_state_elems(g);
    d.ghosts = ghost_points(G);
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
    d.parent = 0;
    const chemora_parent& par = P->parents[q];
    if (par.coarse) {
      d.parent = 1;
      d.PC = grid_geo(par.coarse);
      for (int a = 0; a < 3; ++a) d.poff[a] = P->poff[3 * q + a];
      d.pb = make_box_grid(G, kBatchProlongBox, kBatchProlongBox, kBatchProlongBox,
                           kBatchProlongBox, kBatchProlongBox);
      d.pntimes = par.ntimes;
      for (int l = 0; l < kMaxTimeLevels; ++l) {
        const int ll = l < par.ntimes ? l : 0;  // unused levels repeat level 0
        d.plev[l] = reinterpret_cast<const char*>(par.levels[ll]) -
                    reinterpret_cast<char*>(patches[0].state);
        d.ptimes[l] = par.times[ll];
      }
    }
    mp[q] = ModelPatch{{G.n[0], G.n[1], G.n[2]}, d.ghosts};
  }
  // work-list order: patches by decreasing size (LPT), so the biggest tiles
  // are handed out first and the short ones fill the tail
  const std::vector<int> order = list_order(mp);
  std::vector<PatchDesc> pds(np);
  std::vector<long long> prefix(np + 1), gprefix(np + 1);
  prefix[0] = gprefix[0] = 0;
  for (int r = 0; r < np; ++r) {
    pds[r] = pd[order[r]];
    const PatchDesc& d = pds[r];
    prefix[r + 1] = prefix[r] + (long long)d.tiles[0] * d.tiles[1] * d.tiles[2];
    gprefix[r + 1] = gprefix[r] + (d.parent ? (long long)d.pb.boxes
                                            : (d.ghosts + kGhostChunk - 1) / kGhostChunk);
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
  if (batch_persistent_host(precision, kind)) {
    P->grid_blocks = persistent_blocks(precision, kind, P->ko, P->has_parents);
  } else {  // one workgroup per item of the largest XCD share
    const long long ng = P->n_total - P->n_interior;
    const long long per = (P->n_interior + kNumXcd - 1) / kNumXcd + (ng + kNumXcd - 1) / kNumXcd;
    if (per * kNumXcd > 0x7fffffffLL) return fail(CHEMORA_ERR_INVALID, "batch too large");
    P->grid_blocks = (int)std::max<long long>(kNumXcd, per * kNumXcd);
  }
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

std::vector<Tile> kind_tiles(int kind, int precision, const chemora_patch* patches, int32_t np) {
  std::vector<Tile> tiles(np);
  for (int q = 0; q < np; ++q) {
    const Geo& G = grid_geo(patches[q].grid);
    const int32_t n[3] = {G.n[0], G.n[1], G.n[2]};
    tiles[q] = kind_tile(kind, precision, n);
  }
  return tiles;
}

hipError_t launch_any(const Plan* P, int s, hipStream_t st) {
  const Batch& b = P->batch[s];
  const unsigned g = (unsigned)P->grid_blocks;
  const bool par = P->has_parents;
  switch (P->kind) {
    case 0: return launch_batch_kind<0>(P->precision, P->ko, par, s, b, g, st);
    case 2: return launch_batch_kind<2>(P->precision, P->ko, par, s, b, g, st);
    case 3: return launch_batch_kind<3>(P->precision, P->ko, par, s, b, g, st);
    case 4: return launch_batch_kind<4>(P->precision, P->ko, par, s, b, g, st);
    case 5: return launch_batch_kind<5>(P->precision, P->ko, par, s, b, g, st);
    case 6: return launch_batch_kind<6>(P->precision, P->ko, par, s, b, g, st);
    case 7: return launch_batch_kind<7>(P->precision, P->ko, par, s, b, g, st);
    default: return launch_batch_kind<1>(P->precision, P->ko, par, s, b, g, st);
  }
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

// Time three launches of the second substage of a plan (what a step runs:
// stencils, the RK update and the ghost items; it reads the first stage
// buffer and the state and writes only the workspace, so the patches' states
// are untouched), after a right-hand-side launch that fills the first stage
// buffer and a warm-up launch.  The clock is set to 0 for the ghost items.
int time_plan(const Plan* P, hipEvent_t e0, hipEvent_t e1, float* ms) {
  hipLaunchKernelGGL(set_clock_kernel, dim3(1), dim3(1), 0, nullptr, P->batch[2].clock, 0.0);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_any(P, 0, nullptr);
  if (e == hipSuccess) e = launch_any(P, 2, nullptr);
  if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
  for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch_any(P, 2, nullptr);
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  return device_status(e, "autotune trial");
}

bool same_parent(const chemora_parent& a, const chemora_parent* b) {
  const bool bn = !b || !b->coarse;
  if (!a.coarse || bn) return !a.coarse && bn;
  if (a.coarse != b->coarse || a.ntimes != b->ntimes) return false;
  for (int l = 0; l < a.ntimes; ++l)
    if (a.levels[l] != b->levels[l] || a.times[l] != b->times[l]) return false;
  return true;
}

bool same_patches(const Plan* P, const chemora_patch* patches, int32_t np, double dt,
                  const chemora_parent* parents) {
  if (P->np != np || P->dt != dt) return false;
  for (int q = 0; q < np; ++q)
    if (P->grids[q] != patches[q].grid || P->states[q] != patches[q].state ||
        P->wss[q] != patches[q].workspace || !same_parent(P->parents[q], parents ? &parents[q] : nullptr))
      return false;
  return true;
}

// Parents of a two-level batch: each either none (coarse NULL) or a valid
// prolongation source for its patch (chemora_prolong's checks), 4th order,
// ghost boxes within the kernel's LDS, time levels that no patch of the
// batch writes.  Fills off (3 per patch).
int validate_parents(const chemora_patch* patches, const chemora_parent* parents, int32_t np,
                     int order, int* off) {
  for (int q = 0; q < np; ++q) {
    for (int d = 0; d < 3; ++d) off[3 * q + d] = 0;
    const chemora_parent& par = parents[q];
    if (!par.coarse) continue;
    if (order != 4)
      return fail(CHEMORA_ERR_UNSUPPORTED,
                  "patch %d: prolongated ghosts need fd_order 4 (the staged high-order kinds "
                  "have no room for the prolongation boxes)", q);
    const Geo& G = grid_geo(patches[q].grid);
    const BoxGrid bg = make_box_grid(G, kBatchProlongBox, kBatchProlongBox, kBatchProlongBox,
                                     kBatchProlongBox, kBatchProlongBox);
    if (bg.lds_a > kBatchProlongLds || bg.lds_b > kBatchProlongLds || bg.boxes < 1)
      return fail(CHEMORA_ERR_UNSUPPORTED,
                  "patch %d: prolongated ghosts need a ghost width of at most 5, got %d", q, G.g);
    if (grid_nvars(par.coarse) != 24)
      return fail(CHEMORA_ERR_INVALID, "patch %d: the parent must be a BSSN grid", q);
    const int st = check_prolong_source(par.coarse, patches[q].grid, par.levels, par.times,
                                        par.ntimes, patches[q].state,
                                        grid_state_elems(patches[q].grid) * 8, &off[3 * q]);
    if (st != CHEMORA_OK) return st;
    const long long cb = grid_state_elems(par.coarse) * 8;
    for (int r = 0; r < np; ++r) {
      const long long sb = grid_state_elems(patches[r].grid) * 8;
      for (int l = 0; l < par.ntimes; ++l) {
        const char* a = reinterpret_cast<const char*>(par.levels[l]);
        const char* st0 = reinterpret_cast<const char*>(patches[r].state);
        const char* w0 = static_cast<const char*>(patches[r].workspace);
        if ((a < st0 + sb && st0 < a + cb) || (a < w0 + 3 * sb && w0 < a + cb))
          return fail(CHEMORA_ERR_INVALID,
                      "patch %d: parent time level %d overlaps the state or workspace of patch "
                      "%d, which the batch writes", q, l, r);
      }
    }
  }
  return CHEMORA_OK;
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

int chemora_batch_step_levels(const chemora_patch* patches, const chemora_parent* parents,
                              int32_t npatches, void* meta, double t, double dt, int32_t nsteps,
                              chemora_stream stream) {
  int precision = 0, order = 4;
  int st = validate_patches(patches, npatches, &precision, &order);
  if (st != CHEMORA_OK) return st;
  if (!meta || !aligned(meta)) return fail(CHEMORA_ERR_INVALID, "meta must be a 256-byte aligned device pointer");
  if (nsteps < 0) return fail(CHEMORA_ERR_INVALID, "nsteps must be >= 0");
  if (!std::isfinite(t) || !std::isfinite(dt)) return fail(CHEMORA_ERR_INVALID, "t and dt must be finite");
  std::vector<int> off(3 * (size_t)npatches, 0);
  bool any_parent = false;
  if (parents) {
    st = validate_parents(patches, parents, npatches, order, off.data());
    if (st != CHEMORA_OK) return st;
    for (int q = 0; q < npatches; ++q) any_parent = any_parent || parents[q].coarse;
  }
  const chemora_parent* par = any_parent ? parents : nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Plan* P = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(meta);
    if (it != g_plans.end() && same_patches(it->second, patches, npatches, dt, par) &&
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
      bool ko = false;
      for (int q = 0; q < npatches; ++q) ko = ko || grid_par(patches[q].grid).ko_sigma != 0.0;
      const int kind = plan_kind(precision, order, ko);
      st = build_plan(P, patches, npatches, meta, dt, precision, kind,
                      kind_tiles(kind, precision, patches, npatches), par, off.data());
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
  // the states' ghosts of the patches with a parent: prolongated at t
  for (int q = 0; q < npatches && par; ++q) {
    const chemora_parent& pr = par[q];
    if (!pr.coarse) continue;
    double wt[kMaxTimeLevels];
    time_weights(pr.times, pr.ntimes, t, wt);
    st = device_status(launch_prolong(grid_geo(pr.coarse), pr.levels, wt, pr.ntimes,
                                      grid_geo(patches[q].grid), &off[3 * q], 24,
                                      patches[q].state, s),
                       "batch parent prolongation");
    if (st != CHEMORA_OK) return st;
  }
  for (int n = 0; n < nsteps; ++n) {
    st = device_status(hipGraphLaunch(P->exec, s), "batch graph launch");
    if (st != CHEMORA_OK) return st;
  }
  return CHEMORA_OK;
}

int chemora_batch_step(const chemora_patch* patches, int32_t npatches, void* meta, double t,
                       double dt, int32_t nsteps, chemora_stream stream) {
  return chemora_batch_step_levels(patches, nullptr, npatches, meta, t, dt, nsteps, stream);
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
  const Tile t = kind_tile(plan_kind(precision, 4, false), precision, n);
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
  bool ko = false;
  for (int q = 0; q < npatches; ++q) ko = ko || grid_par(patches[q].grid).ko_sigma != 0.0;
  std::vector<ModelPatch> all;
  for (int q = 0; q < npatches; ++q) {
    const Geo& G = grid_geo(patches[q].grid);
    all.push_back(ModelPatch{{G.n[0], G.n[1], G.n[2]}, ghost_points(G)});
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(CHEMORA_ERR_DEVICE, "event creation failed");
  std::string json = "{\n";
  char buf[512];
  // kind 0 (4th order): its tile per size class -- the model ranks the
  // candidates over the class's patches, the best three are timed
  if (order == 4) {
    std::map<int, std::vector<chemora_patch>> classes;
    std::map<int, std::vector<ModelPatch>> cmodel;
    for (int q = 0; q < npatches; ++q) {
      const int c = size_class(all[q].n);
      classes[c].push_back(patches[q]);
      cmodel[c].push_back(all[q]);
    }
    const int k = per_cu(precision, 0, ko), grid = persistent_blocks(precision, 0, ko);
    for (auto& kv : classes) {
      const std::vector<chemora_patch>& ps = kv.second;
      std::vector<std::pair<double, Tile>> scored;
      for (const Tile& t : kCandidates)
        scored.push_back({model_time(cmodel[kv.first], std::vector<Tile>(ps.size(), t), 0, order,
                                     k, grid, false, !batch_persistent_host(precision, 0)),
                          t});
      std::stable_sort(scored.begin(), scored.end(),
                       [](const std::pair<double, Tile>& a, const std::pair<double, Tile>& b) {
                         return a.first < b.first;
                       });
      Tile best = scored[0].second;
      float best_ms = 1e30f;
      std::string trials;
      for (size_t c = 0; c < scored.size() && c < 3; ++c) {
        Plan P;
        st = build_plan(&P, ps.data(), (int)ps.size(), meta, 0.0, precision, 0,
                        std::vector<Tile>(ps.size(), scored[c].second));
        float ms = 0.f;
        if (st == CHEMORA_OK) st = time_plan(&P, e0, e1, &ms);
        if (st != CHEMORA_OK) break;
        snprintf(buf, sizeof buf,
                 "%s{\"tile\": [%d, %d, %d], \"model\": %.1f, \"ms_per_substage\": %.5f}", c ? ", " : "",
                 scored[c].second.ltx, scored[c].second.lty, scored[c].second.tz, scored[c].first,
                 ms / 3.0);
        trials += buf;
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
      snprintf(buf, sizeof buf,
               "  \"precision%d_kind0_class%d\": {\"tile\": [%d, %d, %d], \"patches\": %zu, "
               "\"trials\": [",
               precision, kv.first, best.ltx, best.lty, best.tz, ps.size());
      json += buf;
      json += trials + "]},\n";
    }
  }
  // the candidate kinds of the order over the whole batch: model prediction
  // and measured time; the untuned default is the 32x8 staged kind
  std::vector<int> kinds = {staged_kind(order, false), staged_kind(order, true)};
  if (order == 4) kinds.insert(kinds.begin(), 0);
  if (zblocked_ok(precision, order, ko)) kinds.push_back(7);
  std::map<int, float> kind_ms;
  std::string ks;
  for (int kind : kinds) {
    if (st != CHEMORA_OK) break;
    const std::vector<Tile> tiles = kind_tiles(kind, precision, patches, npatches);
    const double model = model_time(all, tiles, kind, order, per_cu(precision, kind, ko),
                                    persistent_blocks(precision, kind, ko), false,
                                    !batch_persistent_host(precision, kind));
    Plan P;
    st = build_plan(&P, patches, npatches, meta, 0.0, precision, kind, tiles);
    float ms = 0.f;
    if (st == CHEMORA_OK) st = time_plan(&P, e0, e1, &ms);
    kind_ms[kind] = ms;
    snprintf(buf, sizeof buf, "%s\"%d\": {\"model\": %.1f, \"per_cu\": %d, \"ms_per_substage\": %.5f}",
             ks.empty() ? "" : ", ", kind, model, per_cu(precision, kind, ko), ms / 3.0);
    ks += buf;
  }
  if (st == CHEMORA_OK) {
    int best_kind = kinds[0];
    for (int kind : kinds)
      if (kind_ms[kind] < kind_ms[best_kind]) best_kind = kind;
    {
      std::lock_guard<std::mutex> lk(g_table_mu);
      g_kind[{precision, order}] = best_kind;
    }
    snprintf(buf, sizeof buf,
             "  \"precision%d_order%d_kind\": {\"kind\": %d, \"untuned_kind\": %d, "
             "\"tuned_ms_per_substage\": %.5f, \"untuned_ms_per_substage\": %.5f, \"kinds\": {",
             precision, order, best_kind, staged_kind(order, false), kind_ms[best_kind] / 3.0,
             kind_ms[staged_kind(order, false)] / 3.0);
    json += buf;
    json += ks + "}}";
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

int chemora_batch_model(const int32_t* dims, const int32_t* tiles, int32_t npatches,
                        int32_t kind, int32_t fd_order, int32_t per_cu_wg, int32_t grid,
                        int32_t ghost_width, int32_t per_item, double* out) {
  if (!dims || !tiles || !out) return fail(CHEMORA_ERR_INVALID, "NULL argument");
  if (npatches < 1 || npatches > kMaxPatches)
    return fail(CHEMORA_ERR_INVALID, "npatches must be in [1, %d]", kMaxPatches);
  if (kind < 0 || kind >= kNumKinds) return fail(CHEMORA_ERR_INVALID, "kind must be in [0, 7]");
  if (fd_order != 4 && fd_order != 6 && fd_order != 8)
    return fail(CHEMORA_ERR_INVALID, "fd_order must be 4, 6 or 8");
  if (per_cu_wg < 1 || grid < 1 || ghost_width < 0)
    return fail(CHEMORA_ERR_INVALID, "per_cu and grid must be >= 1, ghost_width >= 0");
  std::vector<ModelPatch> ps(npatches);
  std::vector<Tile> ts(npatches);
  for (int q = 0; q < npatches; ++q) {
    for (int d = 0; d < 3; ++d)
      if (dims[3 * q + d] < 1 || tiles[3 * q + d] < 1)
        return fail(CHEMORA_ERR_INVALID, "patch %d: sizes and tile extents must be >= 1", q);
    Geo G{};
    for (int d = 0; d < 3; ++d) G.n[d] = dims[3 * q + d];
    G.g = ghost_width;
    ps[q] = ModelPatch{{dims[3 * q], dims[3 * q + 1], dims[3 * q + 2]},
                       ghost_width > 0 ? ghost_points(G) : 0};
    ts[q] = Tile{tiles[3 * q], tiles[3 * q + 1], tiles[3 * q + 2]};
  }
  *out = model_time(ps, ts, kind, fd_order, per_cu_wg, grid, ghost_width > 0, per_item != 0);
  return CHEMORA_OK;
}

}  // extern "C"
