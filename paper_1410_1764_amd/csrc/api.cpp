// api.cpp -- the C ABI of libchemora (declared in include/chemora.h): grid
// objects, argument validation, the RK4 driver and error reporting.  Host
// code only; every kernel launch goes through the launchers in internal.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "prolong_box.h"

using namespace chemora;

struct chemora_grid {
  chemora_grid_desc d;
  Geo geo;
  BssnPar par;
  int nvars;
  long long state_elems;
};

namespace chemora {

static thread_local std::string g_err = "no error";

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return status;
}

int device_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return CHEMORA_OK;
  return fail(CHEMORA_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

const Geo& grid_geo(const chemora_grid* g) { return g->geo; }
const BssnPar& grid_par(const chemora_grid* g) { return g->par; }
const chemora_grid_desc& grid_desc(const chemora_grid* g) { return g->d; }
long long grid_state_elems(const chemora_grid* g) { return g->state_elems; }
int grid_nvars(const chemora_grid* g) { return g->nvars; }

// constraints.hip: the static partial-sum buffer of chemora_constraints_noalloc
long long constraints_static_capacity();
hipError_t constraints_static_partials(double** out);
// probe.hip: the FMA throughput probe
long long probe_fma_threads();
hipError_t launch_probe_fma(int precision, void* out, int iters, double* flops, hipStream_t s);

}  // namespace chemora

namespace {

int validate_desc(const chemora_grid_desc* d) {
  if (!d) return fail(CHEMORA_ERR_INVALID, "grid description is NULL");
  if (d->system != CHEMORA_WAVE && d->system != CHEMORA_BSSN && d->system != CHEMORA_WAVE5)
    return fail(CHEMORA_ERR_INVALID,
                "system must be CHEMORA_WAVE (1), CHEMORA_BSSN (2) or CHEMORA_WAVE5 (3), got %d",
                d->system);
  const int gmin = d->system == CHEMORA_BSSN ? 3 : 2;
  if (d->ghost < gmin || d->ghost > kMaxGhost)
    return fail(CHEMORA_ERR_INVALID, "ghost must be in [%d, %d] for this system, got %d", gmin,
                kMaxGhost, d->ghost);
  for (int a = 0; a < 3; ++a) {
    if (d->n[a] < 1) return fail(CHEMORA_ERR_INVALID, "n[%d] must be >= 1, got %d", a, d->n[a]);
    if (!(d->h[a] > 0.0) || !std::isfinite(d->h[a]))
      return fail(CHEMORA_ERR_INVALID, "h[%d] must be finite and > 0", a);
    if (!std::isfinite(d->origin[a]))
      return fail(CHEMORA_ERR_INVALID, "origin[%d] must be finite", a);
  }
  if (d->precision != CHEMORA_FP64 && d->precision != CHEMORA_MIXED)
    return fail(CHEMORA_ERR_INVALID, "precision must be CHEMORA_FP64 or CHEMORA_MIXED, got %d",
                d->precision);
  if (d->boundary < CHEMORA_BC_PERIODIC || d->boundary > CHEMORA_BC_CALLER)
    return fail(CHEMORA_ERR_INVALID, "unknown boundary %d", d->boundary);
  if (d->boundary == CHEMORA_BC_PERIODIC)
    for (int a = 0; a < 3; ++a)
      if (d->n[a] < d->ghost)
        return fail(CHEMORA_ERR_INVALID,
                    "periodic boundary needs n[%d] >= ghost (%d < %d): images would overlap",
                    a, d->n[a], d->ghost);
  if (d->boundary == CHEMORA_BC_GAUGEWAVE) {
    if (d->system != CHEMORA_BSSN)
      return fail(CHEMORA_ERR_INVALID, "the gauge-wave boundary needs the BSSN system");
    if (!(std::fabs(d->gw_amp) < 1.0))
      return fail(CHEMORA_ERR_INVALID, "gauge wave amplitude must satisfy |A| < 1");
    if (!(d->gw_wavelength > 0.0) || !std::isfinite(d->gw_wavelength))
      return fail(CHEMORA_ERR_INVALID, "gauge wave wavelength must be finite and > 0");
    if (d->gw_axis < 0 || d->gw_axis > 2)
      return fail(CHEMORA_ERR_INVALID, "gauge wave axis must be 0, 1 or 2");
  }
  if (d->system == CHEMORA_BSSN) {
    if (d->slicing != CHEMORA_SLICING_1PLUSLOG && d->slicing != CHEMORA_SLICING_HARMONIC)
      return fail(CHEMORA_ERR_INVALID, "unknown slicing %d", d->slicing);
    if (d->shift != CHEMORA_SHIFT_FROZEN && d->shift != CHEMORA_SHIFT_GAMMADRIVER)
      return fail(CHEMORA_ERR_INVALID, "unknown shift condition %d", d->shift);
    if (!std::isfinite(d->shift_F) || !std::isfinite(d->eta))
      return fail(CHEMORA_ERR_INVALID, "shift_F and eta must be finite");
  }
  if (d->enforce != 0 && d->enforce != 1) return fail(CHEMORA_ERR_INVALID, "enforce must be 0 or 1");
  if (!std::isfinite(d->ko_sigma) || d->ko_sigma < 0.0)
    return fail(CHEMORA_ERR_INVALID, "ko_sigma must be finite and >= 0");
  if (d->system != CHEMORA_BSSN && (d->enforce != 0 || d->ko_sigma != 0.0))
    return fail(CHEMORA_ERR_INVALID, "enforce and ko_sigma apply to the BSSN system only");
  if (d->fd_order != 0 && d->fd_order != 4 && d->fd_order != 6 && d->fd_order != 8)
    return fail(CHEMORA_ERR_INVALID, "fd_order must be 0, 4, 6 or 8, got %d", d->fd_order);
  {
    const int order = d->fd_order == 0 ? 4 : d->fd_order;
    if (order != 4 && d->system != CHEMORA_BSSN)
      return fail(CHEMORA_ERR_INVALID, "fd_order 6 and 8 apply to the BSSN system only");
    if (d->system == CHEMORA_BSSN && d->ghost < order / 2 + 1)
      return fail(CHEMORA_ERR_INVALID, "fd_order %d needs ghost >= %d, got %d", order,
                  order / 2 + 1, d->ghost);
    if (order != 4 && d->ko_sigma != 0.0)
      return fail(CHEMORA_ERR_INVALID, "ko_sigma needs fd_order 4");
  }
  // element strides of a grid function must fit in 32 bits
  const long long e0 = d->n[0] + 2LL * d->ghost, e1 = d->n[1] + 2LL * d->ghost;
  const long long e2 = d->n[2] + 2LL * d->ghost;
  const long long sy = ((kAlign + d->n[0] + d->ghost + 1 + kAlign - 1) / kAlign) * kAlign;
  // one grid function must be addressable with 32-bit element offsets
  if (sy * e1 * e2 > (1LL << 31) - 1 || e0 <= 0)
    return fail(CHEMORA_ERR_INVALID, "grid too large: one grid function exceeds 2^31 elements");
  return CHEMORA_OK;
}

}  // namespace

extern "C" {

const char* chemora_last_error(void) { return g_err.c_str(); }

int chemora_grid_create(const chemora_grid_desc* desc, chemora_grid** out) {
  if (!out) return fail(CHEMORA_ERR_INVALID, "out pointer is NULL");
  *out = nullptr;
  int st = validate_desc(desc);
  if (st != CHEMORA_OK) return st;
  chemora_grid* g = new (std::nothrow) chemora_grid;
  if (!g) return fail(CHEMORA_ERR_HOST_NOMEM, "host allocation failed");
  g->d = *desc;
  const int gh = desc->ghost;
  Geo& G = g->geo;
  for (int a = 0; a < 3; ++a) G.n[a] = desc->n[a];
  G.g = gh;
  // row: [pad | ghost | interior (starts at column kAlign) | ghost | pad >= 1]
  // (the pad column lets 16-byte copies start at the last ghost column)
  G.sy = (int)(((kAlign + desc->n[0] + gh + 1 + kAlign - 1) / kAlign) * kAlign);
  G.sz = G.sy * (desc->n[1] + 2 * gh);
  G.sv = (long long)G.sz * (desc->n[2] + 2 * gh);
  G.off0 = kAlign + (long long)gh * G.sy + (long long)gh * G.sz;
  g->nvars = desc->system == CHEMORA_WAVE ? 2 : (desc->system == CHEMORA_WAVE5 ? 5 : 24);
  g->state_elems = G.sv * g->nvars;
  BssnPar& P = g->par;
  for (int a = 0; a < 3; ++a) {
    P.h[a] = desc->h[a];
    P.origin[a] = desc->origin[a];
  }
  P.slicing = desc->slicing;
  P.shift = desc->shift;
  P.F = desc->shift_F;
  P.eta = desc->eta;
  P.gw_A = desc->gw_amp;
  P.gw_d = desc->gw_wavelength;
  P.gw_axis = desc->gw_axis;
  P.enforce = desc->enforce;
  P.ko_sigma = desc->ko_sigma;
  P.fd_order = desc->fd_order == 0 ? 4 : desc->fd_order;
  *out = g;
  return CHEMORA_OK;
}

int chemora_grid_destroy(chemora_grid* grid) {
  delete grid;
  return CHEMORA_OK;
}

int chemora_grid_layout(const chemora_grid* grid, int32_t* nvars, int64_t strides[4],
                        int64_t* interior_offset, int64_t* state_elems) {
  if (!grid) return fail(CHEMORA_ERR_INVALID, "grid is NULL");
  if (nvars) *nvars = grid->nvars;
  if (strides) {
    strides[0] = 1;
    strides[1] = grid->geo.sy;
    strides[2] = grid->geo.sz;
    strides[3] = grid->geo.sv;
  }
  if (interior_offset) *interior_offset = grid->geo.off0;
  if (state_elems) *state_elems = grid->state_elems;
  return CHEMORA_OK;
}

int64_t chemora_workspace_bytes(const chemora_grid* grid) {
  if (!grid) {
    fail(CHEMORA_ERR_INVALID, "grid is NULL");
    return -1;
  }
  return 3LL * grid->state_elems * (int64_t)sizeof(double);
}

int chemora_fill_ghosts(chemora_grid* grid, double* state, double t, chemora_stream stream) {
  if (!grid) return fail(CHEMORA_ERR_INVALID, "grid is NULL");
  if (!state) return fail(CHEMORA_ERR_INVALID, "state is NULL");
  if (!aligned(state)) return fail(CHEMORA_ERR_INVALID, "state must be 256-byte aligned");
  if (!std::isfinite(t)) return fail(CHEMORA_ERR_INVALID, "t must be finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  switch (grid->d.boundary) {
    case CHEMORA_BC_PERIODIC:
      return device_status(launch_fill_periodic(grid->geo, grid->nvars, state, s),
                           "periodic ghost fill");
    case CHEMORA_BC_GAUGEWAVE:
      return device_status(launch_fill_gaugewave(grid->geo, grid->par, t, state, s),
                           "gauge-wave ghost fill");
    default:
      return CHEMORA_OK;
  }
}

// read at every chemora_rk4_step call, like the other ablation switches
static bool periodic_images() {
  const char* e = std::getenv("CHEMORA_PERIODIC");
  return e && std::strcmp(e, "images") == 0;
}

static hipError_t launch_stage(const chemora_grid* g, int stage, bool images, const StageIO& io,
                               hipStream_t s) {
  if (g->d.system == CHEMORA_WAVE)
    return launch_wave_stage(g->geo, g->d.h, stage, g->d.precision, images, io, s);
  if (g->d.system == CHEMORA_WAVE5)
    return launch_wave5_stage(g->geo, g->d.h, stage, g->d.precision, images, io, s);
  return launch_bssn_stage(g->geo, g->par, stage, g->d.precision, images, io, s);
}

int chemora_rhs(chemora_grid* grid, const double* state, double* rhs, chemora_stream stream) {
  if (!grid) return fail(CHEMORA_ERR_INVALID, "grid is NULL");
  if (!state || !rhs) return fail(CHEMORA_ERR_INVALID, "state and rhs must not be NULL");
  if (!aligned(state) || !aligned(rhs))
    return fail(CHEMORA_ERR_INVALID, "state and rhs must be 256-byte aligned");
  const long long bytes = grid->state_elems * (long long)sizeof(double);
  const char* a = reinterpret_cast<const char*>(state);
  const char* b = reinterpret_cast<const char*>(rhs);
  if (a < b + bytes && b < a + bytes) return fail(CHEMORA_ERR_INVALID, "state and rhs overlap");
  StageIO io{state, state, nullptr, rhs, 0.0};
  return device_status(launch_stage(grid, 0, false, io, static_cast<hipStream_t>(stream)),
                       "right-hand-side launch");
}

int chemora_rk4_step(chemora_grid* grid, double* state, void* workspace, double t, double dt,
                     int32_t nsteps, chemora_stream stream) {
  if (!grid) return fail(CHEMORA_ERR_INVALID, "grid is NULL");
  if (!state || !workspace) return fail(CHEMORA_ERR_INVALID, "state and workspace must not be NULL");
  if (!aligned(state) || !aligned(workspace))
    return fail(CHEMORA_ERR_INVALID, "state and workspace must be 256-byte aligned");
  if (nsteps < 0) return fail(CHEMORA_ERR_INVALID, "nsteps must be >= 0");
  if (!std::isfinite(t) || !std::isfinite(dt)) return fail(CHEMORA_ERR_INVALID, "t and dt must be finite");
  if (grid->d.boundary == CHEMORA_BC_CALLER)
    return fail(CHEMORA_ERR_INVALID, "chemora_rk4_step needs a periodic or gauge-wave boundary");
  const long long E = grid->state_elems;
  double* B1 = static_cast<double*>(workspace);
  double* B2 = B1 + E;
  double* acc = B2 + E;
  {
    const char* a = reinterpret_cast<const char*>(state);
    const char* w = reinterpret_cast<const char*>(workspace);
    const long long sb = E * 8, wb = 3 * E * 8;
    if (a < w + wb && w < a + sb) return fail(CHEMORA_ERR_INVALID, "state and workspace overlap");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool periodic = grid->d.boundary == CHEMORA_BC_PERIODIC;
  // periodic ghosts: a separate fill of the stage output (default), or the
  // stage kernels writing every value to its images as well
  // (CHEMORA_PERIODIC=images, ablation switch).  The fill is the faster one:
  // image stores make most boundary tiles' waves branch and issue scattered
  // stores for all 24 grid functions.
  const bool images = periodic && periodic_images();
  int st = chemora_fill_ghosts(grid, state, t, stream);
  if (st != CHEMORA_OK) return st;
  const double cdt[5] = {0.0, 0.5 * dt, 0.5 * dt, dt, dt / 6.0};
  const double ct[5] = {0.0, 0.5, 0.5, 1.0, 1.0};  // time of each stage's output
  for (int n = 0; n < nsteps; ++n) {
    const double tn = t + n * dt;
    double* ins[5] = {nullptr, state, B1, B2, B1};
    double* outs[5] = {nullptr, B1, B2, B1, state};
    for (int stage = 1; stage <= 4; ++stage) {
      // the last stage writes the state itself, which it also reads
      // pointwise as y_n: B2, free by then, takes the split kernels'
      // intermediates
      StageIO io{ins[stage], state, acc, outs[stage], cdt[stage], stage == 4 ? B2 : nullptr};
      st = device_status(launch_stage(grid, stage, images, io, s), "RK4 substage launch");
      if (st != CHEMORA_OK) return st;
      if (periodic && !images) {
        st = device_status(launch_fill_periodic(grid->geo, grid->nvars, outs[stage], s),
                           "periodic ghost fill");
        if (st != CHEMORA_OK) return st;
      } else if (!periodic) {
        st = device_status(launch_fill_gaugewave(grid->geo, grid->par, tn + ct[stage] * dt,
                                                 outs[stage], s),
                           "gauge-wave ghost fill");
        if (st != CHEMORA_OK) return st;
      }
    }
  }
  return CHEMORA_OK;
}

int64_t chemora_constraints_workspace_bytes(const chemora_grid* grid) {
  if (!grid) {
    fail(CHEMORA_ERR_INVALID, "grid is NULL");
    return -1;
  }
  return constraints_partial_count(grid->geo, grid->par.fd_order) * (int64_t)sizeof(double);
}

int chemora_constraints(chemora_grid* grid, const double* state, double* hm, double* norms,
                        void* workspace, chemora_stream stream) {
  if (!grid) return fail(CHEMORA_ERR_INVALID, "grid is NULL");
  if (grid->d.system != CHEMORA_BSSN)
    return fail(CHEMORA_ERR_UNSUPPORTED, "constraints exist for the BSSN system only");
  if (!state || !norms || !workspace)
    return fail(CHEMORA_ERR_INVALID, "state, norms and workspace must not be NULL");
  if (!aligned(state) || !aligned(workspace) || (hm && !aligned(hm)) ||
      (reinterpret_cast<uintptr_t>(norms) & 7u))
    return fail(CHEMORA_ERR_INVALID, "misaligned pointer");
  return device_status(launch_bssn_constraints(grid->geo, grid->par, state, hm, norms,
                                               static_cast<double*>(workspace),
                                               static_cast<hipStream_t>(stream)),
                       "constraints launch");
}

int chemora_constraints_noalloc(chemora_grid* grid, const double* state, double* hm,
                                double* norms, chemora_stream stream) {
  if (!grid) return fail(CHEMORA_ERR_INVALID, "grid is NULL");
  if (grid->d.system != CHEMORA_BSSN)
    return fail(CHEMORA_ERR_UNSUPPORTED, "constraints exist for the BSSN system only");
  if (!state || !norms) return fail(CHEMORA_ERR_INVALID, "state and norms must not be NULL");
  if (!aligned(state) || (hm && !aligned(hm)) || (reinterpret_cast<uintptr_t>(norms) & 7u))
    return fail(CHEMORA_ERR_INVALID, "misaligned pointer");
  const long long need = constraints_partial_count(grid->geo, grid->par.fd_order);
  if (need > constraints_static_capacity())
    return fail(CHEMORA_ERR_INVALID,
                "grid needs %lld partial sums; the static buffer holds %lld (use "
                "chemora_constraints with a workspace)",
                need, constraints_static_capacity());
  double* partial = nullptr;
  const int st = device_status(constraints_static_partials(&partial), "static scratch lookup");
  if (st != CHEMORA_OK) return st;
  return device_status(launch_bssn_constraints(grid->geo, grid->par, state, hm, norms, partial,
                                               static_cast<hipStream_t>(stream)),
                       "constraints launch");
}

int64_t chemora_energy_workspace_bytes(const chemora_grid* grid) {
  if (!grid) {
    fail(CHEMORA_ERR_INVALID, "grid is NULL");
    return -1;
  }
  return energy_partial_count(grid->geo) * (int64_t)sizeof(double);
}

int chemora_energy(chemora_grid* grid, const double* state, double* eps, double* total,
                   void* workspace, chemora_stream stream) {
  if (!grid) return fail(CHEMORA_ERR_INVALID, "grid is NULL");
  if (grid->d.system != CHEMORA_WAVE5)
    return fail(CHEMORA_ERR_UNSUPPORTED, "the energy calculation exists for CHEMORA_WAVE5 only");
  if (!state || !total || !workspace)
    return fail(CHEMORA_ERR_INVALID, "state, total and workspace must not be NULL");
  if (!aligned(state) || !aligned(workspace) || (eps && !aligned(eps)) ||
      (reinterpret_cast<uintptr_t>(total) & 7u))
    return fail(CHEMORA_ERR_INVALID, "misaligned pointer");
  return device_status(launch_wave5_energy(grid->geo, grid->d.h, state, eps, total,
                                           static_cast<double*>(workspace),
                                           static_cast<hipStream_t>(stream)),
                       "energy launch");
}

int chemora_probe_copy(void* dst, const void* src, int64_t nbytes, chemora_stream stream) {
  if (!dst || !src) return fail(CHEMORA_ERR_INVALID, "dst and src must not be NULL");
  if (nbytes < 0 || (nbytes & 15)) return fail(CHEMORA_ERR_INVALID, "nbytes must be a multiple of 16");
  if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15u)
    return fail(CHEMORA_ERR_INVALID, "dst and src must be 16-byte aligned");
  return device_status(launch_probe_copy(dst, src, nbytes, static_cast<hipStream_t>(stream)),
                       "copy probe launch");
}

int64_t chemora_probe_fma_bytes(void) { return probe_fma_threads() * (int64_t)sizeof(double); }

int chemora_probe_fma(int32_t precision, void* out, int32_t iters, double* flops,
                      chemora_stream stream) {
  if (!out || !flops) return fail(CHEMORA_ERR_INVALID, "out and flops must not be NULL");
  if (!aligned(out)) return fail(CHEMORA_ERR_INVALID, "out must be 256-byte aligned");
  if (precision != CHEMORA_FP64 && precision != CHEMORA_MIXED)
    return fail(CHEMORA_ERR_INVALID, "precision must be CHEMORA_FP64 or CHEMORA_MIXED");
  if (iters < 1) return fail(CHEMORA_ERR_INVALID, "iters must be >= 1");
  return device_status(
      launch_probe_fma(precision, out, iters, flops, static_cast<hipStream_t>(stream)),
      "FMA probe launch");
}

// Two refinement levels: checks the pair and returns the fine origin's
// offset from the coarse origin in fine spacings.
static int level_pair(const chemora_grid* c, const chemora_grid* f, int off[3]) {
  if (!c || !f) return fail(CHEMORA_ERR_INVALID, "coarse and fine grids must not be NULL");
  if (c->d.system != f->d.system)
    return fail(CHEMORA_ERR_INVALID, "coarse and fine grids hold different systems");
  for (int a = 0; a < 3; ++a) {
    if (std::fabs(c->d.h[a] - 2.0 * f->d.h[a]) > 1e-12 * c->d.h[a])
      return fail(CHEMORA_ERR_INVALID, "h[%d]: coarse spacing must be twice the fine spacing", a);
    const double r = (f->d.origin[a] - c->d.origin[a]) / f->d.h[a];
    const double q = std::floor(r + 0.5);
    if (std::fabs(r - q) > 1e-9 || std::fabs(q) > 1e9)
      return fail(CHEMORA_ERR_INVALID,
                  "origin[%d]: the fine origin is not a whole number of fine spacings from the "
                  "coarse origin", a);
    off[a] = (int)q;
  }
  return CHEMORA_OK;
}

static bool overlaps(const void* a, long long an, const void* b, long long bn) {
  const char *x = static_cast<const char*>(a), *y = static_cast<const char*>(b);
  return x < y + bn && y < x + an;
}

}  // extern "C"

namespace chemora {

// Shared by chemora_prolong and the batch's prolongation ghosts: the level
// pair, the time levels (1..3 aligned states not overlapping [avoid, avoid +
// avoid_bytes), distinct finite times) and the reach of every fine extended
// point's stencil inside the coarse extended block.
int check_prolong_source(const chemora_grid* coarse, const chemora_grid* fine,
                         const double* const* levels, const double* times, int ntimes,
                         const void* avoid, long long avoid_bytes, int off[3]) {
  int st = level_pair(coarse, fine, off);
  if (st != CHEMORA_OK) return st;
  if (ntimes < 1 || ntimes > kMaxTimeLevels)
    return fail(CHEMORA_ERR_INVALID, "ntimes must be in [1, %d], got %d", kMaxTimeLevels, ntimes);
  if (!levels || !times)
    return fail(CHEMORA_ERR_INVALID, "coarse states and times must not be NULL");
  const long long cb = coarse->state_elems * 8;
  for (int l = 0; l < ntimes; ++l) {
    if (!levels[l] || !aligned(levels[l]))
      return fail(CHEMORA_ERR_INVALID, "coarse_states[%d] is NULL or not 256-byte aligned", l);
    if (!std::isfinite(times[l])) return fail(CHEMORA_ERR_INVALID, "times[%d] is not finite", l);
    if (avoid && overlaps(levels[l], cb, avoid, avoid_bytes))
      return fail(CHEMORA_ERR_INVALID, "coarse_states[%d] overlaps the fine state", l);
    for (int m = 0; m < l; ++m)
      if (times[m] == times[l]) return fail(CHEMORA_ERR_INVALID, "times must be distinct");
  }
  const Geo &C = coarse->geo, &F = fine->geo;
  for (int a = 0; a < 3; ++a) {
    if (C.n[a] + 2 * C.g < 6)
      return fail(CHEMORA_ERR_INVALID, "the coarse block needs >= 6 extended points along axis %d",
                  a);
    for (int i = -F.g; i < F.n[a] + F.g; ++i) {
      const long long q = (long long)off[a] + i;
      const long long b = q >= 0 ? q / 2 : -((-q + 1) / 2);  // floor(q / 2)
      const long long lo = (q & 1) ? b - 2 : b, hi = (q & 1) ? b + 3 : b;
      if (lo < -C.g || hi >= C.n[a] + C.g)
        return fail(CHEMORA_ERR_INVALID,
                    "fine ghost point %d on axis %d needs coarse points [%lld, %lld], outside the "
                    "coarse extended range [%d, %d)", i, a, lo, hi, -C.g, C.n[a] + C.g);
    }
  }
  return CHEMORA_OK;
}

}  // namespace chemora

extern "C" {

int chemora_prolong(const chemora_grid* coarse, const double* const* coarse_states,
                    const double* times, int32_t ntimes, double t, const chemora_grid* fine,
                    double* fine_state, chemora_stream stream) {
  int off[3];
  if (!fine_state) return fail(CHEMORA_ERR_INVALID, "fine_state must not be NULL");
  if (!std::isfinite(t)) return fail(CHEMORA_ERR_INVALID, "t must be finite");
  if (!aligned(fine_state)) return fail(CHEMORA_ERR_INVALID, "fine_state must be 256-byte aligned");
  int st = check_prolong_source(coarse, fine, coarse_states, times, ntimes, fine_state,
                                fine ? fine->state_elems * 8 : 0, off);
  if (st != CHEMORA_OK) return st;
  double wt[kMaxTimeLevels];
  time_weights(times, ntimes, t, wt);
  return device_status(launch_prolong(coarse->geo, coarse_states, wt, ntimes, fine->geo, off,
                                      coarse->nvars, fine_state, static_cast<hipStream_t>(stream)),
                       "prolongation launch");
}

int chemora_restrict(const chemora_grid* coarse, double* coarse_state, const chemora_grid* fine,
                     const double* fine_state, chemora_stream stream) {
  int off[3];
  int st = level_pair(coarse, fine, off);
  if (st != CHEMORA_OK) return st;
  if (!coarse_state || !fine_state)
    return fail(CHEMORA_ERR_INVALID, "coarse_state and fine_state must not be NULL");
  if (!aligned(coarse_state) || !aligned(fine_state))
    return fail(CHEMORA_ERR_INVALID, "states must be 256-byte aligned");
  if (overlaps(coarse_state, coarse->state_elems * 8, fine_state, fine->state_elems * 8))
    return fail(CHEMORA_ERR_INVALID, "coarse_state and fine_state overlap");
  // coarse interior i coincides with fine point 2 i - off, which must be interior
  int lo[3], cnt[3];
  for (int a = 0; a < 3; ++a) {
    const long long o = off[a];
    long long l0 = o >= 0 ? (o + 1) / 2 : -((-o) / 2);  // ceil(off / 2): fine index >= 0
    long long h0 = fine->geo.n[a] - 1 + o;             // fine index <= n_fine - 1
    h0 = h0 >= 0 ? h0 / 2 : -((-h0 + 1) / 2);           // floor
    l0 = std::max(l0, 0LL);
    h0 = std::min(h0, (long long)coarse->geo.n[a] - 1);
    lo[a] = (int)l0;
    cnt[a] = h0 >= l0 ? (int)(h0 - l0 + 1) : 0;
  }
  if ((long long)cnt[0] * cnt[1] * cnt[2] == 0) return CHEMORA_OK;
  return device_status(launch_restrict(coarse->geo, coarse_state, fine->geo, fine_state, off, lo,
                                       cnt, coarse->nvars, static_cast<hipStream_t>(stream)),
                       "restriction launch");
}

}  // extern "C"
