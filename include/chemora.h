/*
 * chemora.h -- C ABI of libchemora: MI355X (gfx950) evaluation of the
 * time-evolution right-hand side of a PDE system on a 3-D uniform grid block
 * with ghost zones, and the RK4 method of lines built on it.
 *
 * The calls follow the paper's statement of the problem (Schnetter et al.,
 * "Chemora: A PDE Solving Framework for Modern HPC Architectures",
 * arXiv:1410.1764):
 *   - a state vector of grid functions plus run-time parameters
 *     (Sec. III.B.1, "Physics system description"; Fig. 1, the groups
 *     "Evolved" and "parameters");
 *   - an RHS calculation, i.e. one loop kernel over the grid (Fig. 1, the
 *     calculation "RHS"; Sec. III.D, several thousand flops per point for the
 *     Einstein equations);
 *   - a driver that owns the grid, its ghost zones and device memory
 *     (Sec. II, the driver thorn);
 *   - a separate Runge-Kutta time integrator (Sec. II, the time-integrator
 *     thorn);
 *   - many grid patches of a mesh-refinement or multi-block hierarchy
 *     (Sec. IV, the Carpet driver) advanced together.
 *
 * Conventions common to every call
 * --------------------------------
 * Memory.  Every array argument named state, rhs, workspace, hm, norms or
 * meta is DEVICE memory owned by the caller (for example a torch tensor's
 * data_ptr()).  The library never allocates or frees device memory for
 * data and never keeps a pointer after a call returns, except the batch
 * plan (chemora_batch_step), which keeps the pointers of its patch list
 * until chemora_batch_release.  Grid objects hold host metadata only.
 *
 * Layout.  A grid function is stored x fastest with element strides
 * (1, sy, sz) reported by chemora_grid_layout; point (i, j, k) with each
 * index in [-ghost, n + ghost) sits at element interior_offset + i + j*sy +
 * k*sz.  Rows are padded so that interior x = 0 starts on a 128-byte
 * boundary.  The nvars grid functions of a state follow each other at the
 * stride sv.  Every value is an IEEE double (FP64) in memory, in both
 * precision modes.  Variable order:
 *   wave (2):  u, rho
 *   wave5 (5): u, rho, v1, v2, v3
 *   BSSN (24): chi, gt11, gt12, gt13, gt22, gt23, gt33, trK, At11, At12,
 *              At13, At22, At23, At33, Gamt1, Gamt2, Gamt3, alpha, beta1,
 *              beta2, beta3, B1, B2, B3
 * Pointers must be 256-byte aligned.
 *
 * Streams.  chemora_stream is a hipStream_t (NULL = the null stream).  Every
 * compute call only enqueues work on that stream and returns; kernel faults
 * surface at the caller's next synchronisation.
 *
 * Errors.  Every call returns a chemora_status.  Argument errors are found
 * before anything is enqueued; a failed launch returns CHEMORA_ERR_DEVICE.
 * chemora_last_error() describes the last failure on the calling thread.
 * Nothing throws or aborts across the ABI.
 */
#ifndef CHEMORA_H
#define CHEMORA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct chemora_grid chemora_grid; /* opaque, host-side metadata */
typedef void* chemora_stream;             /* hipStream_t; NULL = null stream */

typedef enum {
  CHEMORA_OK = 0,
  CHEMORA_ERR_INVALID = 1,     /* bad argument; nothing was enqueued */
  CHEMORA_ERR_UNSUPPORTED = 2, /* valid but not implemented combination */
  CHEMORA_ERR_DEVICE = 3,      /* HIP runtime or launch failure */
  CHEMORA_ERR_HOST_NOMEM = 4   /* host allocation failed */
} chemora_status;

/* WAVE: eq. (1) in the two-variable reading (du/dt = rho, drho/dt = Lap u);
 * BSSN: the Einstein equations (Sec. III.D); WAVE5: eq. (1) in the paper's
 * own first-order form (Fig. 1: u, rho, v_i). */
enum { CHEMORA_WAVE = 1, CHEMORA_BSSN = 2, CHEMORA_WAVE5 = 3 };
/* FP64: all arithmetic in double.  MIXED: differences of neighbouring
 * values in double, then stencil weights and the right-hand-side algebra in
 * float; state, RK4 accumulation and constraints stay double. */
enum { CHEMORA_FP64 = 0, CHEMORA_MIXED = 1 };
/* ghost zones: periodic images; the analytic gauge wave at the (stage)
 * time (BSSN only); or left to the caller (chemora_rhs only). */
enum { CHEMORA_BC_PERIODIC = 0, CHEMORA_BC_GAUGEWAVE = 1, CHEMORA_BC_CALLER = 2 };
enum { CHEMORA_SLICING_1PLUSLOG = 0, CHEMORA_SLICING_HARMONIC = 1 };
enum { CHEMORA_SHIFT_FROZEN = 0, CHEMORA_SHIFT_GAMMADRIVER = 1 };

/* Grid description (Sec. II driver: grid and ghost zones; Sec. III.B.1:
 * run-time parameters of the physics system). */
typedef struct {
  int32_t n[3];      /* interior points per axis, each >= 1 */
  int32_t ghost;     /* ghost width: >= 2 for the wave systems, >= 3 for BSSN, <= 8 */
  double h[3];       /* spacing per axis, > 0 */
  double origin[3];  /* coordinate of interior point (0,0,0) */
  int32_t system;    /* CHEMORA_WAVE, CHEMORA_BSSN or CHEMORA_WAVE5 */
  int32_t precision; /* CHEMORA_FP64 or CHEMORA_MIXED */
  int32_t boundary;  /* CHEMORA_BC_*; periodic needs n >= ghost per axis */
  int32_t slicing;   /* BSSN: 1+log (dt alpha = adv - 2 alpha K) or harmonic (- alpha^2 K) */
  int32_t shift;     /* BSSN: frozen (dt beta = dt B = 0) or Gamma-driver */
  double shift_F;    /* Gamma-driver: dt beta^i = adv + F B^i (usually 0.75) */
  double eta;        /* Gamma-driver damping: dt B^i = ... - eta B^i (usually 2) */
  double gw_amp;     /* gauge wave amplitude A, |A| < 1 */
  double gw_wavelength; /* gauge wave wavelength d > 0 */
  int32_t gw_axis;   /* gauge wave direction 0, 1 or 2 */
  int32_t enforce;   /* BSSN only (else 0): 1 = after every RK substage rescale gt_ij so
                        that det gt = 1, then remove the trace of At_ij; 0 = off */
  double ko_sigma;   /* BSSN only (else 0): Kreiss-Oliger dissipation strength >= 0,
                        adding sigma/64 sum_d (sixth difference along d) / h_d to the
                        right-hand side of every evolved variable; 0 = off; order 4 only */
  int32_t fd_order;  /* finite-difference order (Sec. III.B.2: the order is a parameter of
                        the discretisation): 0 or 4 (default), or 6 or 8 for BSSN, which
                        needs ghost >= fd_order/2 + 1 and runs the LDS-staged high-order
                        kernels (the cached-load ones are an ablation switch) */
} chemora_grid_desc;

/* Create a grid object from a description (copied).  Validates every field
 * (see chemora_grid_desc) and returns CHEMORA_ERR_INVALID with a message on
 * the first violation.  *out receives the new object; destroy it with
 * chemora_grid_destroy. */
int chemora_grid_create(const chemora_grid_desc* desc, chemora_grid** out);
int chemora_grid_destroy(chemora_grid* grid);

/* Layout of one state: nvars grid functions; strides[0..3] = element strides
 * along x, y, z and between variables; interior_offset = element index of
 * interior point (0,0,0) of variable 0; state_elems = number of doubles a
 * state array must hold.  Any output pointer may be NULL. */
int chemora_grid_layout(const chemora_grid* grid, int32_t* nvars, int64_t strides[4],
                        int64_t* interior_offset, int64_t* state_elems);

/* Bytes of device workspace chemora_rk4_step needs: two stage buffers and
 * the RK4 accumulator, each a full state.  Returns -1 for a NULL grid. */
int64_t chemora_workspace_bytes(const chemora_grid* grid);

/* Fill the ghost zones of state (Sec. II: the driver owns ghost zones):
 * periodic images (x, then y, then z, so edges and corners are filled), or
 * the analytic gauge wave evaluated at time t (BSSN).  BC_CALLER: nothing to
 * do, returns CHEMORA_OK. */
int chemora_fill_ghosts(chemora_grid* grid, double* state, double t, chemora_stream stream);

/* One evaluation of the right-hand side (Fig. 1 "RHS"; eq. (1) for the wave
 * system, two-variable reading du/dt = rho, drho/dt = Laplacian u; the BSSN
 * form of the Einstein equations, Sec. III.D) with 4th-order centred
 * differences and 4th-order lopsided (upwind) differences for the advection
 * terms.  Reads state at interior points and their stencil neighbours,
 * i.e. the ghosts must already be valid (chemora_fill_ghosts); writes rhs
 * (same layout as a state, FP64 in both precision modes) at interior points
 * only.  state and rhs must not overlap. */
int chemora_rhs(chemora_grid* grid, const double* state, double* rhs, chemora_stream stream);

/* Advance state by nsteps classical RK4 steps of size dt starting at time t
 * (Sec. II: the time-integrator thorn).  Ghosts are refilled before every
 * right-hand-side evaluation -- periodic ghosts by a fill kernel launched
 * after each substage's kernel (the environment switch
 * CHEMORA_PERIODIC=images makes the substage kernel write the images
 * itself); analytic ghosts use the stage time
 * t_n + c_s dt, c = (0, 1/2, 1/2, 1) -- and are valid on return at time
 * t + nsteps*dt.  workspace: chemora_workspace_bytes(grid) bytes, contents
 * ignored.  BC_CALLER is rejected (CHEMORA_ERR_INVALID). */
int chemora_rk4_step(chemora_grid* grid, double* state, void* workspace, double t, double dt,
                     int32_t nsteps, chemora_stream stream);

/* Hamiltonian and momentum constraints of the BSSN system (Sec. III.B.1:
 * constraints belong to the physics description), FP64 in both precision
 * modes, centred stencils only; ghosts must be valid.  hm (may be NULL):
 * a 4-variable state (H, M1, M2, M3) written at interior points.  norms:
 * device double[4], the RMS over interior points of H, M1, M2, M3, reduced
 * in a fixed order (bitwise reproducible).  workspace:
 * chemora_constraints_workspace_bytes(grid) bytes.  Wave grids:
 * CHEMORA_ERR_UNSUPPORTED. */
int64_t chemora_constraints_workspace_bytes(const chemora_grid* grid);
int chemora_constraints(chemora_grid* grid, const double* state, double* hm, double* norms,
                        void* workspace, chemora_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * computation and results as chemora_constraints (bitwise), with the
 * per-workgroup partial sums in a static device buffer of the library
 * instead of a workspace.  Allocates nothing.  The buffer holds 2^20
 * doubles per GPU (8 MiB, kept until the process ends); a grid whose
 * chemora_constraints_workspace_bytes exceeds 8 MiB returns
 * CHEMORA_ERR_INVALID before any launch.  Every call on one GPU shares that
 * GPU's buffer: calls that overlap on one GPU (other streams, other host
 * threads) race and must be serialised by the caller. */
int chemora_constraints_noalloc(chemora_grid* grid, const double* state, double* hm,
                                double* norms, chemora_stream stream);

/* Fig. 1's "Energy" calculation for the first-order wave system (WAVE5):
 * eps = (rho^2 + v_i v_i)/2 at interior points, written to eps (a 1-variable
 * state, may be NULL), and the total sum(eps) h_x h_y h_z written to the
 * device double *total, summed in a fixed order (bitwise reproducible).
 * workspace: chemora_energy_workspace_bytes(grid) bytes.  Other systems:
 * CHEMORA_ERR_UNSUPPORTED. */
int64_t chemora_energy_workspace_bytes(const chemora_grid* grid);
int chemora_energy(chemora_grid* grid, const double* state, double* eps, double* total,
                   void* workspace, chemora_stream stream);

/* ---- batches of uneven patches (Sec. IV: mesh-refinement / multi-block
 * patches of the Carpet driver; Sec. III.B.3: a GPU run-time library that
 * auto-tunes the thread assignment with a performance model) ----------- */

typedef struct {
  chemora_grid* grid; /* a BSSN grid with boundary CHEMORA_BC_GAUGEWAVE */
  double* state;      /* its state (device) */
  void* workspace;    /* chemora_workspace_bytes(grid) bytes (device) */
} chemora_patch;

/* Device bytes of the plan buffer for a batch of npatches patches (patch
 * descriptors, work list, device clock).  Returns -1 if npatches < 1. */
int64_t chemora_batch_meta_bytes(int32_t npatches);

/* Advance every patch by nsteps RK4 steps of size dt from time t.  All
 * patches must share one system (BSSN), one precision, one fd_order and the
 * gauge-wave boundary (INVALID otherwise); FP64 batches of fd_order 6 return
 * CHEMORA_ERR_UNSUPPORTED (mixed precision and fd_order 8 run).  Each RK
 * substage is ONE kernel launch over a work list of (patch, tile) items
 * plus the analytic ghost zones of the next stage (FP64 4th order: a
 * resident grid that strides the list; otherwise one workgroup per item);
 * the four substages and the clock update are captured once in a HIP graph
 * that is replayed once per step.  The plan (tile shape per
 * patch, work list, graph) is built on the first call for a given meta
 * buffer and patch list, and reused while the same meta pointer, patch list
 * and dt are passed; meta: chemora_batch_meta_bytes(npatches) device bytes
 * that the caller keeps alive until chemora_batch_release(meta). */
int chemora_batch_step(const chemora_patch* patches, int32_t npatches, void* meta, double t,
                       double dt, int32_t nsteps, chemora_stream stream);

/* Coarse parent of a batch patch on a refined level (Sec. IV: the
 * mesh-refinement driver fills a refined patch's ghost zones from the next
 * coarser level). */
typedef struct {
  const chemora_grid* coarse; /* NULL: the patch keeps the analytic gauge-wave ghosts */
  const double* levels[3];    /* ntimes coarse states (device, 256-byte aligned), read only */
  double times[3];            /* their times, distinct */
  int32_t ntimes;             /* 1..3 */
} chemora_parent;

/* chemora_batch_step for a batch in which some patches are refined patches
 * of a coarser grid: parents[q] (host array of npatches entries; NULL = no
 * parents) gives patch q's parent.  The ghost zones of such a patch -- of
 * its state at t and of every RK stage's output, at the stage's time -- are
 * prolongated from the parent's time levels as chemora_prolong does
 * (degree-5 Lagrange in space, Lagrange in time through the levels),
 * instead of the analytic gauge wave: inside the batch's substage launch,
 * one ghost item per box of the patch's ghost shell.  Requirements (INVALID
 * otherwise): each parent a BSSN grid in ratio 2 to its patch whose
 * extended block holds every coarse point the patch's ghost stencils reach
 * (chemora_prolong's checks), time levels that overlap no state or
 * workspace of the batch.  UNSUPPORTED: parents in batches of fd_order 6 or
 * 8, or a patch ghost width above 5.  The plan is rebuilt (and its graph
 * captured again) whenever a parent's grid, levels or times change, so a
 * caller that rotates its coarse levels pays one plan per coarse step. */
int chemora_batch_step_levels(const chemora_patch* patches, const chemora_parent* parents,
                              int32_t npatches, void* meta, double t, double dt, int32_t nsteps,
                              chemora_stream stream);
int chemora_batch_release(void* meta);

/* Choose the kernel kind and tiles of later batch plans for patches like
 * the given ones (same precision and fd_order), recorded in an in-process
 * table.  A performance model ranks the cached-load kind's tile candidates
 * for each size class of patches: every tile costs its whole wavefronts
 * (wave quantisation of ragged tiles) times a halo factor, and the kernel's
 * static assignment of items (one share of the work list per XCD, round
 * robin over a persistent grid, or greedy hand-out of one item per
 * workgroup, as the instance runs) is simulated on a grid of the kernel
 * instance's resident workgroups per CU (occupancy, from its registers and
 * LDS) times the CUs.  The best three are timed and the fastest kept.  Then
 * the candidate kinds of the order (4th: cached loads, staged 32x8, staged
 * 16x16; 6th and 8th: staged 32x8, staged 16x16) are timed over the whole
 * batch and the fastest becomes the kind of later plans (untuned: staged
 * 32x8).  When table_path is not NULL, the model scores and timings are
 * written there as JSON.  Runs kernels on the null stream and synchronises;
 * destroys any plan held for meta.  Same patch validation as
 * chemora_batch_step. */
int chemora_autotune(const chemora_patch* patches, int32_t npatches, void* meta,
                     const char* table_path);

/* The autotuner's performance model, for inspection and testing: predicted
 * duration of one substage launch, in wavefront-plane units, of a batch of
 * npatches patches with interior sizes dims[3q..3q+2] and tiles
 * tiles[3q..3q+2] (x and y threads, planes per item) on kernel kind kind
 * (0 cached loads; staged 1/2 4th order 32x8/16x16, 3/5 6th order, 4/6 8th
 * order; 7 4th order z-blocked 32x8x2) of finite-difference order fd_order,
 * with per_cu resident workgroups per CU and grid of them resident in all;
 * ghost items of ghost_width ghost zones included when ghost_width > 0;
 * per_item != 0: one item per workgroup, handed out by the hardware
 * (greedy), else a persistent grid striding each XCD's share (static).
 * All pointers host memory; *out receives the prediction.  INVALID on NULL
 * or out-of-range arguments. */
int chemora_batch_model(const int32_t* dims, const int32_t* tiles, int32_t npatches,
                        int32_t kind, int32_t fd_order, int32_t per_cu, int32_t grid,
                        int32_t ghost_width, int32_t per_item, double* out);

/* Tile shape the batch planner would use for a 4th-order patch of size n
 * under the current kind of that precision (the tuned one after
 * chemora_autotune; CHEMORA_BATCH_KIND overrides): tile[0..2] in points. */
int chemora_batch_tile(const int32_t n[3], int32_t precision, int32_t tile[3]);

/* ---- two refinement levels (Sec. IV: the mesh-refinement driver) ------ */

/* Levels pair: a coarse and a fine grid of the same system with
 * h_coarse = 2 h_fine on every axis and the fine origin a whole number of
 * fine spacings from the coarse origin (within 1e-9 of one).  Fine point i
 * then either coincides with a coarse point or lies half-way between two.
 * Both grids may use either precision: the values moved are FP64. */

/* Prolongation: fill every ghost point of fine_state from the coarse level.
 * Per axis a coincident point takes the coarse value and a half-way point
 * the degree-5 Lagrange interpolant through the six coarse points around
 * it (weights (3, -25, 150, 150, -25, 3)/256); the tensor product over the
 * axes.  coarse_states: host array of ntimes (1..3) device states of the
 * coarse grid at the distinct times times[0..ntimes-1] (host array), with
 * valid ghost zones; they are combined with the Lagrange weights in time at
 * time t (t outside the levels' span extrapolates).  The fine interior and
 * the coarse states are not written.  Errors (INVALID): levels not a pair as
 * above, different systems, a fine ghost point whose coarse stencil would
 * leave the coarse extended block, a coarse block with fewer than 6
 * extended points along an axis, bad times, NULL, misaligned or
 * overlapping states. */
int chemora_prolong(const chemora_grid* coarse, const double* const* coarse_states,
                    const double* times, int32_t ntimes, double t, const chemora_grid* fine,
                    double* fine_state, chemora_stream stream);

/* Restriction by injection: every interior point of coarse_state that
 * coincides with an interior point of the fine grid takes that point's
 * value, for every grid function; nothing else is written (the coarse ghost
 * zones are the caller's to refill).  No coinciding points: nothing to do,
 * CHEMORA_OK.  Errors (INVALID): levels not a pair, different systems,
 * NULL, misaligned or overlapping states. */
int chemora_restrict(const chemora_grid* coarse, double* coarse_state, const chemora_grid* fine,
                     const double* fine_state, chemora_stream stream);

/* ---- measurement helper --------------------------------------------- */

/* Streaming copy of nbytes (multiple of 16) from src to dst on stream: the
 * denominator used to calibrate hardware counters and achievable HBM
 * bandwidth. */
int chemora_probe_copy(void* dst, const void* src, int64_t nbytes, chemora_stream stream);

/* FMA throughput probe, the measured counterpart of the vector ALU peak:
 * 8192 workgroups of 256 threads, each thread running 16 independent FMA
 * chains for iters steps in FP64 (precision CHEMORA_FP64) or FP32 (
 * CHEMORA_MIXED; FP32 as this library compiles it, unpacked).  out: device
 * buffer of chemora_probe_fma_bytes() bytes (receives one value per thread,
 * so that no FMA is eliminated).  *flops (host) receives the floating-point
 * operations of the launch (2 per FMA).  Asynchronous on stream. */
int64_t chemora_probe_fma_bytes(void);
int chemora_probe_fma(int32_t precision, void* out, int32_t iters, double* flops,
                      chemora_stream stream);

/* Thread-local description of the last failure; never NULL. */
const char* chemora_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CHEMORA_H */
