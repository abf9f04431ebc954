/*
 * oracle.h -- CPU oracle for the Chemora right-hand-side path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this code; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no source with the HIP path.
 *
 * Plain, slow, obviously correct FP64 C.  Compiled with
 * -O2 -fno-fast-math -ffp-contract=off so that every expression rounds in
 * the order it is written; OpenMP only splits loops over z-planes.
 *
 * Layout (the oracle's own, unpadded): a grid function is an array of
 * (n_x+2g)(n_y+2g)(n_z+2g) doubles, x fastest, holding the points with
 * index i in [-g, n+g) per axis; point i sits at x = origin + i*h.  A state
 * of nvar grid functions stores them one after another, in the variable
 * order listed below.
 *
 * Wave system (2 variables): u, rho.
 * First-order wave system (5 variables): u, rho, v1, v2, v3.
 * BSSN system (24 variables): chi, gt11, gt12, gt13, gt22, gt23, gt33, trK,
 *   At11, At12, At13, At22, At23, At33, Gamt1, Gamt2, Gamt3, alpha,
 *   beta1, beta2, beta3, B1, B2, B3.
 */
#ifndef CHEMORA_ORACLE_H
#define CHEMORA_ORACLE_H

typedef struct {
  int n[3];            /* interior points per axis */
  int g;               /* ghost width */
  double h[3];         /* grid spacing per axis */
  double origin[3];    /* coordinate of interior point (0,0,0) */
  int slicing;         /* 0: 1+log, 1: harmonic */
  int shift;           /* 0: frozen, 1: Gamma-driver */
  double shift_F;      /* Gamma-driver coefficient F */
  double eta;          /* Gamma-driver damping eta */
  double gw_amp;       /* gauge wave amplitude A */
  double gw_d;         /* gauge wave wavelength d */
  int gw_axis;         /* gauge wave direction 0,1,2 */
  double ko_sigma;     /* Kreiss-Oliger dissipation strength (0: none) */
  int enforce;         /* 1: det gt = 1 and tr At = 0 after every RK substage */
  int fd_order;        /* BSSN finite-difference order: 4 (also 0), 6 or 8 */
} orc_params;

enum { ORC_WAVE = 1, ORC_BSSN = 2, ORC_WAVE5 = 3 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_GAUGEWAVE = 1 };

int  orc_num_threads(void);
void orc_fill_periodic(const orc_params* p, int nvar, double* f);
void orc_fill_gaugewave(const orc_params* p, double t, double* y);
void orc_wave_rhs(const orc_params* p, const double* y, double* r);
void orc_wave5_rhs(const orc_params* p, const double* y, double* r);
double orc_wave5_energy(const orc_params* p, const double* y, double* eps);
void orc_bssn_rhs(const orc_params* p, const double* y, double* r);
int  orc_rk4(const orc_params* p, int system, int bc, double* y, double t,
             double dt, int nsteps);
/* RK4 steps of a refined block whose ghost zones at every stage time are
 * prolongated (orc_prolong) from ntimes levels of the coarse block at the
 * given times; returns 1 (state partly advanced) if a prolongation fails */
int  orc_rk4_prolong(const orc_params* p, int system, double* y, double t, double dt,
                     int nsteps, const orc_params* coarse, const double* const* yc,
                     const double* times, int ntimes);
void orc_bssn_constraints(const orc_params* p, const double* y, double* hm,
                          double norms[4]);
void orc_stencil(const orc_params* p, const double* f, int kind, int a, int b,
                 const double* sgn, double* out);
void orc_bssn_enforce(const orc_params* p, double* y);
int  orc_prolong(const orc_params* coarse, const double* const* yc, const double* times,
                 int ntimes, double t, const orc_params* fine, double* yf, int nvar);
int  orc_restrict(const orc_params* coarse, double* yc, const orc_params* fine,
                  const double* yf, int nvar);

#endif
