/*
 * oracle.c -- CPU oracle for the Chemora right-hand-side path.
 *
 * TEST INFRASTRUCTURE ONLY: the product library never includes, links or
 * calls this file.  It is the plain definition that the HIP path is checked
 * against, written from the paper and from the standard BSSN literature the
 * paper builds on, in FP64 with no blocking, fusion or reordering:
 *
 *   - the time-evolution right-hand side of a PDE system evaluated by finite
 *     differences on a uniform block with ghost zones (Sec. III "Efficient
 *     collaborations vs. efficient code", eq. (1); Sec. III.B.2
 *     "Discretisation description": standard centred finite-difference
 *     operators, here of 4th order);
 *   - the scalar wave system in the two-variable reading du/dt = rho,
 *     drho/dt = Laplacian(u) (eq. (1) with v_i = d_i u eliminated), and in
 *     the paper's own first-order form with five variables (eq. (1),
 *     Fig. 1: du/dt = rho, drho/dt = d_i v_i, dv_i/dt = d_i rho) with the
 *     energy density eps = (rho^2 + v_i v_i)/2 of Fig. 1's Energy calculation;
 *   - the BSSN form of the Einstein equations that the paper evolves
 *     (Sec. III.D "Single-node performance"; its cited formulation), in the
 *     chi-variant with 1+log or harmonic slicing and a Gamma-driver or
 *     frozen shift, advection terms by lopsided (upwinded) 4th-order stencils;
 *   - ghost-zone filling, periodic or from the analytic gauge wave, and the
 *     classical RK4 method of lines (Sec. II, the driver and time-integrator
 *     thorns);
 *   - the Hamiltonian and momentum constraints with FP64 RMS norms
 *     (Sec. III.B.1 "Physics system description": constraints are part of a
 *     physics system).
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp (no contraction,
 * so every expression rounds in the order written).
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* geometry of one block                                                    */

typedef struct {
  int n[3], g, e[3];
  long sy, sz, npts;
} geom;

static geom mkgeom(const orc_params* p) {
  geom G;
  G.g = p->g;
  for (int d = 0; d < 3; d++) {
    G.n[d] = p->n[d];
    G.e[d] = p->n[d] + 2 * p->g;
  }
  G.sy = G.e[0];
  G.sz = (long)G.e[0] * G.e[1];
  G.npts = G.sz * G.e[2];
  return G;
}

static long idx(const geom* G, int i, int j, int k) {
  return (long)(i + G->g) + (long)(j + G->g) * G->sy + (long)(k + G->g) * G->sz;
}

static int is_interior(const geom* G, int i, int j, int k) {
  return i >= 0 && i < G->n[0] && j >= 0 && j < G->n[1] && k >= 0 && k < G->n[2];
}

int orc_num_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* 4th-order finite-difference operators (Sec. III.B.2: standard centred
 * operators of a chosen order; the lopsided pair is the 4th-order
 * one-sided-by-one-point stencil used for advection terms).
 * f points at the centre value; s is the stride along the axis.
 *
 * Each operator is written on differences of neighbouring values (its
 * weights sum to zero, so this is the same linear combination).  For data
 * that is nearly constant -- e.g. flat space plus 1e-10 noise -- such a
 * difference is exact in floating point, whereas summing the weighted values
 * themselves would round at the size of the constant and lose the signal.  */

static double fd1(const double* f, long s, double h) {
  const double d1 = f[s] - f[-s], d2 = f[2 * s] - f[-2 * s];
  return (8.0 * d1 - d2) / (12.0 * h);
}

static double fd2(const double* f, long s, double h) {
  const double s1 = (f[s] - f[0]) + (f[-s] - f[0]);
  const double s2 = (f[2 * s] - f[0]) + (f[-2 * s] - f[0]);
  return (16.0 * s1 - s2) / (12.0 * h * h);
}

/* mixed derivative: the centred first-derivative stencil applied along both
 * axes, grouped as q_mn = [f(m,n) - f(-m,n)] - [f(m,-n) - f(-m,-n)] with
 * weights 8 (offset 1) and -1 (offset 2) along each axis */
static double fd11(const double* f, long sa, long sb, double ha, double hb) {
  double q[3][3];
  for (int m = 1; m <= 2; m++)
    for (int n = 1; n <= 2; n++)
      q[m][n] = (f[m * sa + n * sb] - f[-m * sa + n * sb]) -
                (f[m * sa - n * sb] - f[-m * sa - n * sb]);
  return (64.0 * q[1][1] - 8.0 * q[1][2] - 8.0 * q[2][1] + q[2][2]) / (144.0 * ha * hb);
}

/* sixth difference along stride s, on neighbour differences:
 * f3 - 6 f2 + 15 f1 - 20 f0 + 15 f-1 - 6 f-2 + f-3
 * = [(f3-f0)+(f-3-f0)] - 6 [(f2-f0)+(f-2-f0)] + 15 [(f1-f0)+(f-1-f0)].
 * Kreiss-Oliger dissipation for a 4th-order scheme adds
 * (sigma / 64) sum_d delta6_d u / h_d to du/dt: the (-1)^(p+1) sigma
 * h^(2p-1) / 2^(2p) (D+ D-)^p form with p = 3; its symbol is
 * -(sigma / h) sin^6(theta / 2), so it damps every mode and vanishes on
 * polynomials of degree <= 5. */
static double delta6(const double* f, long s) {
  const double s1 = (f[s] - f[0]) + (f[-s] - f[0]);
  const double s2 = (f[2 * s] - f[0]) + (f[-2 * s] - f[0]);
  const double s3 = (f[3 * s] - f[0]) + (f[-3 * s] - f[0]);
  return (s3 - 6.0 * s2) + 15.0 * s1;
}

/* lopsided first derivative, shifted one point towards the upwind side
 * chosen by the sign of the advecting velocity: weights (-3, -10, 18, -6, 1)
 * at offsets (-1, 0, 1, 2, 3) for vel >= 0, mirrored for vel < 0 */
static double fdup(const double* f, long s, double h, double vel) {
  const double f0 = f[0];
  if (vel >= 0.0)
    return (-3.0 * (f[-s] - f0) + 18.0 * (f[s] - f0) - 6.0 * (f[2 * s] - f0) +
            (f[3 * s] - f0)) /
           (12.0 * h);
  return (3.0 * (f[s] - f0) - 18.0 * (f[-s] - f0) + 6.0 * (f[-2 * s] - f0) -
          (f[-3 * s] - f0)) /
         (12.0 * h);
}

/* Higher orders (the paper's code generator takes the finite-difference
 * order as a parameter, Sec. III.B.2).  The 4th-order operators above are
 * used for order 4; orders 6 and 8 use these, the standard centred
 * operators and the lopsided ones shifted one point upwind, each the unique
 * stencil on its points that is exact for polynomials of degree <= order,
 * written on neighbour differences with integer weights over a common
 * denominator:
 *   first:  sum_k A_k (f_k - f_-k) / (den h),        k = 1..m (m = order/2)
 *   second: sum_k B_k ((f_k - f0) + (f_-k - f0)) / (den2 h^2)
 *   mixed:  sum_(i,j) A_i A_j q_ij / (den^2 h_a h_b), q as for fd11
 *   upwind: sum_k U_k (f_k - f0) / (den h), k = -(m-1)..m+1, k != 0,
 *           mirrored (k -> -k, sign flipped) for vel < 0.              */
typedef struct {
  int m;                 /* half width of the centred stencils */
  double A[4], den;      /* first derivative */
  double B[4], den2;     /* second derivative */
  double U[10], uden;    /* upwind weights at offsets -(m-1) .. m+1 (index k + m - 1) */
} fdcoef;

static const fdcoef FD6 = {3, {45, -9, 1, 0}, 60, {270, -27, 2, 0}, 180,
                           {2, -24, -35, 80, -30, 8, -1, 0, 0, 0}, 60};
static const fdcoef FD8 = {4, {672, -168, 32, -3}, 840, {8064, -1008, 128, -9}, 5040,
                           {-5, 60, -420, -378, 1050, -420, 140, -30, 3, 0}, 840};

static const fdcoef* fd_table(int order) { return order == 8 ? &FD8 : &FD6; }

static double fd1o(const fdcoef* c, const double* f, long s, double h) {
  double acc = 0.0;
  for (int k = 1; k <= c->m; k++) acc += c->A[k - 1] * (f[k * s] - f[-k * s]);
  return acc / (c->den * h);
}

static double fd2o(const fdcoef* c, const double* f, long s, double h) {
  double acc = 0.0;
  for (int k = 1; k <= c->m; k++) acc += c->B[k - 1] * ((f[k * s] - f[0]) + (f[-k * s] - f[0]));
  return acc / (c->den2 * h * h);
}

static double fd11o(const fdcoef* c, const double* f, long sa, long sb, double ha, double hb) {
  double acc = 0.0;
  for (int i = 1; i <= c->m; i++)
    for (int j = 1; j <= c->m; j++) {
      const double q = (f[i * sa + j * sb] - f[-i * sa + j * sb]) -
                       (f[i * sa - j * sb] - f[-i * sa - j * sb]);
      acc += c->A[i - 1] * c->A[j - 1] * q;
    }
  return acc / (c->den * c->den * ha * hb);
}

static double fdupo(const fdcoef* c, const double* f, long s, double h, double vel) {
  const long dir = vel >= 0.0 ? s : -s;
  double acc = 0.0;
  for (int k = -(c->m - 1); k <= c->m + 1; k++)
    if (k != 0) acc += c->U[k + c->m - 1] * (f[k * dir] - f[0]);
  return (vel >= 0.0 ? acc : -acc) / (c->uden * h);
}

/* order dispatch: 0 or 4 -> the 4th-order operators */
static double D1(int order, const double* f, long s, double h) {
  return (order == 6 || order == 8) ? fd1o(fd_table(order), f, s, h) : fd1(f, s, h);
}
static double D2(int order, const double* f, long s, double h) {
  return (order == 6 || order == 8) ? fd2o(fd_table(order), f, s, h) : fd2(f, s, h);
}
static double D11(int order, const double* f, long sa, long sb, double ha, double hb) {
  return (order == 6 || order == 8) ? fd11o(fd_table(order), f, sa, sb, ha, hb)
                                    : fd11(f, sa, sb, ha, hb);
}
static double DUP(int order, const double* f, long s, double h, double vel) {
  return (order == 6 || order == 8) ? fdupo(fd_table(order), f, s, h, vel) : fdup(f, s, h, vel);
}

/* ------------------------------------------------------------------------ */
/* ghost zones (Sec. II: the driver owns ghost zones)                       */

/* periodic images: x first, then y over the x-extended range, then z over
 * the xy-extended range, so edges and corners are filled too */
void orc_fill_periodic(const orc_params* p, int nvar, double* f) {
  geom G = mkgeom(p);
  const int g = G.g, nx = G.n[0], ny = G.n[1], nz = G.n[2];
  for (int v = 0; v < nvar; v++) {
    double* a = f + v * G.npts;
    for (int k = 0; k < nz; k++)
      for (int j = 0; j < ny; j++)
        for (int i = -g; i < 0; i++) a[idx(&G, i, j, k)] = a[idx(&G, i + nx, j, k)];
    for (int k = 0; k < nz; k++)
      for (int j = 0; j < ny; j++)
        for (int i = nx; i < nx + g; i++) a[idx(&G, i, j, k)] = a[idx(&G, i - nx, j, k)];
    for (int k = 0; k < nz; k++)
      for (int i = -g; i < nx + g; i++) {
        for (int j = -g; j < 0; j++) a[idx(&G, i, j, k)] = a[idx(&G, i, j + ny, k)];
        for (int j = ny; j < ny + g; j++) a[idx(&G, i, j, k)] = a[idx(&G, i, j - ny, k)];
      }
    for (int j = -g; j < ny + g; j++)
      for (int i = -g; i < nx + g; i++) {
        for (int k = -g; k < 0; k++) a[idx(&G, i, j, k)] = a[idx(&G, i, j, k + nz)];
        for (int k = nz; k < nz + g; k++) a[idx(&G, i, j, k)] = a[idx(&G, i, j, k - nz)];
      }
  }
}

/* ------------------------------------------------------------------------ */
/* BSSN variable indices and the symmetric-pair map                         */

enum { CHI = 0, GT = 1, TRK = 7, AT = 8, GAM = 14, ALP = 17, BETA = 18, BB = 21, NB = 24 };
static const int SYM[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

/* Analytic gauge wave: the flat metric in coordinates where
 * ds^2 = -H dt^2 + H dx_a^2 + (other axes)^2, H = 1 - A sin(2 pi (x_a - t)/d),
 * with zero shift; an exact vacuum solution under harmonic slicing.  BSSN
 * variables from its 3-metric gamma_aa = H and extrinsic curvature
 * K_aa = -dt(gamma_aa)/(2 alpha).                                          */
static void gaugewave_point(const orc_params* p, double xa, double t, double* v,
                            long stride) {
  const double A = p->gw_amp, d = p->gw_d;
  const int a = p->gw_axis;
  const double th = 2.0 * M_PI * (xa - t) / d;
  const double H = 1.0 - A * sin(th), c = cos(th);
  for (int q = 0; q < NB; q++) v[q * stride] = 0.0;
  v[CHI * stride] = pow(H, -1.0 / 3.0);
  for (int b = 0; b < 3; b++) {
    v[(GT + SYM[b][b]) * stride] = (b == a) ? pow(H, 2.0 / 3.0) : pow(H, -1.0 / 3.0);
    v[(AT + SYM[b][b]) * stride] =
        (b == a) ? -(2.0 * M_PI * A / (3.0 * d)) * c * pow(H, -5.0 / 6.0)
                 : (M_PI * A / (3.0 * d)) * c * pow(H, -11.0 / 6.0);
  }
  v[TRK * stride] = -(M_PI * A / d) * c * pow(H, -1.5);
  v[(GAM + a) * stride] = -(4.0 * M_PI * A / (3.0 * d)) * c * pow(H, -5.0 / 3.0);
  v[ALP * stride] = sqrt(H);
}

/* fill every ghost point of all 24 BSSN grid functions from the gauge wave
 * evaluated at time t */
void orc_fill_gaugewave(const orc_params* p, double t, double* y) {
  geom G = mkgeom(p);
  const int g = G.g, a = p->gw_axis;
  for (int k = -g; k < G.n[2] + g; k++)
    for (int j = -g; j < G.n[1] + g; j++)
      for (int i = -g; i < G.n[0] + g; i++) {
        if (is_interior(&G, i, j, k)) continue;
        const int ii[3] = {i, j, k};
        const double xa = p->origin[a] + ii[a] * p->h[a];
        gaugewave_point(p, xa, t, y + idx(&G, i, j, k), G.npts);
      }
}

static int nvars_of(int system) {
  return system == ORC_WAVE ? 2 : (system == ORC_WAVE5 ? 5 : NB);
}

static void fill_ghosts(const orc_params* p, int system, int bc, double t, double* y) {
  if (system == ORC_BSSN && bc == ORC_BC_GAUGEWAVE)
    orc_fill_gaugewave(p, t, y);
  else
    orc_fill_periodic(p, nvars_of(system), y);
}

/* ------------------------------------------------------------------------ */
/* Scalar wave, eq. (1) in the two-variable reading:
 *   du/dt = rho,  drho/dt = d_xx u + d_yy u + d_zz u                         */

void orc_wave_rhs(const orc_params* p, const double* y, double* r) {
  geom G = mkgeom(p);
  const long st[3] = {1, G.sy, G.sz};
  const double* u = y;
  const double* rho = y + G.npts;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < G.n[2]; k++)
    for (int j = 0; j < G.n[1]; j++)
      for (int i = 0; i < G.n[0]; i++) {
        const long q = idx(&G, i, j, k);
        r[q] = rho[q];
        r[G.npts + q] = fd2(u + q, st[0], p->h[0]) + fd2(u + q, st[1], p->h[1]) +
                        fd2(u + q, st[2], p->h[2]);
      }
}

/* ------------------------------------------------------------------------ */
/* Scalar wave, eq. (1) in the paper's first-order form (Fig. 1 "RHS"):
 *   du/dt = rho,  drho/dt = d_x v_1 + d_y v_2 + d_z v_3,  dv_i/dt = d_i rho
 * with the 4th-order centred first derivative.                              */

void orc_wave5_rhs(const orc_params* p, const double* y, double* r) {
  geom G = mkgeom(p);
  const long st[3] = {1, G.sy, G.sz};
  const double* rho = y + G.npts;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < G.n[2]; k++)
    for (int j = 0; j < G.n[1]; j++)
      for (int i = 0; i < G.n[0]; i++) {
        const long q = idx(&G, i, j, k);
        r[q] = rho[q];
        double div = 0.0;
        for (int a = 0; a < 3; a++) div += fd1(y + (2 + a) * G.npts + q, st[a], p->h[a]);
        r[G.npts + q] = div;
        for (int a = 0; a < 3; a++) r[(2 + a) * G.npts + q] = fd1(rho + q, st[a], p->h[a]);
      }
}

/* Fig. 1 "Energy": eps = (rho^2 + v_i v_i)/2 at interior points (eps may be
 * NULL); returns the total sum(eps) h_x h_y h_z, summed plane by plane. */
double orc_wave5_energy(const orc_params* p, const double* y, double* eps) {
  geom G = mkgeom(p);
  const int nz = G.n[2];
  double* plane = calloc((size_t)nz, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; k++)
    for (int j = 0; j < G.n[1]; j++)
      for (int i = 0; i < G.n[0]; i++) {
        const long q = idx(&G, i, j, k);
        const double rho = y[G.npts + q], v1 = y[2 * G.npts + q], v2 = y[3 * G.npts + q],
                     v3 = y[4 * G.npts + q];
        const double e = 0.5 * (rho * rho + (v1 * v1 + v2 * v2 + v3 * v3));
        if (eps) eps[q] = e;
        plane[k] += e;
      }
  double s = 0.0;
  for (int k = 0; k < nz; k++) s += plane[k];
  free(plane);
  return s * p->h[0] * p->h[1] * p->h[2];
}

/* ------------------------------------------------------------------------ */
/* BSSN right-hand side at one interior point, in three phases:
 *   1. every stencil (centred 1st, centred 2nd and mixed, lopsided advection)
 *   2. the derived quantities (inverse metric, Christoffels, Ricci, ...)
 *   3. the 24 right-hand sides.
 * chi-form BSSN: chi = det(gamma)^(-1/3), gt_ij = chi gamma_ij,
 * At_ij = chi (K_ij - gamma_ij K / 3); the evolved Gamt^i enters only through
 * its derivatives (Ricci tensor) and its advection; everywhere else the
 * contracted Christoffel symbols recomputed from gt_ij are used.            */

static void bssn_point(const orc_params* p, const geom* G, const double* y, long q,
                       double out[NB], double cons[4]) {
  const long st[3] = {1, G->sy, G->sz};
  const double* h = p->h;
  double u[NB], d1[NB][3], d2[NB][3][3], adv[NB];

  /* phase 1: stencils */
  for (int v = 0; v < NB; v++) {
    const double* f = y + v * G->npts + q;
    u[v] = f[0];
    for (int a = 0; a < 3; a++) d1[v][a] = D1(p->fd_order, f, st[a], h[a]);
    for (int a = 0; a < 3; a++) {
      d2[v][a][a] = D2(p->fd_order, f, st[a], h[a]);
      for (int b = a + 1; b < 3; b++) {
        d2[v][a][b] = D11(p->fd_order, f, st[a], st[b], h[a], h[b]);
        d2[v][b][a] = d2[v][a][b];
      }
    }
  }
  const double beta[3] = {u[BETA], u[BETA + 1], u[BETA + 2]};
  for (int v = 0; v < NB; v++) {
    const double* f = y + v * G->npts + q;
    adv[v] = 0.0;
    for (int k = 0; k < 3; k++) adv[v] += beta[k] * DUP(p->fd_order, f, st[k], h[k], beta[k]);
  }
  /* Kreiss-Oliger dissipation of every variable (added to the right-hand
   * sides in phase 3; the frozen shift and B stay frozen) */
  double diss[NB];
  for (int v = 0; v < NB; v++) {
    const double* f = y + v * G->npts + q;
    diss[v] = 0.0;
    if (p->ko_sigma != 0.0)
      for (int k = 0; k < 3; k++) diss[v] += (p->ko_sigma / 64.0) * delta6(f, st[k]) / h[k];
  }

  /* phase 2: derived quantities */
  const double chi = u[CHI], trK = u[TRK], alpha = u[ALP];
  double gt[3][3], At[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      gt[i][j] = u[GT + SYM[i][j]];
      At[i][j] = u[AT + SYM[i][j]];
    }
  const double det = gt[0][0] * (gt[1][1] * gt[2][2] - gt[1][2] * gt[2][1]) -
                     gt[0][1] * (gt[1][0] * gt[2][2] - gt[1][2] * gt[2][0]) +
                     gt[0][2] * (gt[1][0] * gt[2][1] - gt[1][1] * gt[2][0]);
  double gu[3][3]; /* inverse conformal metric: adjugate over determinant */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      gu[i][j] = (gt[(j + 1) % 3][(i + 1) % 3] * gt[(j + 2) % 3][(i + 2) % 3] -
                  gt[(j + 1) % 3][(i + 2) % 3] * gt[(j + 2) % 3][(i + 1) % 3]) /
                 det;

  /* dgt[i][j][k] = d_k gt_ij */
  double dgt[3][3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++) dgt[i][j][k] = d1[GT + SYM[i][j]][k];

  /* Christoffels of the conformal metric: first index lowered, then raised */
  double cdl[3][3][3], cdu[3][3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++)
        cdl[i][j][k] = 0.5 * (dgt[i][k][j] + dgt[i][j][k] - dgt[j][k][i]);
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++) {
        double s = 0.0;
        for (int l = 0; l < 3; l++) s += gu[i][l] * cdl[l][j][k];
        cdu[i][j][k] = s;
      }
  double Gd[3]; /* contracted Christoffels recomputed from gt */
  for (int i = 0; i < 3; i++) {
    double s = 0.0;
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++) s += gu[j][k] * cdu[i][j][k];
    Gd[i] = s;
  }

  double dchi[3], dK[3], dalp[3], dbeta[3][3], dGam[3][3];
  for (int a = 0; a < 3; a++) {
    dchi[a] = d1[CHI][a];
    dK[a] = d1[TRK][a];
    dalp[a] = d1[ALP][a];
  }
  for (int k = 0; k < 3; k++)
    for (int j = 0; j < 3; j++) {
      dbeta[k][j] = d1[BETA + k][j]; /* d_j beta^k */
      dGam[k][j] = d1[GAM + k][j];   /* d_j Gamt^k */
    }
  double divbeta = 0.0;
  for (int k = 0; k < 3; k++) divbeta += dbeta[k][k];

  /* conformal covariant second derivative of chi */
  double DDchi[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double s = 0.0;
      for (int k = 0; k < 3; k++) s += cdu[k][i][j] * dchi[k];
      DDchi[i][j] = d2[CHI][i][j] - s;
    }
  double trDDchi = 0.0, dchi2 = 0.0;
  for (int l = 0; l < 3; l++)
    for (int m = 0; m < 3; m++) {
      trDDchi += gu[l][m] * DDchi[l][m];
      dchi2 += gu[l][m] * dchi[l] * dchi[m];
    }

  /* Ricci tensor: conformal part plus chi part */
  double R[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double t1 = 0.0, t2 = 0.0, t3 = 0.0, t4 = 0.0;
      for (int l = 0; l < 3; l++)
        for (int m = 0; m < 3; m++) t1 += gu[l][m] * d2[GT + SYM[i][j]][l][m];
      t1 = -0.5 * t1;
      for (int k = 0; k < 3; k++) t2 += gt[k][i] * dGam[k][j] + gt[k][j] * dGam[k][i];
      t2 = 0.5 * t2;
      for (int k = 0; k < 3; k++) t3 += Gd[k] * (cdl[i][j][k] + cdl[j][i][k]);
      t3 = 0.5 * t3;
      for (int l = 0; l < 3; l++)
        for (int m = 0; m < 3; m++) {
          double s = 0.0;
          for (int k = 0; k < 3; k++)
            s += cdu[k][l][i] * cdl[j][k][m] + cdu[k][l][j] * cdl[i][k][m] +
                 cdu[k][i][m] * cdl[k][l][j];
          t4 += gu[l][m] * s;
        }
      const double Rt = t1 + t2 + t3 + t4;
      const double Rchi = (DDchi[i][j] + gt[i][j] * trDDchi) / (2.0 * chi) -
                          (dchi[i] * dchi[j] + 3.0 * gt[i][j] * dchi2) / (4.0 * chi * chi);
      R[i][j] = Rt + Rchi;
    }
  double Rsc = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) Rsc += gu[i][j] * R[i][j];
  Rsc = chi * Rsc;

  /* physical Christoffels and the covariant second derivative of the lapse */
  double DDalp[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double s = 0.0;
      for (int k = 0; k < 3; k++) {
        double gul = 0.0;
        for (int l = 0; l < 3; l++) gul += gu[k][l] * dchi[l];
        const double dik = (k == i) ? 1.0 : 0.0, djk = (k == j) ? 1.0 : 0.0;
        const double Gphys =
            cdu[k][i][j] - (dik * dchi[j] + djk * dchi[i] - gt[i][j] * gul) / (2.0 * chi);
        s += Gphys * dalp[k];
      }
      DDalp[i][j] = d2[ALP][i][j] - s;
    }
  double lapalp = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) lapalp += gu[i][j] * DDalp[i][j];
  lapalp = chi * lapalp;

  /* traceless extrinsic curvature with indices raised by gu */
  double Atm[3][3], Atu[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double s = 0.0;
      for (int k = 0; k < 3; k++) s += gu[i][k] * At[k][j];
      Atm[i][j] = s; /* At^i_j */
    }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double s = 0.0;
      for (int k = 0; k < 3; k++) s += Atm[i][k] * gu[k][j];
      Atu[i][j] = s; /* At^ij */
    }
  double AtAt = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) AtAt += Atm[i][j] * Atm[j][i];

  /* trace-free part of -D_i D_j alpha + alpha R_ij */
  double X[3][3], trX = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) X[i][j] = -DDalp[i][j] + alpha * R[i][j];
  for (int k = 0; k < 3; k++)
    for (int l = 0; l < 3; l++) trX += gu[k][l] * X[k][l];

  if (cons) {
    /* Hamiltonian and momentum constraints (centred stencils only) */
    cons[0] = Rsc + (2.0 / 3.0) * trK * trK - AtAt;
    for (int i = 0; i < 3; i++) {
      double s = 0.0;
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
          for (int j = 0; j < 3; j++) {
            double DAt = d1[AT + SYM[a][b]][j];
            for (int m = 0; m < 3; m++) DAt -= cdu[m][j][a] * At[m][b] + cdu[m][j][b] * At[a][m];
            s += gu[i][a] * gu[j][b] * DAt;
          }
      double s2 = 0.0, s3 = 0.0;
      for (int j = 0; j < 3; j++) {
        s2 += gu[i][j] * dK[j];
        s3 += Atu[i][j] * dchi[j];
      }
      cons[1 + i] = s - (2.0 / 3.0) * s2 - 1.5 * s3 / chi;
    }
  }
  if (!out) return;

  /* phase 3: right-hand sides */
  out[CHI] = adv[CHI] + (2.0 / 3.0) * chi * (alpha * trK - divbeta);
  for (int i = 0; i < 3; i++)
    for (int j = i; j < 3; j++) {
      double s1 = 0.0, s2 = 0.0, s3 = 0.0;
      for (int k = 0; k < 3; k++) {
        s1 += gt[i][k] * dbeta[k][j];
        s2 += gt[j][k] * dbeta[k][i];
        s3 += At[i][k] * Atm[k][j];
      }
      out[GT + SYM[i][j]] =
          adv[GT + SYM[i][j]] - 2.0 * alpha * At[i][j] + s1 + s2 - (2.0 / 3.0) * gt[i][j] * divbeta;
      double a1 = 0.0, a2 = 0.0;
      for (int k = 0; k < 3; k++) {
        a1 += At[i][k] * dbeta[k][j];
        a2 += At[j][k] * dbeta[k][i];
      }
      const double XTF = X[i][j] - gt[i][j] * trX / 3.0;
      out[AT + SYM[i][j]] = adv[AT + SYM[i][j]] + chi * XTF +
                            alpha * (trK * At[i][j] - 2.0 * s3) + a1 + a2 -
                            (2.0 / 3.0) * At[i][j] * divbeta;
    }
  out[TRK] = adv[TRK] - lapalp + alpha * (AtAt + trK * trK / 3.0);

  double Gnoadv[3];
  for (int i = 0; i < 3; i++) {
    double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0, s5 = 0.0, s6 = 0.0, s7 = 0.0;
    for (int k = 0; k < 3; k++) s1 += Gd[k] * dbeta[i][k];
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++) {
        s2 += gu[j][k] * d2[BETA + i][j][k];
        s4 += cdu[i][j][k] * Atu[j][k];
      }
    for (int j = 0; j < 3; j++) {
      double dd = 0.0;
      for (int k = 0; k < 3; k++) dd += d2[BETA + k][j][k];
      s3 += gu[i][j] * dd;
      s5 += Atu[i][j] * dalp[j];
      s6 += Atu[i][j] * dchi[j];
      s7 += gu[i][j] * dK[j];
    }
    Gnoadv[i] = -s1 + (2.0 / 3.0) * Gd[i] * divbeta + s2 + s3 / 3.0 - 2.0 * s5 +
                2.0 * alpha * (s4 - 1.5 * s6 / chi - (2.0 / 3.0) * s7);
    out[GAM + i] = adv[GAM + i] + Gnoadv[i];
  }

  /* gauge */
  if (p->slicing == 1)
    out[ALP] = adv[ALP] - alpha * alpha * trK;
  else
    out[ALP] = adv[ALP] - 2.0 * alpha * trK;
  for (int i = 0; i < 3; i++) {
    if (p->shift == 1) {
      out[BETA + i] = adv[BETA + i] + p->shift_F * u[BB + i];
      out[BB + i] = adv[BB + i] + Gnoadv[i] - p->eta * u[BB + i];
    } else {
      out[BETA + i] = 0.0;
      out[BB + i] = 0.0;
    }
  }

  /* dissipation */
  for (int v = 0; v < NB; v++) {
    const int frozen = p->shift != 1 && v >= BETA;
    if (!frozen) out[v] += diss[v];
  }
}

void orc_bssn_rhs(const orc_params* p, const double* y, double* r) {
  geom G = mkgeom(p);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < G.n[2]; k++)
    for (int j = 0; j < G.n[1]; j++)
      for (int i = 0; i < G.n[0]; i++) {
        const long q = idx(&G, i, j, k);
        double o[NB];
        bssn_point(p, &G, y, q, o, NULL);
        for (int v = 0; v < NB; v++) r[v * G.npts + q] = o[v];
      }
}

/* Hamiltonian and momentum constraints; hm (4 grid functions, may be NULL)
 * receives H, M^1, M^2, M^3 at interior points; norms[c] = sqrt(mean over
 * interior points of the square), summed plane by plane in a fixed order. */
void orc_bssn_constraints(const orc_params* p, const double* y, double* hm,
                          double norms[4]) {
  geom G = mkgeom(p);
  const int nz = G.n[2];
  double* plane = calloc((size_t)nz * 4, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; k++)
    for (int j = 0; j < G.n[1]; j++)
      for (int i = 0; i < G.n[0]; i++) {
        const long q = idx(&G, i, j, k);
        double c[4];
        bssn_point(p, &G, y, q, NULL, c);
        for (int v = 0; v < 4; v++) {
          if (hm) hm[v * G.npts + q] = c[v];
          plane[k * 4 + v] += c[v] * c[v];
        }
      }
  const double npts = (double)G.n[0] * G.n[1] * G.n[2];
  for (int v = 0; v < 4; v++) {
    double s = 0.0;
    for (int k = 0; k < nz; k++) s += plane[k * 4 + v];
    norms[v] = sqrt(s / npts);
  }
  free(plane);
}

/* ------------------------------------------------------------------------ */
/* Classical RK4 method of lines (Sec. II: the time-integrator thorn).
 * Ghosts are refilled before every right-hand-side evaluation, analytic
 * ghosts at the stage time t_n + c_s dt with c = (0, 1/2, 1/2, 1).        */

static void rhs(const orc_params* p, int system, const double* y, double* r) {
  if (system == ORC_WAVE)
    orc_wave_rhs(p, y, r);
  else if (system == ORC_WAVE5)
    orc_wave5_rhs(p, y, r);
  else
    orc_bssn_rhs(p, y, r);
}

/* out = y + c * k on interior points */
static void axpy_interior(const geom* G, int nvar, const double* y, double c,
                          const double* k, double* out) {
  for (int v = 0; v < nvar; v++) {
    const long o = v * G->npts;
#pragma omp parallel for schedule(static)
    for (int kk = 0; kk < G->n[2]; kk++)
      for (int j = 0; j < G->n[1]; j++)
        for (int i = 0; i < G->n[0]; i++) {
          const long q = o + idx(G, i, j, kk);
          out[q] = y[q] + c * k[q];
        }
  }
}

/* Algebraic constraints of the conformal variables at one point (stride
 * between variables): rescale gt_ij by det(gt)^(-1/3) so that its
 * determinant is 1, then remove the trace of At_ij with respect to the
 * rescaled metric, At_ij -= gt_ij gt^kl At_kl / 3 (gt^kl = adjugate /
 * determinant). */
static void enforce_point(double* u, long stride) {
  double gt[3][3], At[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      gt[i][j] = u[(GT + SYM[i][j]) * stride];
      At[i][j] = u[(AT + SYM[i][j]) * stride];
    }
  const double det = gt[0][0] * (gt[1][1] * gt[2][2] - gt[1][2] * gt[2][1]) -
                     gt[0][1] * (gt[1][0] * gt[2][2] - gt[1][2] * gt[2][0]) +
                     gt[0][2] * (gt[1][0] * gt[2][1] - gt[1][1] * gt[2][0]);
  const double sc = 1.0 / cbrt(det);
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) gt[i][j] *= sc;
  const double det2 = gt[0][0] * (gt[1][1] * gt[2][2] - gt[1][2] * gt[2][1]) -
                      gt[0][1] * (gt[1][0] * gt[2][2] - gt[1][2] * gt[2][0]) +
                      gt[0][2] * (gt[1][0] * gt[2][1] - gt[1][1] * gt[2][0]);
  double tr = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      const double gu = (gt[(j + 1) % 3][(i + 1) % 3] * gt[(j + 2) % 3][(i + 2) % 3] -
                         gt[(j + 1) % 3][(i + 2) % 3] * gt[(j + 2) % 3][(i + 1) % 3]) /
                        det2;
      tr += gu * At[i][j];
    }
  for (int i = 0; i < 3; i++)
    for (int j = i; j < 3; j++) {
      u[(GT + SYM[i][j]) * stride] = gt[i][j];
      u[(AT + SYM[i][j]) * stride] = At[i][j] - gt[i][j] * tr / 3.0;
    }
}

/* enforce the algebraic constraints at every interior point */
void orc_bssn_enforce(const orc_params* p, double* y) {
  geom G = mkgeom(p);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < G.n[2]; k++)
    for (int j = 0; j < G.n[1]; j++)
      for (int i = 0; i < G.n[0]; i++) enforce_point(y + idx(&G, i, j, k), G.npts);
}

static void maybe_enforce(const orc_params* p, int system, double* y) {
  if (system == ORC_BSSN && p->enforce) orc_bssn_enforce(p, y);
}

int orc_prolong(const orc_params* cp, const double* const* yc, const double* times, int ntimes,
                double t, const orc_params* fp, double* yf, int nvar);

/* where the ghost zones of each RK stage come from: the boundary condition
 * bc, or (coarse != NULL) prolongation from ntimes coarse time levels at the
 * stage time (Sec. IV: a refined block's ghosts come from the next coarser
 * level) */
typedef struct {
  int bc;
  const orc_params* coarse;
  const double* const* yc;
  const double* times;
  int ntimes;
} ghost_source;

static int stage_ghosts(const orc_params* p, int system, const ghost_source* gs, double t,
                        double* y) {
  if (!gs->coarse) {
    fill_ghosts(p, system, gs->bc, t, y);
    return 0;
  }
  return orc_prolong(gs->coarse, gs->yc, gs->times, gs->ntimes, t, p, y, nvars_of(system));
}

/* the classical RK4 method of lines, ghosts of every stage from gs at the
 * stage's time (t, t + dt/2, t + dt/2, t + dt, then t + dt for the result) */
static int rk4_steps(const orc_params* p, int system, const ghost_source* gs, double* y,
                     double t, double dt, int nsteps) {
  geom G = mkgeom(p);
  const int nvar = nvars_of(system);
  const size_t N = (size_t)nvar * G.npts;
  double* ys = calloc(N, sizeof(double));
  double* k1 = calloc(N, sizeof(double));
  double* k2 = calloc(N, sizeof(double));
  double* k3 = calloc(N, sizeof(double));
  double* k4 = calloc(N, sizeof(double));
  int fail = 0;
  if (!ys || !k1 || !k2 || !k3 || !k4) {
    free(ys); free(k1); free(k2); free(k3); free(k4);
    return 1;
  }
  memcpy(ys, y, N * sizeof(double));
  for (int n = 0; n < nsteps && !fail; n++) {
    fail |= stage_ghosts(p, system, gs, t, y);
    rhs(p, system, y, k1);
    axpy_interior(&G, nvar, y, 0.5 * dt, k1, ys);
    maybe_enforce(p, system, ys);
    fail |= stage_ghosts(p, system, gs, t + 0.5 * dt, ys);
    rhs(p, system, ys, k2);
    axpy_interior(&G, nvar, y, 0.5 * dt, k2, ys);
    maybe_enforce(p, system, ys);
    fail |= stage_ghosts(p, system, gs, t + 0.5 * dt, ys);
    rhs(p, system, ys, k3);
    axpy_interior(&G, nvar, y, dt, k3, ys);
    maybe_enforce(p, system, ys);
    fail |= stage_ghosts(p, system, gs, t + dt, ys);
    rhs(p, system, ys, k4);
    for (int v = 0; v < nvar; v++) {
      const long o = v * G.npts;
#pragma omp parallel for schedule(static)
      for (int kk = 0; kk < G.n[2]; kk++)
        for (int j = 0; j < G.n[1]; j++)
          for (int i = 0; i < G.n[0]; i++) {
            const long q = o + idx(&G, i, j, kk);
            y[q] = y[q] + (dt / 6.0) * (((k1[q] + 2.0 * k2[q]) + 2.0 * k3[q]) + k4[q]);
          }
    }
    maybe_enforce(p, system, y);
    t = t + dt;
  }
  if (!fail) fail |= stage_ghosts(p, system, gs, t, y);
  free(ys); free(k1); free(k2); free(k3); free(k4);
  return fail;
}

int orc_rk4(const orc_params* p, int system, int bc, double* y, double t, double dt,
            int nsteps) {
  const ghost_source gs = {bc, NULL, NULL, NULL, 0};
  return rk4_steps(p, system, &gs, y, t, dt, nsteps);
}

int orc_rk4_prolong(const orc_params* p, int system, double* y, double t, double dt, int nsteps,
                    const orc_params* coarse, const double* const* yc, const double* times,
                    int ntimes) {
  if (!coarse || !yc || !times) return 1;
  const ghost_source gs = {0, coarse, yc, times, ntimes};
  return rk4_steps(p, system, &gs, y, t, dt, nsteps);
}

/* ------------------------------------------------------------------------ */
/* single stencil probe on interior points, for checking the operators on
 * their own: kind 1 = centred first derivative along a; kind 2 = centred
 * second derivative d_a d_b (pure when a == b, mixed otherwise); kind 3 =
 * lopsided derivative along a, upwind side from the sign of sgn (NULL: +);
 * kind 4 = sixth difference along a (the Kreiss-Oliger stencil, unscaled). */
void orc_stencil(const orc_params* p, const double* f, int kind, int a, int b,
                 const double* sgn, double* out) {
  geom G = mkgeom(p);
  const long st[3] = {1, G.sy, G.sz};
#pragma omp parallel for schedule(static)
  for (int k = 0; k < G.n[2]; k++)
    for (int j = 0; j < G.n[1]; j++)
      for (int i = 0; i < G.n[0]; i++) {
        const long q = idx(&G, i, j, k);
        double v;
        if (kind == 1)
          v = D1(p->fd_order, f + q, st[a], p->h[a]);
        else if (kind == 2)
          v = (a == b) ? D2(p->fd_order, f + q, st[a], p->h[a])
                       : D11(p->fd_order, f + q, st[a], st[b], p->h[a], p->h[b]);
        else if (kind == 3)
          v = DUP(p->fd_order, f + q, st[a], p->h[a], sgn ? sgn[q] : 1.0);
        else
          v = delta6(f + q, st[a]);
        out[q] = v;
      }
}

/* ------------------------------------------------------------------------ */
/* Two refinement levels (Sec. IV: Carpet's mesh refinement couples patches
 * of different resolution through their ghost zones).  Refinement ratio 2:
 * h_coarse = 2 h_fine on every axis, and every fine point either coincides
 * with a coarse point or lies half-way between two.
 *
 * Prolongation fills every ghost point of the fine block from the coarse
 * block (whose ghosts must be valid): per axis, a coincident point takes the
 * coarse value, a half-way point the degree-5 Lagrange interpolant through
 * the coarse points at offsets -2 .. 3 around it, weights
 * (3, -25, 150, 150, -25, 3) / 256; the tensor product over the three axes,
 * summed z outermost, x innermost.  With several coarse time levels y_l at
 * times t_l the spatial interpolants are combined with the Lagrange weights
 * in time, prod_{m != l} (t - t_m) / (t_l - t_m), at the requested time t.
 *
 * Restriction copies fine values into every coarse interior point that
 * coincides with a fine interior point (injection).
 *
 * Both return 1 (and do nothing) if the spacings are not in ratio 2, the
 * fine points are not aligned with the coarse ones, or (prolongation) a
 * coarse stencil point lies outside the coarse block's extended range.   */

static int axis_map(const orc_params* c, const orc_params* f, int d, int i, int* base,
                    int* half) {
  const double r = (f->origin[d] + i * f->h[d] - c->origin[d]) / c->h[d];
  const double fl = floor(r + 1e-9);
  const double fr = r - fl;
  if (fabs(fr) < 1e-9) {
    *half = 0;
  } else if (fabs(fr - 0.5) < 1e-9) {
    *half = 1;
  } else {
    return 1;
  }
  *base = (int)fl;
  return 0;
}

static int check_levels(const orc_params* c, const orc_params* f) {
  for (int d = 0; d < 3; d++) {
    if (fabs(c->h[d] - 2.0 * f->h[d]) > 1e-12 * c->h[d]) return 1;
    const double off = (f->origin[d] - c->origin[d]) / f->h[d];
    if (fabs(off - floor(off + 0.5)) > 1e-9) return 1;
  }
  return 0;
}

int orc_prolong(const orc_params* cp, const double* const* yc, const double* times, int ntimes,
                double t, const orc_params* fp, double* yf, int nvar) {
  if (check_levels(cp, fp)) return 1;
  if (ntimes < 1 || ntimes > 3) return 1;
  double wt[3];
  for (int l = 0; l < ntimes; l++) {
    wt[l] = 1.0;
    for (int m = 0; m < ntimes; m++)
      if (m != l) {
        if (times[l] == times[m]) return 1;
        wt[l] *= (t - times[m]) / (times[l] - times[m]);
      }
  }
  const geom C = mkgeom(cp), F = mkgeom(fp);
  static const double W[6] = {3.0 / 256, -25.0 / 256, 150.0 / 256,
                              150.0 / 256, -25.0 / 256, 3.0 / 256};
  /* reach check over the fine extended range */
  for (int d = 0; d < 3; d++)
    for (int i = -F.g; i < F.n[d] + F.g; i++) {
      int b, hf;
      if (axis_map(cp, fp, d, i, &b, &hf)) return 1;
      const int lo = hf ? b - 2 : b, hi = hf ? b + 3 : b;
      if (lo < -C.g || hi >= C.n[d] + C.g) return 1;
    }
  int fail = 0;
#pragma omp parallel for schedule(static) reduction(| : fail)
  for (int k = -F.g; k < F.n[2] + F.g; k++)
    for (int j = -F.g; j < F.n[1] + F.g; j++)
      for (int i = -F.g; i < F.n[0] + F.g; i++) {
        if (is_interior(&F, i, j, k)) continue;
        const int ii[3] = {i, j, k};
        int b[3], hf[3], cnt[3];
        double w[3][6];
        for (int d = 0; d < 3; d++) {
          fail |= axis_map(cp, fp, d, ii[d], &b[d], &hf[d]);
          if (hf[d]) {
            cnt[d] = 6;
            for (int m = 0; m < 6; m++) w[d][m] = W[m];
            b[d] -= 2;
          } else {
            cnt[d] = 1;
            w[d][0] = 1.0;
          }
        }
        for (int v = 0; v < nvar; v++) {
          double val = 0.0;
          for (int l = 0; l < ntimes; l++) {
            const double* src = yc[l] + (long)v * C.npts;
            double acc = 0.0;
            for (int c = 0; c < cnt[2]; c++)
              for (int bb = 0; bb < cnt[1]; bb++)
                for (int a = 0; a < cnt[0]; a++)
                  acc += w[2][c] * w[1][bb] * w[0][a] *
                         src[idx(&C, b[0] + a, b[1] + bb, b[2] + c)];
            val += wt[l] * acc;
          }
          yf[(long)v * F.npts + idx(&F, i, j, k)] = val;
        }
      }
  return fail;
}

int orc_restrict(const orc_params* cp, double* yc, const orc_params* fp, const double* yf,
                 int nvar) {
  if (check_levels(cp, fp)) return 1;
  const geom C = mkgeom(cp), F = mkgeom(fp);
  for (int k = 0; k < C.n[2]; k++)
    for (int j = 0; j < C.n[1]; j++)
      for (int i = 0; i < C.n[0]; i++) {
        const int ii[3] = {i, j, k};
        int fi[3], inside = 1;
        for (int d = 0; d < 3; d++) {
          const double r = (cp->origin[d] + ii[d] * cp->h[d] - fp->origin[d]) / fp->h[d];
          fi[d] = (int)floor(r + 0.5);
          if (fabs(r - fi[d]) > 1e-9 || fi[d] < 0 || fi[d] >= F.n[d]) inside = 0;
        }
        if (!inside) continue;
        for (int v = 0; v < nvar; v++)
          yc[(long)v * C.npts + idx(&C, i, j, k)] =
              yf[(long)v * F.npts + idx(&F, fi[0], fi[1], fi[2])];
      }
  return 0;
}
