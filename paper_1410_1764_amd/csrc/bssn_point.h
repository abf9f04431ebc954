// bssn_point.h -- device code for the BSSN right-hand side at one grid point
// (the Einstein equations evolved in Sec. III.D of arXiv:1410.1764, "several
// thousand floating point operations ... at a single grid point"), shared by
// the single-block kernels and the persistent batch kernel.
//
// System (chi variant of BSSN; state chi, gt_ij, trK, At_ij, Gamt^i, alpha,
// beta^i, B^i):
//   dt chi   = A(chi) + 2/3 chi (alpha K - div beta)
//   dt gt_ij = A(gt_ij) - 2 alpha At_ij + gt_ik d_j beta^k + gt_jk d_i beta^k
//              - 2/3 gt_ij div beta
//   dt K     = A(K) - D^2 alpha + alpha (At^ij At_ij + K^2/3)
//   dt At_ij = A(At_ij) + chi [-D_i D_j alpha + alpha R_ij]^TF
//              + alpha (K At_ij - 2 At_ik At^k_j) + At_ik d_j beta^k
//              + At_jk d_i beta^k - 2/3 At_ij div beta
//   dt Gt^i  = A(Gt^i) - Gd^k d_k beta^i + 2/3 Gd^i div beta
//              + gt^jk d_j d_k beta^i + 1/3 gt^ij d_j d_k beta^k
//              - 2 At^ij d_j alpha
//              + 2 alpha (Gt^i_jk At^jk - 3/2 At^ij d_j chi / chi - 2/3 gt^ij d_j K)
//   gauge: dt alpha = A(alpha) - 2 alpha K (1+log) or - alpha^2 K (harmonic);
//          Gamma-driver dt beta^i = A(beta^i) + F B^i,
//          dt B^i = A(B^i) + [dt Gt^i - A(Gt^i)] - eta B^i; frozen: 0.
// A(f) = beta^k d_k f with lopsided (upwind) derivatives; Gd^i = gt^jk Gt^i_jk
// recomputed from gt (the evolved Gamt^i enters only differentiated and
// advected); R_ij = conformal Ricci + chi part.
//
// Evaluation order is chosen for register pressure ("consume derivatives as
// they are produced"): the second derivatives of gt_ij are contracted into
// R_ij right after they are formed, the 18 Christoffels are built from the
// 18 first derivatives of gt and those are dropped, and so on.  Each
// variable's stencil values are loaded once and shared by its centred,
// second and lopsided derivatives.
//
// Precision: T is double (FP64) or float (MIXED).  Differences of neighbour
// values are formed in double, then weighted and combined in T.
#pragma once

#include "internal.h"

namespace chemora {

enum : int {
  V_CHI = 0, V_GT = 1, V_TRK = 7, V_AT = 8, V_GAM = 14, V_ALP = 17, V_BETA = 18, V_B = 21,
  V_N = 24
};

// Scheduling fences.  Without them the compiler issues the ~700 stencil
// loads of a point ahead of the arithmetic that consumes them and spills
// several KB per lane to scratch.  pin() is an empty asm that claims to
// rewrite x in a VGPR: the value must exist at that point, so the
// arithmetic producing it cannot sink below the next group's loads, which
// in turn cannot rise above the memory fence.  No instruction is emitted.
// CHEMORA_BSSN_FENCE selects the policy (an ablation switch; every level
// computes the same values): 3 = also after each mixed derivative (the
// register-capped split kernels), 2 = fence after every stencil group
// (default), 1 = fence once per grid function, 0 = no fences.
#ifndef CHEMORA_BSSN_FENCE
#define CHEMORA_BSSN_FENCE 2
#endif
template <typename T>
__device__ __forceinline__ void pin(T& x) {
  asm volatile("" : "+v"(x));
}
__device__ __forceinline__ void fence_memory() { asm volatile("" ::: "memory"); }

// index of the symmetric pair (i, j) in (xx, xy, xz, yy, yz, zz); closed
// form so that it folds to a constant inside unrolled loops
__host__ __device__ constexpr int sidx(int i, int j) {
  return (i < j ? i : j) * (5 - (i < j ? i : j)) / 2 + (i < j ? j : i);
}

// Stencil weights for one block: the stencils' integer weights are applied
// in the code, these carry the common denominators (order 4: 12, 12 and
// 144; order 6: 60, 180, 3600; order 8: 840, 5040, 840^2).
struct Weights {
  double w1[3];   // first derivatives (centred and lopsided): 1 / (den1 h_d)
  double w2[3];   // pure second derivatives: 1 / (den2 h_d^2)
  double w11[3];  // mixed: 1 / (den1^2 h_a h_b) for (x,y), (x,z), (y,z)
  double ko[3];   // Kreiss-Oliger: sigma / (64 h_d), all 0 when off
};

inline Weights make_weights(const double h[3], double ko_sigma = 0.0, int order = 4) {
  const double den1 = order == 8 ? 840.0 : (order == 6 ? 60.0 : 12.0);
  const double den2 = order == 8 ? 5040.0 : (order == 6 ? 180.0 : 12.0);
  Weights w;
  for (int d = 0; d < 3; ++d) {
    w.w1[d] = 1.0 / (den1 * h[d]);
    w.w2[d] = 1.0 / (den2 * h[d] * h[d]);
    w.ko[d] = ko_sigma / (64.0 * h[d]);
  }
  w.w11[0] = 1.0 / (den1 * den1 * h[0] * h[1]);
  w.w11[1] = 1.0 / (den1 * den1 * h[0] * h[2]);
  w.w11[2] = 1.0 / (den1 * den1 * h[1] * h[2]);
  return w;
}

// Integer weights of the 6th- and 8th-order operators (order 4 is written
// out in axis_derivs): centred first derivative A_k on f_k - f_-k and
// second derivative B_k on (f_k - f0) + (f_-k - f0), k = 1..M; lopsided
// first derivative U on f_k - f0 at offsets k = -(M-1) .. M+1 towards the
// upwind side (index k + M - 1; the centre's weight is implied).  Each is
// the unique stencil on its points exact for polynomials up to the order.
template <int ORD>
struct FDC;
template <>
struct FDC<6> {
  static constexpr int M = 3;
  static constexpr double A[3] = {45.0, -9.0, 1.0};
  static constexpr double B[3] = {270.0, -27.0, 2.0};
  static constexpr double U[7] = {2.0, -24.0, -35.0, 80.0, -30.0, 8.0, -1.0};
};
template <>
struct FDC<8> {
  static constexpr int M = 4;
  static constexpr double A[4] = {672.0, -168.0, 32.0, -3.0};
  static constexpr double B[4] = {8064.0, -1008.0, 128.0, -9.0};
  static constexpr double U[9] = {-5.0, 60.0, -420.0, -378.0, 1050.0, -420.0, 140.0, -30.0, 3.0};
};

// Stencil accessors.  A grid function's neighbourhood is read through an
// accessor f(dx, dy, dz) (offsets from the point; compile-time constants
// once the loops are unrolled) and f.sel(up, dx, dy, dz), the value at
// +(dx,dy,dz) if up else at -(dx,dy,dz) (one load through a selected
// address).  GAcc reads global memory; the LDS tile accessor is in
// bssn_lds.h.
struct GAcc {
  const double* f;  // centre value
  long long sy, sz;
  __device__ __forceinline__ double operator()(int dx, int dy, int dz) const {
    return f[dx + dy * sy + dz * sz];
  }
  __device__ __forceinline__ double sel(bool up, int dx, int dy, int dz) const {
    const long long o = dx + dy * sy + dz * sz;
    return f[up ? o : -o];
  }
};

// Source of all 24 grid functions at one point, reading global memory:
// center(v) is the value of variable v at the point, acquire(v) the
// accessor of its neighbourhood.  Sources are acquired in a fixed order
// (the LDS source stages them one by one).
struct GSrc {
  const double* Y;  // centre value of variable 0
  long long sv, sy, sz;
  __device__ __forceinline__ double center(int v) const { return Y[v * sv]; }
  __device__ __forceinline__ GAcc acquire(int v) { return GAcc{Y + v * sv, sy, sz}; }
};

// Centred first derivatives (D1), pure second derivatives (D2) and the
// advection term beta^k d_k f with the lopsided stencil on the upwind side
// (ADV) of one grid function.
// KOM: Kreiss-Oliger mode of the advected variables: 0 off, 1 on, 2 decided
// at run time (w.ko != 0), for kernels that keep one instance for both.
enum : int { KO_OFF = 0, KO_ON = 1, KO_RUNTIME = 2 };

template <typename T, bool D1, bool D2, bool ADV, int KOM, typename Acc>
__device__ __forceinline__ void axis_derivs4(const Acc& f, const Weights& w, const bool bpos[3],
                                            const T beta[3], T d1[3], T d2[3], T& adv) {
  const double f0 = f(0, 0, 0);
  adv = (T)0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int ex = d == 0, ey = d == 1, ez = d == 2;
    const double m1 = f(-ex, -ey, -ez), p1 = f(ex, ey, ez);
    const double m2 = f(-2 * ex, -2 * ey, -2 * ez), p2 = f(2 * ex, 2 * ey, 2 * ez);
    if (D1) d1[d] = ((T)8 * (T)(p1 - m1) - (T)(p2 - m2)) * (T)w.w1[d];
    if (D2)
      d2[d] = ((T)16 * (T)((p1 - f0) + (m1 - f0)) - (T)((p2 - f0) + (m2 - f0))) * (T)w.w2[d];
    if (ADV) {
      const bool up = bpos[d];
      const double u1 = up ? p1 : m1, um1 = up ? m1 : p1, u2 = up ? p2 : m2;
      const double u3 = f.sel(up, 3 * ex, 3 * ey, 3 * ez);
      T l = ((T)18 * (T)(u1 - f0) - (T)3 * (T)(um1 - f0) - (T)6 * (T)(u2 - f0) + (T)(u3 - f0)) *
            (T)w.w1[d];
      l = up ? l : -l;
      adv += beta[d] * l;
    }
  }
  // Kreiss-Oliger dissipation rides on the advection term (every evolved
  // variable has one): sigma/64 sum_d delta6_d f / h_d, the sixth difference
  // on neighbour differences.
  if (ADV && (KOM == KO_ON || (KOM == KO_RUNTIME && w.ko[0] != 0.0))) {
    T ko = (T)0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int ex = d == 0, ey = d == 1, ez = d == 2;
      const double s1 = (f(ex, ey, ez) - f0) + (f(-ex, -ey, -ez) - f0);
      const double s2 = (f(2 * ex, 2 * ey, 2 * ez) - f0) + (f(-2 * ex, -2 * ey, -2 * ez) - f0);
      const double s3 = (f(3 * ex, 3 * ey, 3 * ez) - f0) + (f(-3 * ex, -3 * ey, -3 * ez) - f0);
      ko += (((T)s3 - (T)6 * (T)s2) + (T)15 * (T)s1) * (T)w.ko[d];
    }
    adv += ko;
  }
  if (CHEMORA_BSSN_FENCE >= 2 || (CHEMORA_BSSN_FENCE == 1 && !D2)) {
    if (D1) {
      pin(d1[0]);
      pin(d1[1]);
      pin(d1[2]);
    }
    if (D2) {
      pin(d2[0]);
      pin(d2[1]);
      pin(d2[2]);
    }
    if (ADV) pin(adv);
    fence_memory();
  }
}

// The same derivatives at order 6 or 8 (cached-load kernels only; no
// dissipation at these orders).  Sums run over increasing offsets.
template <typename T, bool D1, bool D2, bool ADV, int ORD, typename Acc>
__device__ __forceinline__ void axis_derivs_hi(const Acc& f, const Weights& w,
                                               const bool bpos[3], const T beta[3], T d1[3],
                                               T d2[3], T& adv) {
  using C = FDC<ORD>;
  const double f0 = f(0, 0, 0);
  adv = (T)0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int ex = d == 0, ey = d == 1, ez = d == 2;
    if (D1) {
      T acc = (T)0;
#pragma unroll
      for (int k = 1; k <= C::M; ++k)
        acc += (T)C::A[k - 1] * (T)(f(k * ex, k * ey, k * ez) - f(-k * ex, -k * ey, -k * ez));
      d1[d] = acc * (T)w.w1[d];
    }
    if (D2) {
      T acc = (T)0;
#pragma unroll
      for (int k = 1; k <= C::M; ++k)
        acc += (T)C::B[k - 1] *
               (T)((f(k * ex, k * ey, k * ez) - f0) + (f(-k * ex, -k * ey, -k * ez) - f0));
      d2[d] = acc * (T)w.w2[d];
    }
    if (ADV) {
      const bool up = bpos[d];
      T acc = (T)0;
#pragma unroll
      for (int k = -(C::M - 1); k <= C::M + 1; ++k)
        if (k != 0) acc += (T)C::U[k + C::M - 1] * (T)(f.sel(up, k * ex, k * ey, k * ez) - f0);
      T l = acc * (T)w.w1[d];
      l = up ? l : -l;
      adv += beta[d] * l;
    }
  }
  if (CHEMORA_BSSN_FENCE >= 2 || (CHEMORA_BSSN_FENCE == 1 && !D2)) {
    if (D1) {
      pin(d1[0]);
      pin(d1[1]);
      pin(d1[2]);
    }
    if (D2) {
      pin(d2[0]);
      pin(d2[1]);
      pin(d2[2]);
    }
    if (ADV) pin(adv);
    fence_memory();
  }
}

// ORD: finite-difference order (4, 6 or 8)
template <typename T, bool D1, bool D2, bool ADV, int KOM, int ORD = 4, typename Acc>
__device__ __forceinline__ void axis_derivs(const Acc& f, const Weights& w, const bool bpos[3],
                                            const T beta[3], T d1[3], T d2[3], T& adv) {
  if constexpr (ORD == 4)
    axis_derivs4<T, D1, D2, ADV, KOM>(f, w, bpos, beta, d1, d2, adv);
  else
    axis_derivs_hi<T, D1, D2, ADV, ORD>(f, w, bpos, beta, d1, d2, adv);
}

// Mixed derivative d_a d_b f (a < b): first-derivative stencil along both
// axes, q_mn = [f(m,n) - f(-m,n)] - [f(m,-n) - f(-m,-n)], weights 8 / -1.
template <typename T, int ORD = 4, typename Acc>
__device__ __forceinline__ T mixed_deriv(const Acc& f, int a, int b, double wab) {
  // value at alpha e_a + beta e_b
  auto at = [&](int alpha, int beta) {
    return f(alpha * (a == 0) + beta * (b == 0), alpha * (a == 1) + beta * (b == 1),
             alpha * (a == 2) + beta * (b == 2));
  };
  if constexpr (ORD != 4) {  // sum over (i, j) of A_i A_j q_ij, increasing i then j
    using C = FDC<ORD>;
    T acc = (T)0;
#pragma unroll
    for (int i = 1; i <= C::M; ++i)
#pragma unroll
      for (int j = 1; j <= C::M; ++j)
        acc += (T)(C::A[i - 1] * C::A[j - 1]) *
               (T)((at(i, j) - at(-i, j)) - (at(i, -j) - at(-i, -j)));
    return acc * (T)wab;
  }
  double q[2][2];
#pragma unroll
  for (int m = 1; m <= 2; ++m)
#pragma unroll
    for (int n = 1; n <= 2; ++n)
      q[m - 1][n - 1] = (at(m, n) - at(-m, n)) - (at(m, -n) - at(-m, -n));
  return ((T)64 * (T)q[0][0] - (T)8 * (T)q[0][1] - (T)8 * (T)q[1][0] + (T)q[1][1]) * (T)wab;
}

// All six second derivatives d_a d_b f in symmetric order.
template <typename T, int ORD = 4, typename Acc>
__device__ __forceinline__ void second_derivs(const Acc& f, const Weights& w, const T d2pure[3],
                                              T dd[6]) {
  dd[0] = d2pure[0];
  dd[3] = d2pure[1];
  dd[5] = d2pure[2];
  dd[1] = mixed_deriv<T, ORD>(f, 0, 1, w.w11[0]);
  if (CHEMORA_BSSN_FENCE >= 3) {
    pin(dd[1]);
    fence_memory();
  }
  dd[2] = mixed_deriv<T, ORD>(f, 0, 2, w.w11[1]);
  if (CHEMORA_BSSN_FENCE >= 3) {
    pin(dd[2]);
    fence_memory();
  }
  dd[4] = mixed_deriv<T, ORD>(f, 1, 2, w.w11[2]);
  if (CHEMORA_BSSN_FENCE >= 1) {
    pin(dd[0]);
    pin(dd[1]);
    pin(dd[2]);
    pin(dd[3]);
    pin(dd[4]);
    pin(dd[5]);
    fence_memory();
  }
}

// Geometry shared by the right-hand side and the constraints: inverse
// conformal metric gu, Christoffels cdu (Gt^i_jk) and their contraction Gd,
// d_i chi, and the Ricci tensor R_ij (conformal part + chi part).  With ADV
// the advection terms of gt_ij, Gamt^i and chi are written to rhs[v] as
// well (rhs: a T[V_N] array, or any object whose operator[] gives a T&).
template <typename T, bool ADV, int KOM, int ORD, typename Src, typename Out>
__device__ __forceinline__ void bssn_geometry(Src& src, const Weights& w, const bool bpos[3],
                                              const T beta[3], const T gt[6], T gu[6],
                                              T cdu[3][6], T Gd[3], T dchi[3], T R[6],
                                              Out& rhs) {
  // ---- inverse conformal metric (adjugate / determinant)
  {
    const T c00 = gt[3] * gt[5] - gt[4] * gt[4];
    const T c01 = gt[2] * gt[4] - gt[1] * gt[5];
    const T c02 = gt[1] * gt[4] - gt[2] * gt[3];
    const T c11 = gt[0] * gt[5] - gt[2] * gt[2];
    const T c12 = gt[1] * gt[2] - gt[0] * gt[4];
    const T c22 = gt[0] * gt[3] - gt[1] * gt[1];
    const T idet = (T)1 / (gt[0] * c00 + gt[1] * c01 + gt[2] * c02);
    gu[0] = c00 * idet;
    gu[1] = c01 * idet;
    gu[2] = c02 * idet;
    gu[3] = c11 * idet;
    gu[4] = c12 * idet;
    gu[5] = c22 * idet;
  }

  T dd[6], dpure[3], adv;
  T dgt[6][3];

  // ---- gt_ij: first derivatives kept; second derivatives contracted into
  // R_ij = -1/2 gt^lm d_l d_m gt_ij right away; advection
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const auto f = src.acquire(V_GT + q);
    axis_derivs<T, true, true, ADV, KOM, ORD>(f, w, bpos, beta, dgt[q], dpure, adv);
    if (ADV) rhs[V_GT + q] = adv;
    second_derivs<T, ORD>(f, w, dpure, dd);
    R[q] = (T)(-0.5) * (gu[0] * dd[0] + gu[3] * dd[3] + gu[5] * dd[5] +
                        (T)2 * (gu[1] * dd[1] + gu[2] * dd[2] + gu[4] * dd[4]));
  }

  // ---- Christoffels of the conformal metric
  // cdl[i][jk] = 1/2 (d_j gt_ik + d_k gt_ij - d_i gt_jk); cdu = gt^il cdl[l]
  T cdl[3][6];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = j; k < 3; ++k)
        cdl[i][sidx(j, k)] =
            (T)0.5 * (dgt[sidx(i, k)][j] + dgt[sidx(i, j)][k] - dgt[sidx(j, k)][i]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int q = 0; q < 6; ++q)
      cdu[i][q] = gu[sidx(i, 0)] * cdl[0][q] + gu[sidx(i, 1)] * cdl[1][q] +
                  gu[sidx(i, 2)] * cdl[2][q];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    Gd[i] = gu[0] * cdu[i][0] + gu[3] * cdu[i][3] + gu[5] * cdu[i][5] +
            (T)2 * (gu[1] * cdu[i][1] + gu[2] * cdu[i][2] + gu[4] * cdu[i][4]);

  // ---- evolved Gamt^i: R_ij += 1/2 (gt_ki d_j Gt^k + gt_kj d_i Gt^k); advection
  {
    T dG[3][3];  // dG[k][j] = d_j Gt^k
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      axis_derivs<T, true, false, ADV, KOM, ORD>(src.acquire(V_GAM + k), w, bpos, beta, dG[k], dpure, adv);
      if (ADV) rhs[V_GAM + k] = adv;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        T s = (T)0;
#pragma unroll
        for (int k = 0; k < 3; ++k) s += gt[sidx(k, i)] * dG[k][j] + gt[sidx(k, j)] * dG[k][i];
        R[sidx(i, j)] += (T)0.5 * s;
      }
  }

  // ---- Christoffel products:
  // R_ij += 1/2 Gd^k (cdl_ijk + cdl_jik)
  //       + gt^lm (cdu^k_li cdl_jkm + cdu^k_lj cdl_ikm + cdu^k_im cdl_klj)
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      T s = (T)0;
#pragma unroll
      for (int k = 0; k < 3; ++k) s += Gd[k] * (cdl[i][sidx(j, k)] + cdl[j][sidx(i, k)]);
      T t = (T)0;
#pragma unroll
      for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          T u = (T)0;
#pragma unroll
          for (int k = 0; k < 3; ++k)
            u += cdu[k][sidx(l, i)] * cdl[j][sidx(k, m)] + cdu[k][sidx(l, j)] * cdl[i][sidx(k, m)] +
                 cdu[k][sidx(i, m)] * cdl[k][sidx(l, j)];
          t += gu[sidx(l, m)] * u;
        }
      R[sidx(i, j)] += (T)0.5 * s + t;
    }

  // ---- chi: D_i D_j chi = d_i d_j chi - Gt^k_ij d_k chi; chi part of R_ij
  {
    const auto f = src.acquire(V_CHI);
    // chi at the point, read from its own neighbourhood (the same value as
    // the centre load), so that it is not held through the metric phase
    const T chi = (T)f(0, 0, 0);
    axis_derivs<T, true, true, ADV, KOM, ORD>(f, w, bpos, beta, dchi, dpure, adv);
    if (ADV) rhs[V_CHI] = adv;
    second_derivs<T, ORD>(f, w, dpure, dd);
#pragma unroll
    for (int q = 0; q < 6; ++q)
      dd[q] -= cdu[0][q] * dchi[0] + cdu[1][q] * dchi[1] + cdu[2][q] * dchi[2];
    T trDD = gu[0] * dd[0] + gu[3] * dd[3] + gu[5] * dd[5] +
             (T)2 * (gu[1] * dd[1] + gu[2] * dd[2] + gu[4] * dd[4]);
    T dchi2 = (T)0;
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int m = 0; m < 3; ++m) dchi2 += gu[sidx(l, m)] * dchi[l] * dchi[m];
    const T i2chi = (T)0.5 / chi;
    const T i4chi2 = (T)0.25 / (chi * chi);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        const int q = sidx(i, j);
        R[q] += (dd[q] + gt[q] * trDD) * i2chi - (dchi[i] * dchi[j] + (T)3 * gt[q] * dchi2) * i4chi2;
      }
  }
}

// Order in which bssn_rhs_point acquires the neighbourhoods of the 24
// grid functions (a staging source prefetches them in this order).
__device__ constexpr int kRhsOrder[V_N] = {
    V_GT + 0, V_GT + 1, V_GT + 2, V_GT + 3, V_GT + 4, V_GT + 5, V_GAM + 0, V_GAM + 1,
    V_GAM + 2, V_CHI, V_ALP, V_BETA + 0, V_BETA + 1, V_BETA + 2, V_TRK, V_AT + 0,
    V_AT + 1, V_AT + 2, V_AT + 3, V_AT + 4, V_AT + 5, V_B + 0, V_B + 1, V_B + 2};

// Acquisition orders, as types for the staging sources: the right-hand
// side acquires all 24 grid functions (kRhsOrder); the constraints acquire
// the ones the geometry needs (gt, Gamt, chi), then K and At.
struct RhsOrder {
  static constexpr int N = V_N;
  __device__ static constexpr int at(int s) { return kRhsOrder[s]; }
};
__device__ constexpr int kConsOrder[17] = {V_GT + 0, V_GT + 1, V_GT + 2, V_GT + 3, V_GT + 4,
                                           V_GT + 5, V_GAM + 0, V_GAM + 1, V_GAM + 2, V_CHI,
                                           V_TRK, V_AT + 0, V_AT + 1, V_AT + 2, V_AT + 3,
                                           V_AT + 4, V_AT + 5};
struct ConsOrder {
  static constexpr int N = 17;
  __device__ static constexpr int at(int s) { return kConsOrder[s]; }
};

// Right-hand side of all 24 variables at one point, reading through src.
template <typename T, int KOM, int ORD = 4, typename Src>
__device__ __forceinline__ void bssn_rhs_point(Src& src, const Weights& w, const BssnPar& P,
                                               T rhs[V_N]) {
  // ---- centre values, upwind sides
  bool bpos[3];
  T beta[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double b = src.center(V_BETA + d);
    bpos[d] = b >= 0.0;
    beta[d] = (T)b;
  }
  const T chi = (T)src.center(V_CHI);
  const T trK = (T)src.center(V_TRK);
  const T alpha = (T)src.center(V_ALP);
  T gt[6], At[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    gt[q] = (T)src.center(V_GT + q);
    At[q] = (T)src.center(V_AT + q);
  }

  T gu[6], cdu[3][6], Gd[3], dchi[3], R[6];
  bssn_geometry<T, true, KOM, ORD>(src, w, bpos, beta, gt, gu, cdu, Gd, dchi, R, rhs);
  T dd[6], dpure[3], d1v[3], adv;

  // ---- lapse: D_i D_j alpha with the physical Christoffels
  // Gamma^k_ij = Gt^k_ij - (delta^k_i d_j chi + delta^k_j d_i chi - gt_ij gt^kl d_l chi) / (2 chi)
  T dalp[3];
  T lapalp;
  T X[6];
  {
    const auto f = src.acquire(V_ALP);
    axis_derivs<T, true, true, true, KOM, ORD>(f, w, bpos, beta, dalp, dpure, adv);
    rhs[V_ALP] = adv;
    second_derivs<T, ORD>(f, w, dpure, dd);
    const T i2chi = (T)0.5 / chi;
    T uchi[3];  // gt^kl d_l chi
#pragma unroll
    for (int k = 0; k < 3; ++k)
      uchi[k] = gu[sidx(k, 0)] * dchi[0] + gu[sidx(k, 1)] * dchi[1] + gu[sidx(k, 2)] * dchi[2];
    const T ua = uchi[0] * dalp[0] + uchi[1] * dalp[1] + uchi[2] * dalp[2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        const int q = sidx(i, j);
        T G = cdu[0][q] * dalp[0] + cdu[1][q] * dalp[1] + cdu[2][q] * dalp[2];
        G -= (dchi[j] * dalp[i] + dchi[i] * dalp[j] - gt[q] * ua) * i2chi;
        dd[q] -= G;  // D_i D_j alpha
      }
    lapalp = chi * (gu[0] * dd[0] + gu[3] * dd[3] + gu[5] * dd[5] +
                    (T)2 * (gu[1] * dd[1] + gu[2] * dd[2] + gu[4] * dd[4]));
#pragma unroll
    for (int q = 0; q < 6; ++q) X[q] = alpha * R[q] - dd[q];
  }

  // ---- everything that needs the Christoffels, d chi or d alpha is finished
  // here, so that those die before the shift derivatives are loaded
  T Atm[3][3];  // At^i_j
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Atm[i][j] = gu[sidx(i, 0)] * At[sidx(0, j)] + gu[sidx(i, 1)] * At[sidx(1, j)] +
                  gu[sidx(i, 2)] * At[sidx(2, j)];
  T Atu[6];  // At^ij
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j)
      Atu[sidx(i, j)] = Atm[i][0] * gu[sidx(0, j)] + Atm[i][1] * gu[sidx(1, j)] +
                        Atm[i][2] * gu[sidx(2, j)];
  T AtAt = (T)0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) AtAt += Atm[i][j] * Atm[j][i];

  const T two3 = (T)2 / (T)3, third = (T)1 / (T)3;
  const T ichi = (T)1 / chi;
  // non-advective part of dt Gt^i (also drives B^i), accumulated in Gs
  T Gs[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T aal = (T)0, ach = (T)0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      aal += Atu[sidx(i, j)] * dalp[j];
      ach += Atu[sidx(i, j)] * dchi[j];
    }
    const T cA = cdu[i][0] * Atu[0] + cdu[i][3] * Atu[3] + cdu[i][5] * Atu[5] +
                 (T)2 * (cdu[i][1] * Atu[1] + cdu[i][2] * Atu[2] + cdu[i][4] * Atu[4]);
    Gs[i] = (T)(-2) * aal + (T)2 * alpha * (cA - (T)1.5 * ach * ichi);
  }
  // dt K and dt At_ij without their shift and advection terms
  T rK = -lapalp + alpha * (AtAt + trK * trK * third);
  T rA[6];
  {
    const T trX = gu[0] * X[0] + gu[3] * X[3] + gu[5] * X[5] +
                  (T)2 * (gu[1] * X[1] + gu[2] * X[2] + gu[4] * X[4]);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        const int q = sidx(i, j);
        T aa = (T)0;
#pragma unroll
        for (int k = 0; k < 3; ++k) aa += At[sidx(i, k)] * Atm[k][j];
        rA[q] = chi * (X[q] - gt[q] * trX * third) + alpha * (trK * At[q] - (T)2 * aa);
      }
  }

  // ---- shift derivatives: d_j beta^k, gt^jk d_j d_k beta^i, d_j d_k beta^k
  T dbeta[3][3];  // dbeta[k][j] = d_j beta^k
  T lapb[3], gdiv[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const auto f = src.acquire(V_BETA + k);
    axis_derivs<T, true, true, true, KOM, ORD>(f, w, bpos, beta, dbeta[k], dpure, adv);
    rhs[V_BETA + k] = adv;
    second_derivs<T, ORD>(f, w, dpure, dd);
    lapb[k] = gu[0] * dd[0] + gu[3] * dd[3] + gu[5] * dd[5] +
              (T)2 * (gu[1] * dd[1] + gu[2] * dd[2] + gu[4] * dd[4]);
    // gdiv[j] += d_j d_k beta^k (k fixed here)
    if (k == 0) {
      gdiv[0] = dd[sidx(0, 0)];
      gdiv[1] = dd[sidx(1, 0)];
      gdiv[2] = dd[sidx(2, 0)];
    } else {
      gdiv[0] += dd[sidx(0, k)];
      gdiv[1] += dd[sidx(1, k)];
      gdiv[2] += dd[sidx(2, k)];
    }
  }
  const T divb = dbeta[0][0] + dbeta[1][1] + dbeta[2][2];
  rhs[V_CHI] += two3 * chi * (alpha * trK - divb);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      const int q = sidx(i, j);
      T sg = (T)0, sa = (T)0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sg += gt[sidx(i, k)] * dbeta[k][j] + gt[sidx(j, k)] * dbeta[k][i];
        sa += At[sidx(i, k)] * dbeta[k][j] + At[sidx(j, k)] * dbeta[k][i];
      }
      rhs[V_GT + q] += sg - (T)2 * alpha * At[q] - two3 * gt[q] * divb;
      rA[q] += sa - two3 * At[q] * divb;
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
    Gs[i] += -(Gd[0] * dbeta[i][0] + Gd[1] * dbeta[i][1] + Gd[2] * dbeta[i][2]) +
             two3 * Gd[i] * divb + lapb[i] +
             third * (gu[sidx(i, 0)] * gdiv[0] + gu[sidx(i, 1)] * gdiv[1] + gu[sidx(i, 2)] * gdiv[2]);

  // ---- trK (first derivatives + advection), At and B (advection only)
  {
    T dK[3];
    axis_derivs<T, true, false, true, KOM, ORD>(src.acquire(V_TRK), w, bpos, beta, dK, dpure, adv);
    rhs[V_TRK] = adv + rK;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T gk = gu[sidx(i, 0)] * dK[0] + gu[sidx(i, 1)] * dK[1] + gu[sidx(i, 2)] * dK[2];
      Gs[i] -= (T)2 * alpha * two3 * gk;
    }
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    axis_derivs<T, false, false, true, KOM, ORD>(src.acquire(V_AT + q), w, bpos, beta, d1v, dpure, adv);
    rhs[V_AT + q] = adv + rA[q];
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    axis_derivs<T, false, false, true, KOM, ORD>(src.acquire(V_B + q), w, bpos, beta, d1v, dpure, adv);
    rhs[V_B + q] = adv;
  }

  // ---- gauge
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    rhs[V_GAM + i] += Gs[i];
    if (P.shift == 1) {
      rhs[V_BETA + i] += (T)P.F * (T)src.center(V_B + i);
      rhs[V_B + i] += Gs[i] - (T)P.eta * (T)src.center(V_B + i);
    } else {
      rhs[V_BETA + i] = (T)0;
      rhs[V_B + i] = (T)0;
    }
  }
  if (P.slicing == 1)
    rhs[V_ALP] -= alpha * alpha * trK;
  else
    rhs[V_ALP] -= (T)2 * alpha * trK;
}

// RK4 substage update of one point (see StageIO) from the right-hand side.
// All pointwise loads (y0, acc) are issued before the first store: the
// output may alias nothing here, but the compiler cannot know that, and a
// load after a store to a possibly aliasing address would serialise the
// 24 updates into 24 memory round trips.
// Streaming hints for the pointwise traffic of a substage (outputs, y_n and
// the accumulator are touched once per launch): nontemporal accesses keep
// them from evicting the stencil planes that neighbouring tiles still need
// from L2.  CHEMORA_STREAM_HINTS=0 turns them off (ablation switch).
#ifndef CHEMORA_STREAM_HINTS
#define CHEMORA_STREAM_HINTS 1
#endif
__device__ __forceinline__ void st_stream(double* p, double v) {
#if CHEMORA_STREAM_HINTS
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}
__device__ __forceinline__ double ld_stream(const double* p) {
#if CHEMORA_STREAM_HINTS
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

// Algebraic constraints of the conformal variables at one point: rescale
// gt_ij by det(gt)^(-1/3) so that its determinant is 1, then remove the
// trace of At_ij with respect to the rescaled metric (inverse = adjugate /
// determinant): At_ij -= gt_ij gt^kl At_kl / 3.  FP64, on the stage output.
__device__ __forceinline__ double det3(const double g[6]) {
  return g[0] * (g[3] * g[5] - g[4] * g[4]) - g[1] * (g[1] * g[5] - g[4] * g[2]) +
         g[2] * (g[1] * g[4] - g[3] * g[2]);
}
__device__ __forceinline__ void enforce_point(double u[V_N]) {
  double g[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) g[q] = u[V_GT + q];
  const double sc = 1.0 / cbrt(det3(g));
#pragma unroll
  for (int q = 0; q < 6; ++q) g[q] *= sc;
  const double id = 1.0 / det3(g);
  // adjugate of the symmetric metric, (xx, xy, xz, yy, yz, zz)
  const double a[6] = {g[3] * g[5] - g[4] * g[4], g[2] * g[4] - g[1] * g[5],
                       g[1] * g[4] - g[2] * g[3], g[0] * g[5] - g[2] * g[2],
                       g[1] * g[2] - g[0] * g[4], g[0] * g[3] - g[1] * g[1]};
  const double tr = (a[0] * u[V_AT + 0] + a[3] * u[V_AT + 3] + a[5] * u[V_AT + 5] +
                     2.0 * (a[1] * u[V_AT + 1] + a[2] * u[V_AT + 2] + a[4] * u[V_AT + 4])) *
                    id;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    u[V_GT + q] = g[q];
    u[V_AT + q] -= g[q] * tr / 3.0;
  }
}

template <int STAGE, typename T>
__device__ __forceinline__ void bssn_store(const StageIO& io, const Geo& G, long long p, int i,
                                           int j, int k, const T rhs[V_N], bool images,
                                           bool enforce) {
  double* out = io.out + G.off0;
  if (STAGE == 0) {
#pragma unroll
    for (int v = 0; v < V_N; ++v) st_stream(out + p + v * G.sv, (double)rhs[v]);
    return;
  }
  double y0[V_N], ac[V_N];
#pragma unroll
  for (int v = 0; v < V_N; ++v) {
    y0[v] = ld_stream(io.y0 + G.off0 + p + v * G.sv);
    ac[v] = (STAGE == 2 || STAGE == 3 || STAGE == 4) ? ld_stream(io.acc + G.off0 + p + v * G.sv)
                                                      : 0.0;
  }
  double nv[V_N];
#pragma unroll
  for (int v = 0; v < V_N; ++v) {
    const long long q = p + v * G.sv;
    const double kv = (double)rhs[v];
    if (STAGE == 1) {
      st_stream(io.acc + G.off0 + q, kv);
      nv[v] = y0[v] + io.cdt * kv;
    } else if (STAGE == 2 || STAGE == 3) {
      st_stream(io.acc + G.off0 + q, ac[v] + 2.0 * kv);
      nv[v] = y0[v] + io.cdt * kv;
    } else {
      nv[v] = y0[v] + io.cdt * (ac[v] + kv);
    }
  }
  if (enforce) enforce_point(nv);
#pragma unroll
  for (int v = 0; v < V_N; ++v) {
    if (images) {
      store_with_images(out + v * G.sv, G, i, j, k, nv[v], true);
    } else {
      st_stream(out + p + v * G.sv, nv[v]);
    }
  }
}

}  // namespace chemora
