// bssn_split.hip -- the BSSN right-hand side (Sec. III.D of arXiv:1410.1764)
// split into two kernels per substage: the paper's kernel fission (Sec.
// III.B.3, Code Transformations), applied where the fused kernel runs out of
// registers.  The fused FP64 kernel needs 256 VGPRs + ~170 AGPRs, so a SIMD
// holds one of its waves and cannot hide the latency of its dependent FP64
// chains; each half here fits in 256 registers (two waves per SIMD).
//
//   curvature kernel: stages gt_ij, Gamt^i, chi, alpha (the grid functions
//     whose second derivatives or Christoffels the geometry needs) and
//     computes the Ricci tensor, D_i D_j alpha and everything built from
//     them at the point; 13 intermediates per point:
//       rA_ij = chi [-D_i D_j alpha + alpha R_ij]^TF + alpha (K At_ij - 2 At_ik At^k_j)
//       rK    = -D^2 alpha + alpha (At_ij At^ij + K^2/3)
//       Gs^i  = -2 At^ij d_j alpha + 2 alpha (Gt^i_jk At^jk - 3/2 At^ij d_j chi / chi)
//       Gd^i  = gt^jk Gt^i_jk
//   rest kernel: stages the shift (centred first and second derivatives),
//     K (first derivatives) and every grid function's advection stencils,
//     adds the shift, advection and gauge terms, and does the RK4 update.
//
// The intermediates go to the interior of a state-sized buffer (StageIO::tmp,
// default the stage output), in the slots of At_ij, trK, Gamt^i and B^i:
// each thread of the rest kernel reads its own point's 13 values before it
// writes any value of that point, so the output can hold them.  The
// arithmetic of every term is the fused kernel's, in the same order.
#include <cstdlib>
#include <cstring>

#include "bssn_args.h"

namespace chemora {
namespace {

// slots of the intermediates in the tmp buffer
enum : int { I_RA = V_AT, I_RK = V_TRK, I_GS = V_GAM, I_GD = V_B };

struct CurvOrder {  // the first 11 grid functions of the fused order
  static constexpr int N = 11;
  __device__ static constexpr int at(int s) { return kRhsOrder[s]; }
};
__device__ constexpr int kRestOrder[V_N] = {
    V_BETA + 0, V_BETA + 1, V_BETA + 2, V_TRK,     V_GT + 0,  V_GT + 1,  V_GT + 2,  V_GT + 3,
    V_GT + 4,   V_GT + 5,   V_GAM + 0,  V_GAM + 1, V_GAM + 2, V_CHI,     V_ALP,     V_AT + 0,
    V_AT + 1,   V_AT + 2,   V_AT + 3,   V_AT + 4,  V_AT + 5,  V_B + 0,   V_B + 1,   V_B + 2};
struct RestOrder {
  static constexpr int N = V_N;
  __device__ static constexpr int at(int s) { return kRestOrder[s]; }
};

// inverse conformal metric (adjugate / determinant), as in bssn_geometry
template <typename T>
__device__ __forceinline__ void inverse_metric(const T gt[6], T gu[6]) {
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

// ---- curvature half ---------------------------------------------------------
// Writes the point's intermediates to o (slot v at o[v * sv]) as soon as
// each is complete, so that the values feeding it die early: with all 13
// (and the terms they are built from) live at once the FP64 instance does
// not fit in 256 registers.
template <typename T, typename Src>
__device__ __forceinline__ void bssn_curv_point(Src& src, const Weights& w, double* o,
                                                long long sv, bool active) {
  const T chi = (T)src.center(V_CHI);
  const T alpha = (T)src.center(V_ALP);
  T gt[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) gt[q] = (T)src.center(V_GT + q);
  const bool bpos[3] = {true, true, true};  // no advection here
  const T beta[3] = {(T)0, (T)0, (T)0};
  T gu[6], cdu[3][6], Gd[3], dchi[3], R[6], unused[V_N];
  bssn_geometry<T, false, KO_OFF, 4>(src, w, bpos, beta, chi, gt, gu, cdu, Gd, dchi, R, unused);
  if (active) {
#pragma unroll
    for (int d = 0; d < 3; ++d) o[(I_GD + d) * sv] = (double)Gd[d];
  }

  T dd[6], dpure[3], adv;
  T dalp[3];
  T lapalp;
  T X[6];
  {
    const auto f = src.acquire(V_ALP);
    axis_derivs<T, true, true, false, KO_OFF, 4>(f, w, bpos, beta, dalp, dpure, adv);
    second_derivs<T, 4>(f, w, dpure, dd);
    const T i2chi = (T)0.5 / chi;
    T uchi[3];
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
        dd[q] -= G;
      }
    lapalp = chi * (gu[0] * dd[0] + gu[3] * dd[3] + gu[5] * dd[5] +
                    (T)2 * (gu[1] * dd[1] + gu[2] * dd[2] + gu[4] * dd[4]));
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      X[q] = alpha * R[q] - dd[q];
      pin(X[q]);
    }
    pin(lapalp);
  }
  // K and At only enter from here on: loaded after the last grid function
  // is staged (no copy is in flight any more), so that they hold no
  // registers through the geometry
  const T trK = (T)src.center(V_TRK);
  T At[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) At[q] = (T)src.center(V_AT + q);

  T Atm[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Atm[i][j] = gu[sidx(i, 0)] * At[sidx(0, j)] + gu[sidx(i, 1)] * At[sidx(1, j)] +
                  gu[sidx(i, 2)] * At[sidx(2, j)];
  {
    T Atu[6];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j)
        Atu[sidx(i, j)] = Atm[i][0] * gu[sidx(0, j)] + Atm[i][1] * gu[sidx(1, j)] +
                          Atm[i][2] * gu[sidx(2, j)];
    const T ichi = (T)1 / chi;
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
      T Gs = (T)(-2) * aal + (T)2 * alpha * (cA - (T)1.5 * ach * ichi);
      pin(Gs);
      if (active) o[(I_GS + i) * sv] = (double)Gs;
    }
    fence_memory();
  }
  const T third = (T)1 / (T)3;
  {
    T AtAt = (T)0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) AtAt += Atm[i][j] * Atm[j][i];
    T rK = -lapalp + alpha * (AtAt + trK * trK * third);
    pin(rK);
    if (active) o[I_RK * sv] = (double)rK;
    fence_memory();
  }
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
      T rA = chi * (X[q] - gt[q] * trX * third) + alpha * (trK * At[q] - (T)2 * aa);
      if (active) o[(I_RA + q) * sv] = (double)rA;
    }
}

// ---- rest: shift, advection, gauge, assembly ------------------------------
// I: the point's intermediates (slot v at I[v * sv]), read with the centre
// values, before the staging copies start.
template <typename T, int KOM, typename Src>
__device__ __forceinline__ void bssn_rest_point(Src& src, const double* I, long long sv,
                                                const Weights& w, const BssnPar& P,
                                                T rhs[V_N]) {
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
  T rA[6], rK, Gs[3], Gd[3];
#pragma unroll
  for (int q = 0; q < 6; ++q) rA[q] = (T)I[(I_RA + q) * sv];
  rK = (T)I[I_RK * sv];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Gs[i] = (T)I[(I_GS + i) * sv];
    Gd[i] = (T)I[(I_GD + i) * sv];
  }
  T gu[6];
  inverse_metric(gt, gu);

  const T two3 = (T)2 / (T)3, third = (T)1 / (T)3;
  T dd[6], dpure[3], d1v[3], adv;
  // shift: d_j beta^k, gt^jk d_j d_k beta^i, d_j d_k beta^k
  T dbeta[3][3];
  T lapb[3], gdiv[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const auto f = src.acquire(V_BETA + k);
    axis_derivs<T, true, true, true, KOM, 4>(f, w, bpos, beta, dbeta[k], dpure, adv);
    rhs[V_BETA + k] = adv;
    second_derivs<T, 4>(f, w, dpure, dd);
    lapb[k] = gu[0] * dd[0] + gu[3] * dd[3] + gu[5] * dd[5] +
              (T)2 * (gu[1] * dd[1] + gu[2] * dd[2] + gu[4] * dd[4]);
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
#pragma unroll
  for (int i = 0; i < 3; ++i)
    Gs[i] += -(Gd[0] * dbeta[i][0] + Gd[1] * dbeta[i][1] + Gd[2] * dbeta[i][2]) +
             two3 * Gd[i] * divb + lapb[i] +
             third * (gu[sidx(i, 0)] * gdiv[0] + gu[sidx(i, 1)] * gdiv[1] + gu[sidx(i, 2)] * gdiv[2]);
  {
    T dK[3];
    axis_derivs<T, true, false, true, KOM, 4>(src.acquire(V_TRK), w, bpos, beta, dK, dpure, adv);
    rhs[V_TRK] = adv + rK;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T gk = gu[sidx(i, 0)] * dK[0] + gu[sidx(i, 1)] * dK[1] + gu[sidx(i, 2)] * dK[2];
      Gs[i] -= (T)2 * alpha * two3 * gk;
    }
  }
  // gt_ij: advection plus the shift terms
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    axis_derivs<T, false, false, true, KOM, 4>(src.acquire(V_GT + q), w, bpos, beta, d1v, dpure,
                                               adv);
    rhs[V_GT + q] = adv;
  }
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
  for (int k = 0; k < 3; ++k) {
    axis_derivs<T, false, false, true, KOM, 4>(src.acquire(V_GAM + k), w, bpos, beta, d1v, dpure,
                                               adv);
    rhs[V_GAM + k] = adv;
  }
  axis_derivs<T, false, false, true, KOM, 4>(src.acquire(V_CHI), w, bpos, beta, d1v, dpure, adv);
  rhs[V_CHI] = adv;
  rhs[V_CHI] += two3 * chi * (alpha * trK - divb);
  axis_derivs<T, false, false, true, KOM, 4>(src.acquire(V_ALP), w, bpos, beta, d1v, dpure, adv);
  rhs[V_ALP] = adv;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    axis_derivs<T, false, false, true, KOM, 4>(src.acquire(V_AT + q), w, bpos, beta, d1v, dpure,
                                               adv);
    rhs[V_AT + q] = adv + rA[q];
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    axis_derivs<T, false, false, true, KOM, 4>(src.acquire(V_B + q), w, bpos, beta, d1v, dpure,
                                               adv);
    rhs[V_B + q] = adv;
  }
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

// CHEMORA_SPLIT_WAVES: minimum waves per SIMD the register allocator must
// allow in both halves (2: at most 256 VGPRs + AGPRs)
#ifndef CHEMORA_SPLIT_WAVES
#define CHEMORA_SPLIT_WAVES 2
#endif

constexpr int kSplitBufs = 3;

template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CHEMORA_SPLIT_WAVES)))
bssn_curv_kernel(BssnArgs a) {
  using S = LdsShape<32, 8>;
  __shared__ double L0[S::TOTAL], L1[S::TOTAL], L2[S::TOTAL];
  double* const bufs[3] = {L0, L1, L2};
  const Geo& G = a.G;
  int bx, by, k;
  if (!plane_tile(a, blockIdx.x, bx, by, k)) return;  // whole workgroup: no barrier yet
  const int tx = (int)threadIdx.x % 32, ty = (int)threadIdx.x / 32;
  const int i = bx * 32 + tx, j = by * 8 + ty;
  ASrc<32, 8, kSplitBufs, CurvOrder> src;
  src.init(G, a.io.yin, bufs, bx * 32, by * 8, k, tx, ty);
  const bool active = i < G.n[0] && j < G.n[1];
  double* o = (a.io.tmp ? a.io.tmp : a.io.out) + G.off0 + (active ? i : 0) +
              (long long)(active ? j : 0) * G.sy + (long long)k * G.sz;
  bssn_curv_point<T>(src, a.W, o, G.sv, active);
}

template <int STAGE, typename T, int KOM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CHEMORA_SPLIT_WAVES)))
bssn_rest_kernel(BssnArgs a) {
  using S = LdsShape<32, 8>;
  __shared__ double L0[S::TOTAL], L1[S::TOTAL], L2[S::TOTAL];
  double* const bufs[3] = {L0, L1, L2};
  const Geo& G = a.G;
  int bx, by, k;
  if (!plane_tile(a, blockIdx.x, bx, by, k)) return;  // whole workgroup: no barrier yet
  const int tx = (int)threadIdx.x % 32, ty = (int)threadIdx.x / 32;
  const int i = bx * 32 + tx, j = by * 8 + ty;
  const bool active = i < G.n[0] && j < G.n[1];
  ASrc<32, 8, kSplitBufs, RestOrder> src;
  src.init(G, a.io.yin, bufs, bx * 32, by * 8, k, tx, ty);
  // the point's intermediates (a ragged tile's idle threads read the
  // clamped point, as their centre values do)
  const int ci = i < G.n[0] ? i : G.n[0] - 1, cj = j < G.n[1] ? j : G.n[1] - 1;
  const double* I = (a.io.tmp ? a.io.tmp : a.io.out) + G.off0 + ci + (long long)cj * G.sy +
                    (long long)k * G.sz;
  T rhs[V_N];
  bssn_rest_point<T, KOM>(src, I, G.sv, a.W, a.P, rhs);
  if (active)
    bssn_store<STAGE, T>(a.io, G, i + (long long)j * G.sy + (long long)k * G.sz, i, j, k, rhs,
                         a.images != 0, a.P.enforce != 0);
}

template <int STAGE, typename T>
void launch_pair(const BssnArgs& a, dim3 grid, hipStream_t s) {
  hipLaunchKernelGGL((bssn_curv_kernel<T>), grid, dim3(256), 0, s, a);
  if (a.P.ko_sigma != 0.0)
    hipLaunchKernelGGL((bssn_rest_kernel<STAGE, T, KO_ON>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((bssn_rest_kernel<STAGE, T, KO_OFF>), grid, dim3(256), 0, s, a);
}

template <typename T>
void launch_pair_t(int stage, const BssnArgs& a, dim3 grid, hipStream_t s) {
  switch (stage) {
    case 0: launch_pair<0, T>(a, grid, s); break;
    case 1: launch_pair<1, T>(a, grid, s); break;
    case 2: launch_pair<2, T>(a, grid, s); break;
    case 3: launch_pair<3, T>(a, grid, s); break;
    default: launch_pair<4, T>(a, grid, s); break;
  }
}

// CHEMORA_BSSN_SPLIT=0|1 switches the split form off or on for both
// precisions (ablation switch, read at every launch); unset: the measured
// default per precision
int split_override() {
  const char* e = std::getenv("CHEMORA_BSSN_SPLIT");
  if (e && std::strcmp(e, "0") == 0) return 0;
  if (e && std::strcmp(e, "1") == 0) return 1;
  return -1;
}

bool split_default(int precision) {
  (void)precision;
  return false;
}

}  // namespace

bool launch_bssn_split(int stage, int precision, const BssnArgs& a, dim3 grid, hipStream_t s,
                       hipError_t* err) {
  const int o = split_override();
  const bool on = o >= 0 ? o == 1 : split_default(precision);
  if (!on || a.P.fd_order != 4 || a.ltx != 32 || a.lty != 8) return false;
  if (precision == CHEMORA_MIXED)
    launch_pair_t<float>(stage, a, grid, s);
  else
    launch_pair_t<double>(stage, a, grid, s);
  *err = hipGetLastError();
  return true;
}

}  // namespace chemora
