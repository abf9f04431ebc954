// bssn_split.hip -- the BSSN right-hand side (Sec. III.D of arXiv:1410.1764)
// split into two kernels per substage: the paper's kernel fission (Sec.
// III.B.3, Code Transformations), applied where the fused kernel runs out of
// registers.  The fused FP64 kernel needs 256 VGPRs + ~170 AGPRs, so a SIMD
// holds one of its waves; each half here fits in 256 registers, so a
// workgroup of 512 threads (two waves per SIMD) can evaluate two z-planes
// of a 32 x 8 tile from one z-blocked staging of each grid function
// (bssn_zsrc.h: 7.2 staged values per point and grid function against 10.8
// for one plane).
//
//   curvature kernel: stages gt_ij, Gamt^i, chi, alpha (the grid functions
//     whose second derivatives or Christoffels the geometry needs) and
//     computes the Ricci tensor, D_i D_j alpha, everything built from them,
//     and the advection terms of those 11 grid functions; 24 values per
//     point (one per slot of the output):
//       slot gt_ij, Gamt^i, chi, alpha: beta^k d_k of that grid function
//       slot At_ij: chi [-D_i D_j alpha + alpha R_ij]^TF + alpha (K At_ij - 2 At_ik At^k_j)
//       slot trK:   -D^2 alpha + alpha (At_ij At^ij + K^2/3)
//       slot beta^i: -2 At^ij d_j alpha + 2 alpha (Gt^i_jk At^jk - 3/2 At^ij d_j chi / chi)
//       slot B^i:   Gd^i = gt^jk Gt^i_jk
//   rest kernel: stages the shift (centred first and second derivatives),
//     K (first derivatives), At_ij and B^i (advection), adds the shift,
//     advection and gauge terms to the intermediates and does the RK4 update.
//
// The intermediates go to the interior of a state-sized buffer (StageIO::tmp,
// default the stage output): each thread of the rest kernel reads its own
// point's values before it writes any value of that point, so the output
// can hold them.  They are written and read once each, with nontemporal
// stores and loads (st_stream / ld_stream), so that they pass through L2
// without evicting the staged grid functions that neighbouring workgroups
// still read.  Every term is computed with the fused kernel's arithmetic
// in the same order (sums of the same two operands may swap sides).
#include <cstdlib>
#include <cstring>

// the point code of this file's kernels fences every mixed derivative, so
// that no more than one mixed stencil's loads are in registers at a time
#define CHEMORA_BSSN_FENCE 3
#include "bssn_args.h"
#include "bssn_zsrc.h"

namespace chemora {
namespace {

constexpr int kTX = 32, kTY = 8, kTZ = 2, kThreadsZ = kTX * kTY * kTZ, kZBufs = 3;

// slots of the curvature kernel's intermediates
enum : int { I_RA = V_AT, I_RK = V_TRK, I_GS = V_BETA, I_GD = V_B };

struct CurvOrder {  // the first 11 grid functions of the fused order
  static constexpr int N = 11;
  __device__ static constexpr int at(int s) { return kRhsOrder[s]; }
};
__device__ constexpr int kRestOrder[13] = {V_BETA + 0, V_BETA + 1, V_BETA + 2, V_TRK,
                                           V_AT + 0,   V_AT + 1,   V_AT + 2,   V_AT + 3,
                                           V_AT + 4,   V_AT + 5,   V_B + 0,    V_B + 1,
                                           V_B + 2};
struct RestOrder {
  static constexpr int N = 13;
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

// upwind sides and shift at the point
template <typename T, typename Src>
__device__ __forceinline__ void shift_at(const Src& src, bool bpos[3], T beta[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double b = src.center(V_BETA + d);
    bpos[d] = b >= 0.0;
    beta[d] = (T)b;
  }
}

// ---- curvature half ---------------------------------------------------------
// The advection terms of chi, gt_ij and Gamt^i are formed while the geometry
// is being built and are parked in LDS until it is done: held in registers
// they push the FP64 instance past 256, and stored to memory in between they
// would sit among the staging copies that the vmcnt hand-offs count.
constexpr int kStash = 10;
template <typename T, int NT>
struct AdvStash {
  T* base;  // slot s of this thread at base[s * NT]
  __device__ __forceinline__ T& operator[](int v) const {
    const int s = v == V_CHI ? 0 : (v < V_GAM ? v : v - V_GAM + 7);
    return base[s * NT];
  }
};

// Writes the point's 24 intermediates to o (slot v at o[v * sv]) as soon as
// each is complete, so that the values feeding it die early.
template <typename T, int KOM, typename Src, typename Stash>
__device__ __forceinline__ void bssn_curv_point(Src& src, const Weights& w, Stash& adv10,
                                                double* o, long long sv, bool active) {
  bool bpos[3];
  T beta[3];
  shift_at(src, bpos, beta);
  T gt[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) gt[q] = (T)src.center(V_GT + q);
  T gu[6], cdu[3][6], Gd[3], dchi[3], R[6];
  bssn_geometry<T, true, KOM, 4>(src, w, bpos, beta, gt, gu, cdu, Gd, dchi, R, adv10);
  // chi after the geometry: no copy in flight any more (the last grid
  // function's copies are waited for next anyway)
  const T chi = (T)src.center(V_CHI);
  if (active) {
#pragma unroll
    for (int d = 0; d < 3; ++d) st_stream(&o[(I_GD + d) * sv], (double)Gd[d]);
  }

  T dd[6], dpure[3], adv;
  T dalp[3];
  T lapalp, alpha;
  T X[6];
  {
    const auto f = src.acquire(V_ALP);
    alpha = (T)f(0, 0, 0);  // the staged centre: not held through the geometry
    axis_derivs<T, true, true, true, KOM, 4>(f, w, bpos, beta, dalp, dpure, adv);
    if (active) st_stream(&o[V_ALP * sv], (double)adv);
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
  const T trK = (T)src.center_nt(V_TRK);
  T At[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) At[q] = (T)src.center_nt(V_AT + q);

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
      if (active) st_stream(&o[(I_GS + i) * sv], (double)Gs);
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
    if (active) st_stream(&o[I_RK * sv], (double)rK);
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
      if (active) st_stream(&o[(I_RA + q) * sv], (double)rA);
    }
  if (active) {
#pragma unroll
    for (int q = 0; q < 6; ++q) st_stream(&o[(V_GT + q) * sv], (double)adv10[V_GT + q]);
#pragma unroll
    for (int d = 0; d < 3; ++d) st_stream(&o[(V_GAM + d) * sv], (double)adv10[V_GAM + d]);
    st_stream(&o[V_CHI * sv], (double)adv10[V_CHI]);
  }
}

// ---- rest: shift, K, At and B, gauge, assembly -------------------------------
// I: the point's intermediates (slot v at I[v * sv]).  Those needed while
// grid functions are still being staged are read with the centre values,
// before the copies start; the rest after the last grid function is staged.
template <typename T, int KOM, typename Src>
__device__ __forceinline__ void bssn_rest_point(Src& src, const double* I, long long sv,
                                                const Weights& w, const BssnPar& P,
                                                T rhs[V_N]) {
  bool bpos[3];
  T beta[3];
  shift_at(src, bpos, beta);
  const T chi = (T)src.center_nt(V_CHI);
  const T trK = (T)src.center(V_TRK);
  const T alpha = (T)src.center_nt(V_ALP);
  T gt[6], At[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    gt[q] = (T)src.center_nt(V_GT + q);
    At[q] = (T)src.center(V_AT + q);
  }
  T Gs[3], Gd[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Gs[i] = (T)ld_stream(&I[(I_GS + i) * sv]);
    Gd[i] = (T)ld_stream(&I[(I_GD + i) * sv]);
  }
  const T rK = (T)ld_stream(&I[I_RK * sv]);
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
  // shift terms of gt_ij and At_ij (their advection and the curvature
  // part of At_ij are added at the end)
  T sA[6];
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
      rhs[V_GT + q] = sg - (T)2 * alpha * At[q] - two3 * gt[q] * divb;
      sA[q] = sa - two3 * At[q] * divb;
    }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    axis_derivs<T, false, false, true, KOM, 4>(src.acquire(V_AT + q), w, bpos, beta, d1v, dpure,
                                               adv);
    rhs[V_AT + q] = adv;
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    axis_derivs<T, false, false, true, KOM, 4>(src.acquire(V_B + q), w, bpos, beta, d1v, dpure,
                                               adv);
    rhs[V_B + q] = adv;
  }
  // every grid function is staged: the remaining intermediates
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    rhs[V_GT + q] = (T)ld_stream(&I[(V_GT + q) * sv]) + rhs[V_GT + q];
    const T rA = (T)ld_stream(&I[(I_RA + q) * sv]) + sA[q];
    rhs[V_AT + q] = rhs[V_AT + q] + rA;
  }
  rhs[V_CHI] = (T)ld_stream(&I[V_CHI * sv]);
  rhs[V_CHI] += two3 * chi * (alpha * trK - divb);
  rhs[V_ALP] = (T)ld_stream(&I[V_ALP * sv]);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    rhs[V_GAM + i] = (T)ld_stream(&I[(V_GAM + i) * sv]);
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
// allow in both halves (2: at most 256 VGPRs + AGPRs, which the 512-thread
// workgroups need)
#ifndef CHEMORA_SPLIT_WAVES
#define CHEMORA_SPLIT_WAVES 2
#endif

// thread (tx, ty, pz) of a kTX x TY x kTZ block; false: no tile for this
// workgroup (uneven XCD columns)
template <int TY>
__device__ __forceinline__ bool zblock(const BssnArgs& a, int& x0, int& y0, int& k0, int& tx,
                                       int& ty, int& pz) {
  int bx, by, bz;
  if (!plane_tile(a, blockIdx.x, bx, by, bz)) return false;
  const int t = (int)threadIdx.x;
  tx = t % kTX;
  ty = (t / kTX) % TY;
  pz = t / (kTX * TY);
  x0 = bx * kTX;
  y0 = by * TY;
  k0 = bz * kTZ;
  return true;
}

template <typename T, int KOM, int TY, int NB>
__global__ void __launch_bounds__(kTX * TY * kTZ)
__attribute__((amdgpu_waves_per_eu(CHEMORA_SPLIT_WAVES))) bssn_curv_kernel(BssnArgs a) {
  using S = ZShape<kTX, TY, kTZ>;
  constexpr int NT = kTX * TY * kTZ;
  static_assert(NB == 2 || NB == 3, "two or three staging buffers");
  // separate arrays: the compiler then knows that an asynchronous copy into
  // one buffer cannot alias the reads of another, and does not wait for it
  __shared__ double L0[S::TOTAL], L1[S::TOTAL], L2[NB == 3 ? S::TOTAL : 1];
  __shared__ T stash[kStash * NT];
  double* const bufs[3] = {L0, L1, L2};
  const Geo& G = a.G;
  int x0, y0, k0, tx, ty, pz;
  if (!zblock<TY>(a, x0, y0, k0, tx, ty, pz)) return;  // whole workgroup: no barrier yet
  const int i = x0 + tx, j = y0 + ty, k = k0 + pz;
  const bool active = i < G.n[0] && j < G.n[1] && k < G.n[2];
  ZSrc<kTX, TY, kTZ, NB, CurvOrder> src;
  src.init(G, a.io.yin, bufs, x0, y0, k0, tx, ty, pz);
  double* o = (a.io.tmp ? a.io.tmp : a.io.out) + G.off0 +
              (active ? i + (long long)j * G.sy + (long long)k * G.sz : 0);
  AdvStash<T, NT> adv10{stash + threadIdx.x};
  bssn_curv_point<T, KOM>(src, a.W, adv10, o, G.sv, active);
}

template <int STAGE, typename T, int KOM, int TY>
__global__ void __launch_bounds__(kTX * TY * kTZ)
__attribute__((amdgpu_waves_per_eu(CHEMORA_SPLIT_WAVES))) bssn_rest_kernel(BssnArgs a) {
  using S = ZShape<kTX, TY, kTZ>;
  __shared__ double L0[S::TOTAL], L1[S::TOTAL], L2[S::TOTAL];
  double* const bufs[3] = {L0, L1, L2};
  const Geo& G = a.G;
  int x0, y0, k0, tx, ty, pz;
  if (!zblock<TY>(a, x0, y0, k0, tx, ty, pz)) return;  // whole workgroup: no barrier yet
  const int i = x0 + tx, j = y0 + ty, k = k0 + pz;
  const bool active = i < G.n[0] && j < G.n[1] && k < G.n[2];
  ZSrc<kTX, TY, kTZ, kZBufs, RestOrder> src;
  src.init(G, a.io.yin, bufs, x0, y0, k0, tx, ty, pz);
  // the point's intermediates (an idle thread of a ragged block reads the
  // clamped point, as its centre values do; it stores nothing)
  const int ci = i < G.n[0] ? i : G.n[0] - 1, cj = j < G.n[1] ? j : G.n[1] - 1;
  const int ck = k < G.n[2] ? k : G.n[2] - 1;
  const double* I = (a.io.tmp ? a.io.tmp : a.io.out) + G.off0 + ci + (long long)cj * G.sy +
                    (long long)ck * G.sz;
  T rhs[V_N];
  bssn_rest_point<T, KOM>(src, I, G.sv, a.W, a.P, rhs);
  if (active)
    bssn_store<STAGE, T>(a.io, G, i + (long long)j * G.sy + (long long)k * G.sz, i, j, k, rhs,
                         a.images != 0, a.P.enforce != 0);
}

// the fused point code over the same z-blocked staging (registers permitting)
template <int STAGE, typename T, int KOM, int TY>
__global__ void __launch_bounds__(kTX * TY * kTZ)
__attribute__((amdgpu_waves_per_eu(CHEMORA_SPLIT_WAVES))) bssn_zfused_kernel(BssnArgs a) {
  using S = ZShape<kTX, TY, kTZ>;
  __shared__ double L0[S::TOTAL], L1[S::TOTAL], L2[S::TOTAL];
  double* const bufs[3] = {L0, L1, L2};
  const Geo& G = a.G;
  int x0, y0, k0, tx, ty, pz;
  if (!zblock<TY>(a, x0, y0, k0, tx, ty, pz)) return;  // whole workgroup: no barrier yet
  const int i = x0 + tx, j = y0 + ty, k = k0 + pz;
  const bool active = i < G.n[0] && j < G.n[1] && k < G.n[2];
  ZSrc<kTX, TY, kTZ, kZBufs, RhsOrder> src;
  src.init(G, a.io.yin, bufs, x0, y0, k0, tx, ty, pz);
  T rhs[V_N];
  bssn_rhs_point<T, KOM>(src, a.W, a.P, rhs);
  if (active)
    bssn_store<STAGE, T>(a.io, G, i + (long long)j * G.sy + (long long)k * G.sz, i, j, k, rhs,
                         a.images != 0, a.P.enforce != 0);
}

// launch arguments of a z-blocked kernel with kTX x ty x kTZ blocks, in the
// XCD column walk
BssnArgs zargs(const BssnArgs& a0, int ty, dim3& grid) {
  BssnArgs a = a0;
  a.ltx = kTX;
  a.lty = ty;
  a.tiles[0] = (a.G.n[0] + kTX - 1) / kTX;
  a.tiles[1] = (a.G.n[1] + ty - 1) / ty;
  a.tiles[2] = (a.G.n[2] + kTZ - 1) / kTZ;
  long long blocks = (long long)a.tiles[0] * a.tiles[1] * a.tiles[2];
  a.cols[0] = a.cols[1] = 0;
  if (a0.cols[0] > 0) {
    const ColumnSplit c = column_split(a.tiles, a.ltx, a.lty);
    if (c.cx > 0) {
      a.cols[0] = c.cx;
      a.cols[1] = c.cy;
      blocks = c.blocks_per_plane * a.tiles[2];
    }
  }
  grid = dim3((unsigned)blocks);
  return a;
}

// CHEMORA_SPLIT_TY=8|4: tile height of the rest and z-blocked fused kernels
// (8: 512-thread workgroups, one per CU; 4: 256 threads, two per CU)
// (ablation switch, read at every launch)
int zty() {
  const char* e = std::getenv("CHEMORA_SPLIT_TY");
  return (e && e[0] == '4' && e[1] == 0) ? 4 : 8;
}

// CHEMORA_CURV_TY=8|4: tile height of the curvature kernel (8, default:
// 32 x 8 x 2 blocks, 512 threads, three staging buffers, one workgroup per
// CU; 4: 32 x 4 x 2 blocks, 256 threads, two buffers, two workgroups per CU
// whose barriers do not wait on each other, for more staging per point)
// (ablation switch, read at every launch).  Measured at 128^3, FP64, same
// job: right-hand side 0.720 ms (8) against 0.723 ms (4), RK4 step 3.79
// against 3.81 ms.
int curv_ty() {
  const char* e = std::getenv("CHEMORA_CURV_TY");
  return (e && e[0] == '4' && e[1] == 0) ? 4 : 8;
}

template <int STAGE, typename T, int TY>
void launch_pair_ty(int mode, const BssnArgs& a0, hipStream_t s) {
  dim3 grid;
  if constexpr (sizeof(T) == 4) {
    if (mode == 2) {
      const BssnArgs a = zargs(a0, TY, grid);
      hipLaunchKernelGGL((bssn_zfused_kernel<STAGE, T, KO_OFF, TY>), grid, dim3(kTX * TY * kTZ),
                         0, s, a);
      return;
    }
  }
  if (curv_ty() == 4) {
    const BssnArgs ac = zargs(a0, 4, grid);
    hipLaunchKernelGGL((bssn_curv_kernel<T, KO_OFF, 4, 2>), grid, dim3(kTX * 4 * kTZ), 0, s, ac);
  } else {
    const BssnArgs ac = zargs(a0, kTY, grid);
    hipLaunchKernelGGL((bssn_curv_kernel<T, KO_OFF, kTY, kZBufs>), grid, dim3(kThreadsZ), 0, s,
                       ac);
  }
  const BssnArgs ar = zargs(a0, TY, grid);
  hipLaunchKernelGGL((bssn_rest_kernel<STAGE, T, KO_OFF, TY>), grid, dim3(kTX * TY * kTZ), 0, s,
                     ar);
}

template <int STAGE, typename T>
void launch_pair(int mode, const BssnArgs& a, hipStream_t s) {
  if (zty() == 4)
    launch_pair_ty<STAGE, T, 4>(mode, a, s);
  else
    launch_pair_ty<STAGE, T, 8>(mode, a, s);
}

template <typename T>
void launch_pair_t(int mode, int stage, const BssnArgs& a, hipStream_t s) {
  switch (stage) {
    case 0: launch_pair<0, T>(mode, a, s); break;
    case 1: launch_pair<1, T>(mode, a, s); break;
    case 2: launch_pair<2, T>(mode, a, s); break;
    case 3: launch_pair<3, T>(mode, a, s); break;
    default: launch_pair<4, T>(mode, a, s); break;
  }
}

// CHEMORA_BSSN_SPLIT=0|1|2: 0 the fused single-plane kernel, 1 the split
// pair, 2 the fused point code over the z-blocked staging in mixed
// precision (the pair in FP64) (ablation switch, read at every launch).
// Default, measured at 128^3: FP64 the pair (right-hand side 0.725 ms
// against 0.760 ms fused; RK4 step 3.80 ms against 3.83 ms, the rest
// kernel's stage updates included); mixed the z-blocked fused kernel
// (right-hand side 0.53 ms against 0.59 ms, the pair 0.73 ms; RK4 step
// 2.89 ms against 3.15 ms).
int split_mode(int precision, int stage) {
  (void)stage;
  const char* e = std::getenv("CHEMORA_BSSN_SPLIT");
  if (e && (e[0] == '0' || e[0] == '1' || e[0] == '2') && e[1] == 0) return e[0] - '0';
  return precision == CHEMORA_MIXED ? 2 : 1;
}

}  // namespace

bool launch_bssn_split(int stage, int precision, const BssnArgs& a, dim3 grid, hipStream_t s,
                       hipError_t* err) {
  const int mode = split_mode(precision, stage);
  // dissipation: the fused kernels (the split curvature kernel's dissipative
  // instance would not fit in 256 registers)
  if (mode == 0 || a.P.fd_order != 4 || a.P.ko_sigma != 0.0 || a.ltx != kTX || a.lty != kTY)
    return false;
  (void)grid;
  if (precision == CHEMORA_MIXED)
    launch_pair_t<float>(mode, stage, a, s);
  else
    launch_pair_t<double>(mode, stage, a, s);
  *err = hipGetLastError();
  return true;
}

}  // namespace chemora
