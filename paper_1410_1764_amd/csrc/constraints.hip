// constraints.hip -- Hamiltonian and momentum constraints of the BSSN system
// (constraints are part of a physics system's description, Sec. III.B.1 of
// arXiv:1410.1764), always in FP64, centred stencils only, and their RMS
// norms over the interior by a deterministic two-pass reduction:
//   H   = R + 2/3 K^2 - At^ij At_ij,   R = chi gt^ij R_ij
//   M^i = gt^ia gt^jb (d_j At_ab - Gt^m_ja At_mb - Gt^m_jb At_am)
//         - 2/3 gt^ij d_j K - 3/2 At^ij d_j chi / chi
#include "bssn_point.h"

namespace chemora {
namespace {

constexpr int CT = 256;

struct ConsArgs {
  Geo G;
  Weights W;
  const double* y;
  double* hm;       // may be null
  double* partial;  // 4 doubles per workgroup
  int ltx, lty, zc;
  int tiles[3];
};

__device__ __forceinline__ void constraints_point(const double* __restrict__ Y, long long sv,
                                                  const long long st[3], const Weights& w,
                                                  double c[4]) {
  GSrc src{Y, sv, st[1], st[2]};
  auto F = [&](int v) { return Y + v * sv; };
  const bool bpos[3] = {true, true, true};
  const double beta[3] = {0.0, 0.0, 0.0};
  const double chi = F(V_CHI)[0], trK = F(V_TRK)[0];
  double gt[6], At[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    gt[q] = F(V_GT + q)[0];
    At[q] = F(V_AT + q)[0];
  }
  double gu[6], cdu[3][6], Gd[3], dchi[3], R[6], unused[V_N];
  bssn_geometry<double, false, KO_OFF>(src, w, bpos, beta, chi, gt, gu, cdu, Gd, dchi, R, unused);
  const double Rsc = chi * (gu[0] * R[0] + gu[3] * R[3] + gu[5] * R[5] +
                            2.0 * (gu[1] * R[1] + gu[2] * R[2] + gu[4] * R[4]));
  double Atm[3][3], Atu[6];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Atm[i][j] = gu[sidx(i, 0)] * At[sidx(0, j)] + gu[sidx(i, 1)] * At[sidx(1, j)] +
                  gu[sidx(i, 2)] * At[sidx(2, j)];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j)
      Atu[sidx(i, j)] = Atm[i][0] * gu[sidx(0, j)] + Atm[i][1] * gu[sidx(1, j)] +
                        Atm[i][2] * gu[sidx(2, j)];
  double AtAt = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) AtAt += Atm[i][j] * Atm[j][i];
  c[0] = Rsc + (2.0 / 3.0) * trK * trK - AtAt;

  double dpure[3], adv, dK[3], dAt[6][3];
  axis_derivs<double, true, false, false, KO_OFF>(src.acquire(V_TRK), w, bpos, beta, dK, dpure, adv);
#pragma unroll
  for (int q = 0; q < 6; ++q)
    axis_derivs<double, true, false, false, KO_OFF>(src.acquire(V_AT + q), w, bpos, beta, dAt[q], dpure,
                                            adv);
  // DA[j][ab] = D_j At_ab (conformal covariant derivative)
  double DA[3][6];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a; b < 3; ++b) {
        double s = dAt[sidx(a, b)][j];
#pragma unroll
        for (int m = 0; m < 3; ++m)
          s -= cdu[m][sidx(j, a)] * At[sidx(m, b)] + cdu[m][sidx(j, b)] * At[sidx(a, m)];
        DA[j][sidx(a, b)] = s;
      }
  const double ichi = 1.0 / chi;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int b = 0; b < 3; ++b) s += gu[sidx(i, a)] * gu[sidx(j, b)] * DA[j][sidx(a, b)];
    double gk = 0.0, ach = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      gk += gu[sidx(i, j)] * dK[j];
      ach += Atu[sidx(i, j)] * dchi[j];
    }
    c[1 + i] = s - (2.0 / 3.0) * gk - 1.5 * ach * ichi;
  }
}

__global__ void __launch_bounds__(CT) constraints_kernel(ConsArgs a) {
  __shared__ double red[4][CT];
  const Geo& G = a.G;
  const int nb = a.tiles[0] * a.tiles[1] * a.tiles[2];
  const int b = xcd_tile(blockIdx.x, nb);
  const int bx = b % a.tiles[0], by = (b / a.tiles[0]) % a.tiles[1];
  const int bz = b / (a.tiles[0] * a.tiles[1]);
  const int i = bx * a.ltx + (int)threadIdx.x % a.ltx;
  const int j = by * a.lty + (int)threadIdx.x / a.ltx;
  double sum[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < G.n[0] && j < G.n[1]) {
    const int k0 = bz * a.zc, k1 = min(k0 + a.zc, G.n[2]);
    const long long st[3] = {1, G.sy, G.sz};
    for (int k = k0; k < k1; ++k) {
      const long long p = i + (long long)j * G.sy + (long long)k * G.sz;
      double c[4];
      constraints_point(a.y + G.off0 + p, G.sv, st, a.W, c);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        sum[q] += c[q] * c[q];
        if (a.hm) a.hm[G.off0 + p + q * G.sv] = c[q];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = sum[q];
  __syncthreads();
  for (int w = CT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) a.partial[4LL * b + threadIdx.x] = red[threadIdx.x][0];
}

// Sum the per-workgroup partials in a fixed order and take sqrt(sum / N).
__global__ void __launch_bounds__(CT) norms_kernel(const double* partial, int nb, double npts,
                                                   double* norms) {
  __shared__ double red[4][CT];
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int t = threadIdx.x; t < nb; t += CT)
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] += partial[4LL * t + q];
#pragma unroll
  for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = s[q];
  __syncthreads();
  for (int w = CT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) norms[threadIdx.x] = sqrt(red[threadIdx.x][0] / npts);
}

void plan(const Geo& G, ConsArgs& a) {
  a.ltx = G.n[0] >= 48 ? 64 : (G.n[0] >= 24 ? 32 : 16);
  a.lty = CT / a.ltx;
  a.tiles[0] = (G.n[0] + a.ltx - 1) / a.ltx;
  a.tiles[1] = (G.n[1] + a.lty - 1) / a.lty;
  const long long xy = (long long)a.tiles[0] * a.tiles[1];
  int zsplit = (int)((4096 + xy - 1) / xy);
  if (zsplit > G.n[2]) zsplit = G.n[2];
  if (zsplit < 1) zsplit = 1;
  a.zc = (G.n[2] + zsplit - 1) / zsplit;
  a.tiles[2] = (G.n[2] + a.zc - 1) / a.zc;
}

}  // namespace

long long constraints_partial_count(const Geo& G) {
  ConsArgs a;
  plan(G, a);
  return 4LL * a.tiles[0] * a.tiles[1] * a.tiles[2];
}

hipError_t launch_bssn_constraints(const Geo& G, const BssnPar& P, const double* y, double* hm,
                                   double* norms, double* partial, hipStream_t s) {
  ConsArgs a;
  a.G = G;
  a.W = make_weights(P.h);
  a.y = y;
  a.hm = hm;
  a.partial = partial;
  plan(G, a);
  const int nb = a.tiles[0] * a.tiles[1] * a.tiles[2];
  hipLaunchKernelGGL(constraints_kernel, dim3(nb), dim3(CT), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double npts = (double)G.n[0] * G.n[1] * G.n[2];
  hipLaunchKernelGGL(norms_kernel, dim3(1), dim3(CT), 0, s, partial, nb, npts, norms);
  return hipGetLastError();
}

}  // namespace chemora
