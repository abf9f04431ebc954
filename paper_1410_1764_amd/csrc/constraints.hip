// constraints.hip -- Hamiltonian and momentum constraints of the BSSN system
// (constraints are part of a physics system's description, Sec. III.B.1 of
// arXiv:1410.1764), always in FP64, centred stencils only, and their RMS
// norms over the interior by a deterministic two-pass reduction:
//   H   = R + 2/3 K^2 - At^ij At_ij,   R = chi gt^ij R_ij
//   M^i = gt^ia gt^jb (d_j At_ab - Gt^m_ja At_mb - Gt^m_jb At_am)
//         - 2/3 gt^ij d_j K - 3/2 At^ij d_j chi / chi
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "bssn_lds.h"

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
  int cols[2];  // staged kernel: column split of the tile grid (0: XCD-contiguous order)
};

// H and M^i at one point, reading through a neighbourhood source (GSrc or
// the LDS-staged ASrc with the constraints' acquisition order)
template <int ORD, typename Src>
__device__ __forceinline__ void constraints_point(Src& src, const Weights& w, double c[4]) {
  const bool bpos[3] = {true, true, true};
  const double beta[3] = {0.0, 0.0, 0.0};
  const double chi = src.center(V_CHI), trK = src.center(V_TRK);
  double gt[6], At[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    gt[q] = src.center(V_GT + q);
    At[q] = src.center(V_AT + q);
  }
  double gu[6], cdu[3][6], Gd[3], dchi[3], R[6], unused[V_N];
  bssn_geometry<double, false, KO_OFF, ORD>(src, w, bpos, beta, gt, gu, cdu, Gd, dchi, R, unused);
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
  axis_derivs<double, true, false, false, KO_OFF, ORD>(src.acquire(V_TRK), w, bpos, beta, dK, dpure, adv);
#pragma unroll
  for (int q = 0; q < 6; ++q)
    axis_derivs<double, true, false, false, KO_OFF, ORD>(src.acquire(V_AT + q), w, bpos, beta, dAt[q], dpure,
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

template <int ORD>
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
      GSrc src{a.y + G.off0 + p, G.sv, st[1], st[2]};
      constraints_point<ORD>(src, a.W, c);
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

// LDS-staged variant (the right-hand side's async staging with the
// constraints' 17 grid functions): one plane of a TX x TY tile per
// workgroup, tiles in the XCD column walk; workgroup b writes partial b
// (zeros when the column walk gives it no tile).
template <int TX, int TY, int NBUF>
__global__ void __launch_bounds__(TX * TY) constraints_async_kernel(ConsArgs a) {
  using S = LdsShape<TX, TY>;
  constexpr int NT = TX * TY;
  __shared__ double L0[S::TOTAL], L1[S::TOTAL], L2[S::TOTAL], L3[S::TOTAL], L4[S::TOTAL],
      L5[S::TOTAL];
  __shared__ double red[4][NT];
  double* const bufs[6] = {L0, L1, L2, L3, L4, L5};
  const Geo& G = a.G;
  int bx, by, k;
  bool has;
  if (a.cols[0] > 0) {
    has = column_tile(blockIdx.x, a.tiles, a.cols[0], a.cols[1], bx, by, k);
  } else {
    const int t = xcd_tile(blockIdx.x, a.tiles[0] * a.tiles[1] * a.tiles[2]);
    bx = t % a.tiles[0];
    by = (t / a.tiles[0]) % a.tiles[1];
    k = t / (a.tiles[0] * a.tiles[1]);
    has = true;
  }
  if (!has) {  // whole workgroup, before any barrier
    if (threadIdx.x < 4) a.partial[4LL * blockIdx.x + threadIdx.x] = 0.0;
    return;
  }
  const int tx = (int)threadIdx.x % TX, ty = (int)threadIdx.x / TX;
  const int x0 = bx * TX, y0 = by * TY;
  const int i = x0 + tx, j = y0 + ty;
  const bool active = i < G.n[0] && j < G.n[1];
  ASrc<TX, TY, NBUF, ConsOrder> src;
  src.init(G, a.y, bufs, x0, y0, k, tx, ty);
  double c[4];
  constraints_point<4>(src, a.W, c);
  const long long p = i + (long long)j * G.sy + (long long)k * G.sz;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (a.hm && active) a.hm[G.off0 + p + q * G.sv] = c[q];
    red[q][threadIdx.x] = active ? c[q] * c[q] : 0.0;
  }
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) a.partial[4LL * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// 6th- and 8th-order constraints: the same tiling with the wider staged
// neighbourhood of those orders (HSrc: two buffers, one barrier per grid
// function, any acquisition order)
template <int TX, int TY, int ORD>
__global__ void __launch_bounds__(TX * TY) constraints_hi_kernel(ConsArgs a) {
  constexpr int R = ORD / 2 + 1;
  using S = HShape<TX, TY, R>;
  constexpr int NT = TX * TY;
  __shared__ double L0[S::TOTAL], L1[S::TOTAL];
  __shared__ int tab[S::TOTAL];
  __shared__ double red[4][NT];
  const Geo& G = a.G;
  int bx, by, k;
  bool has;
  if (a.cols[0] > 0) {
    has = column_tile(blockIdx.x, a.tiles, a.cols[0], a.cols[1], bx, by, k);
  } else {
    const int t = xcd_tile(blockIdx.x, a.tiles[0] * a.tiles[1] * a.tiles[2]);
    bx = t % a.tiles[0];
    by = (t / a.tiles[0]) % a.tiles[1];
    k = t / (a.tiles[0] * a.tiles[1]);
    has = true;
  }
  if (!has) {  // whole workgroup, before any barrier
    if (threadIdx.x < 4) a.partial[4LL * blockIdx.x + threadIdx.x] = 0.0;
    return;
  }
  const int tx = (int)threadIdx.x % TX, ty = (int)threadIdx.x / TX;
  const int x0 = bx * TX, y0 = by * TY;
  const int i = x0 + tx, j = y0 + ty;
  const bool active = i < G.n[0] && j < G.n[1];
  HSrc<TX, TY, R> src;
  src.init(G, a.y, L0, L1, tab, x0, y0, k, tx, ty);
  double c[4];
  constraints_point<ORD>(src, a.W, c);
  const long long p = i + (long long)j * G.sy + (long long)k * G.sz;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (a.hm && active) a.hm[G.off0 + p + q * G.sv] = c[q];
    red[q][threadIdx.x] = active ? c[q] * c[q] : 0.0;
  }
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) a.partial[4LL * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
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

// CHEMORA_CONS_NBUF=3|6: staging buffers of the staged kernel (3: two
// workgroups fit a CU; ablation switch, read at every launch)
int cons_nbuf() {
  const int v = [] {
    const char* e = std::getenv("CHEMORA_CONS_NBUF");
    return (e && std::atoi(e) == 6) ? 6 : 3;
  }();
  return v;
}

// CHEMORA_CONS_KERNEL=global selects the cached-load kernel (ablation switch,
// read once per process: it sets the number of workgroups, and with it the
// size of the caller's partial-sum workspace)
bool staged() {
  static const bool v = [] {
    const char* e = std::getenv("CHEMORA_CONS_KERNEL");
    return !(e && std::strcmp(e, "global") == 0);
  }();
  return v;
}

// returns the number of workgroups
long long plan(const Geo& G, int order, ConsArgs& a) {
  a.cols[0] = a.cols[1] = 0;
  (void)order;
  if (staged()) {
    a.ltx = G.n[0] >= 24 ? 32 : 16;
    a.lty = CT / a.ltx;
    a.tiles[0] = (G.n[0] + a.ltx - 1) / a.ltx;
    a.tiles[1] = (G.n[1] + a.lty - 1) / a.lty;
    a.zc = 1;
    a.tiles[2] = G.n[2];
    const ColumnSplit c = column_split(a.tiles, a.ltx, a.lty);
    if (c.cx > 0) {
      a.cols[0] = c.cx;
      a.cols[1] = c.cy;
      return c.blocks_per_plane * a.tiles[2];
    }
    return (long long)a.tiles[0] * a.tiles[1] * a.tiles[2];
  }
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
  return (long long)a.tiles[0] * a.tiles[1] * a.tiles[2];
}

}  // namespace

long long constraints_partial_count(const Geo& G, int order) {
  ConsArgs a;
  return 4LL * plan(G, order, a);
}

hipError_t launch_bssn_constraints(const Geo& G, const BssnPar& P, const double* y, double* hm,
                                   double* norms, double* partial, hipStream_t s) {
  ConsArgs a;
  a.G = G;
  a.W = make_weights(P.h, 0.0, P.fd_order);
  a.y = y;
  a.hm = hm;
  a.partial = partial;
  const int nb = (int)plan(G, P.fd_order, a);
  if (P.fd_order == 6 && !staged())
    hipLaunchKernelGGL(constraints_kernel<6>, dim3(nb), dim3(CT), 0, s, a);
  else if (P.fd_order == 8 && !staged())
    hipLaunchKernelGGL(constraints_kernel<8>, dim3(nb), dim3(CT), 0, s, a);
  else if (P.fd_order == 6 && a.ltx == 32)
    hipLaunchKernelGGL((constraints_hi_kernel<32, 8, 6>), dim3(nb), dim3(CT), 0, s, a);
  else if (P.fd_order == 6)
    hipLaunchKernelGGL((constraints_hi_kernel<16, 16, 6>), dim3(nb), dim3(CT), 0, s, a);
  else if (P.fd_order == 8 && a.ltx == 32)
    hipLaunchKernelGGL((constraints_hi_kernel<32, 8, 8>), dim3(nb), dim3(CT), 0, s, a);
  else if (P.fd_order == 8)
    hipLaunchKernelGGL((constraints_hi_kernel<16, 16, 8>), dim3(nb), dim3(CT), 0, s, a);
  else if (!staged())
    hipLaunchKernelGGL(constraints_kernel<4>, dim3(nb), dim3(CT), 0, s, a);
  else if (a.ltx == 32 && cons_nbuf() == 6)
    hipLaunchKernelGGL((constraints_async_kernel<32, 8, 6>), dim3(nb), dim3(CT), 0, s, a);
  else if (a.ltx == 32)
    hipLaunchKernelGGL((constraints_async_kernel<32, 8, 3>), dim3(nb), dim3(CT), 0, s, a);
  else
    hipLaunchKernelGGL((constraints_async_kernel<16, 16, 3>), dim3(nb), dim3(CT), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double npts = (double)G.n[0] * G.n[1] * G.n[2];
  hipLaunchKernelGGL(norms_kernel, dim3(1), dim3(CT), 0, s, partial, nb, npts, norms);
  return hipGetLastError();
}

// ---- partial sums without a caller workspace ----------------------------
// For callers that cannot allocate (graph capture, serving loops): the
// per-workgroup partial sums of chemora_constraints_noalloc live in this
// file-scope device array.  Every GPU the library runs on holds its own copy
// until the process ends; every call on a GPU shares that GPU's copy, so
// calls that overlap on one GPU race.  Nothing in it has to start at zero:
// each workgroup of the constraint kernel writes its 4 partials (zeros when
// the column walk gives it no tile) before the norms kernel reads them.
constexpr long long kStaticPartials = 1LL << 20;  // doubles: 8 MiB per GPU
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kStaticPartials];

long long constraints_static_capacity() { return kStaticPartials; }

hipError_t constraints_static_partials(double** out) {
  static std::mutex mu;
  static double* ptrs[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!ptrs[dev]) {
    // the array's name is a host-side stand-in: its address on this device
    // (current here) comes from the runtime, once per device
    double* p = nullptr;
    e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptrs[dev] = p;
  }
  *out = ptrs[dev];
  return hipSuccess;
}

}  // namespace chemora
