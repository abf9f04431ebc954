// bssn.hip -- BSSN right-hand side over one block, alone or fused with an
// RK4 substage (Sec. III.D of arXiv:1410.1764: the Einstein equations; Sec. II:
// the time integrator).  The per-point arithmetic is in bssn_point.h.
//
// Mapping: a workgroup of 256 threads covers a tile of ltx x lty points in
// xy (ltx = 64, 32 or 16; x contiguous within a wavefront so that every
// stencil load of a wavefront is a coalesced row segment) and marches zc
// planes along z, one point per thread per plane.  Tiles are laid out
// XCD-contiguously (xcd_tile).  Two kernels:
//   bssn_lds_kernel (default): each grid function's tile neighbourhood is
//     staged in LDS by one cooperative, double-buffered burst (bssn_lds.h);
//   bssn_stage_kernel (ablation, CHEMORA_BSSN_KERNEL=global): stencil
//     neighbours are read straight from global memory through L1/L2.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "bssn_lds.h"

namespace chemora {
namespace {

struct BssnArgs {
  Geo G;
  BssnPar P;
  Weights W;
  StageIO io;
  int ltx, lty, zc;
  int tiles[3];
  int images;
};

// CHEMORA_BSSN_WAVES: minimum waves per SIMD the register allocator must
// allow (an ablation switch; 1 lets the FP64 kernel use VGPRs + AGPRs).
#ifndef CHEMORA_BSSN_WAVES
#define CHEMORA_BSSN_WAVES 1
#endif

template <int STAGE, typename T>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(CHEMORA_BSSN_WAVES))) bssn_stage_kernel(BssnArgs a) {
  const Geo& G = a.G;
  const int nb = a.tiles[0] * a.tiles[1] * a.tiles[2];
  const int b = xcd_tile(blockIdx.x, nb);
  const int bx = b % a.tiles[0], by = (b / a.tiles[0]) % a.tiles[1];
  const int bz = b / (a.tiles[0] * a.tiles[1]);
  const int i = bx * a.ltx + (int)threadIdx.x % a.ltx;
  const int j = by * a.lty + (int)threadIdx.x / a.ltx;
  if (i >= G.n[0] || j >= G.n[1]) return;
  const int k0 = bz * a.zc, k1 = min(k0 + a.zc, G.n[2]);
  for (int k = k0; k < k1; ++k) {
    const long long p = i + (long long)j * G.sy + (long long)k * G.sz;
    T rhs[V_N];
    GSrc src{a.io.yin + G.off0 + p, G.sv, G.sy, G.sz};
    bssn_rhs_point<T>(src, a.W, a.P, rhs);
    bssn_store<STAGE, T>(a.io, G, p, i, j, k, rhs, a.images != 0);
  }
}

template <int STAGE, typename T, int TX, int TY>
__global__ void __launch_bounds__(TX * TY) bssn_lds_kernel(BssnArgs a) {
  using S = LdsShape<TX, TY>;
  __shared__ double lds[2 * S::TOTAL];
  const Geo& G = a.G;
  const int nb = a.tiles[0] * a.tiles[1] * a.tiles[2];
  const int b = xcd_tile(blockIdx.x, nb);
  const int bx = b % a.tiles[0], by = (b / a.tiles[0]) % a.tiles[1];
  const int bz = b / (a.tiles[0] * a.tiles[1]);
  const int tx = (int)threadIdx.x % TX, ty = (int)threadIdx.x / TX;
  const int x0 = bx * TX, y0 = by * TY;
  const int i = x0 + tx, j = y0 + ty;
  const bool active = i < G.n[0] && j < G.n[1];
  // one plane per workgroup: marching several planes in one workgroup keeps
  // the staging state live across the loop and roughly doubles the
  // register footprint
  const int k = bz;
  LSrc<TX, TY> src;
  src.init(G, a.io.yin, lds, lds + S::TOTAL, x0, y0, k, tx, ty);
  src.prefetch(kRhsOrder[0]);
  T rhs[V_N];
  bssn_rhs_point<T>(src, a.W, a.P, rhs);
  if (active)
    bssn_store<STAGE, T>(a.io, G, i + (long long)j * G.sy + (long long)k * G.sz, i, j, k, rhs,
                         a.images != 0);
}

template <int STAGE, typename T, int TX, int TY, int NBUF>
__global__ void __launch_bounds__(TX * TY) bssn_async_kernel(BssnArgs a) {
  static_assert(NBUF >= 2 && NBUF <= 6, "1 to 5 grid functions in flight");
  using S = LdsShape<TX, TY>;
  // separate arrays, one per buffer (see ASrc); unused ones are not allocated
  __shared__ double L0[S::TOTAL], L1[S::TOTAL], L2[S::TOTAL], L3[S::TOTAL], L4[S::TOTAL],
      L5[S::TOTAL];
  double* const bufs[6] = {L0, L1, L2, L3, L4, L5};
  const Geo& G = a.G;
  const int nb = a.tiles[0] * a.tiles[1] * a.tiles[2];
  const int b = xcd_tile(blockIdx.x, nb);
  const int bx = b % a.tiles[0], by = (b / a.tiles[0]) % a.tiles[1];
  const int k = b / (a.tiles[0] * a.tiles[1]);
  const int tx = (int)threadIdx.x % TX, ty = (int)threadIdx.x / TX;
  const int x0 = bx * TX, y0 = by * TY;
  const int i = x0 + tx, j = y0 + ty;
  const bool active = i < G.n[0] && j < G.n[1];
  ASrc<TX, TY, NBUF> src;
  src.init(G, a.io.yin, bufs, x0, y0, k, tx, ty);
  T rhs[V_N];
  bssn_rhs_point<T>(src, a.W, a.P, rhs);
  if (active)
    bssn_store<STAGE, T>(a.io, G, i + (long long)j * G.sy + (long long)k * G.sz, i, j, k, rhs,
                         a.images != 0);
}

// CHEMORA_BSSN_TILE=64|32|16 forces the tile width (ablation switch)
int forced_tile_width() {
  static const int w = [] {
    const char* e = std::getenv("CHEMORA_BSSN_TILE");
    const int v = e ? std::atoi(e) : 0;
    return (v == 64 || v == 32 || v == 16) ? v : 0;
  }();
  return w;
}

// Kernel choice (measured at 128^3): FP64 -> async staging (five grid
// functions in flight hide the memory latency that one wave per SIMD
// cannot); mixed -> LDS staging (its 248 VGPRs and 44 KB of LDS allow two
// waves per SIMD).  CHEMORA_BSSN_KERNEL=global|lds|async overrides it
// (ablation switch).
int kernel_override() {
  static const int v = [] {
    const char* e = std::getenv("CHEMORA_BSSN_KERNEL");
    if (e && std::strcmp(e, "global") == 0) return 0;
    if (e && std::strcmp(e, "lds") == 0) return 1;
    if (e && std::strcmp(e, "async") == 0) return 2;
    return -1;
  }();
  return v;
}
int kernel_variant(int precision) {
  const int o = kernel_override();
  return o >= 0 ? o : (precision == CHEMORA_MIXED ? 1 : 2);
}

template <int STAGE, typename T>
void launch_shape(const BssnArgs& a, dim3 grid, hipStream_t s) {
  const int variant = kernel_variant(sizeof(T) == 4 ? CHEMORA_MIXED : CHEMORA_FP64);
  if (variant == 0) {
    hipLaunchKernelGGL((bssn_stage_kernel<STAGE, T>), grid, dim3(256), 0, s, a);
  } else if (variant == 2) {
    if (a.ltx == 64)
      hipLaunchKernelGGL((bssn_async_kernel<STAGE, T, 64, 4, 5>), grid, dim3(256), 0, s, a);
    else if (a.ltx == 32)
      hipLaunchKernelGGL((bssn_async_kernel<STAGE, T, 32, 8, 6>), grid, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((bssn_async_kernel<STAGE, T, 16, 16, 6>), grid, dim3(256), 0, s, a);
  } else if (a.ltx == 64) {
    hipLaunchKernelGGL((bssn_lds_kernel<STAGE, T, 64, 4>), grid, dim3(256), 0, s, a);
  } else if (a.ltx == 32) {
    hipLaunchKernelGGL((bssn_lds_kernel<STAGE, T, 32, 8>), grid, dim3(256), 0, s, a);
  } else {
    hipLaunchKernelGGL((bssn_lds_kernel<STAGE, T, 16, 16>), grid, dim3(256), 0, s, a);
  }
}

template <typename T>
hipError_t launch_t(int stage, const BssnArgs& a, dim3 grid, hipStream_t s) {
  switch (stage) {
    case 0: launch_shape<0, T>(a, grid, s); break;
    case 1: launch_shape<1, T>(a, grid, s); break;
    case 2: launch_shape<2, T>(a, grid, s); break;
    case 3: launch_shape<3, T>(a, grid, s); break;
    default: launch_shape<4, T>(a, grid, s); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_bssn_stage(const Geo& G, const BssnPar& P, int stage, int precision,
                             bool images, const StageIO& io, hipStream_t s) {
  BssnArgs a;
  a.G = G;
  a.P = P;
  a.W = make_weights(P.h);
  a.io = io;
  a.images = images ? 1 : 0;
  a.ltx = G.n[0] >= 24 ? 32 : 16;
  if (forced_tile_width()) a.ltx = forced_tile_width();
  a.lty = 256 / a.ltx;
  a.tiles[0] = (G.n[0] + a.ltx - 1) / a.ltx;
  a.tiles[1] = (G.n[1] + a.lty - 1) / a.lty;
  const long long xy = (long long)a.tiles[0] * a.tiles[1];
  // global kernel: enough workgroups for several rounds per CU, each
  // marching zc planes; LDS kernel: one plane per workgroup
  const long long want = kernel_variant(precision) == 0 ? 8192 : (long long)1 << 40;
  int zsplit = (int)std::min<long long>((want + xy - 1) / xy, G.n[2]);
  if (zsplit > G.n[2]) zsplit = G.n[2];
  if (zsplit < 1) zsplit = 1;
  a.zc = (G.n[2] + zsplit - 1) / zsplit;
  a.tiles[2] = (G.n[2] + a.zc - 1) / a.zc;
  const dim3 grid((unsigned)(a.tiles[0] * a.tiles[1] * a.tiles[2]));
  return precision == CHEMORA_MIXED ? launch_t<float>(stage, a, grid, s)
                                    : launch_t<double>(stage, a, grid, s);
}

}  // namespace chemora
