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
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "bssn_args.h"

namespace chemora {
namespace {

// CHEMORA_BSSN_WAVES: minimum waves per SIMD the register allocator must
// allow (an ablation switch; 1 lets the FP64 kernel use VGPRs + AGPRs).
#ifndef CHEMORA_BSSN_WAVES
#define CHEMORA_BSSN_WAVES 1
#endif

template <int STAGE, typename T, int KOM, int ORD>
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
    bssn_rhs_point<T, KOM, ORD>(src, a.W, a.P, rhs);
    bssn_store<STAGE, T>(a.io, G, p, i, j, k, rhs, a.images != 0, a.P.enforce != 0);
  }
}

template <int STAGE, typename T, int TX, int TY, int KOM>
__global__ void __launch_bounds__(TX * TY) bssn_lds_kernel(BssnArgs a) {
  using S = LdsShape<TX, TY>;
  __shared__ double lds[2 * S::TOTAL];
  const Geo& G = a.G;
  int bx, by, bz;
  if (!plane_tile(a, blockIdx.x, bx, by, bz)) return;  // whole workgroup: no barrier yet
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
  bssn_rhs_point<T, KOM>(src, a.W, a.P, rhs);
  if (active)
    bssn_store<STAGE, T>(a.io, G, i + (long long)j * G.sy + (long long)k * G.sz, i, j, k, rhs,
                         a.images != 0, a.P.enforce != 0);
}

// 6th- and 8th-order operators: the tile's radius-(order/2 + 1)
// neighbourhood of each grid function staged in LDS with asynchronous
// copies (AHSrc, three buffers: two grid functions in flight), one plane per
// workgroup, no dissipation
template <int STAGE, typename T, int TX, int TY, int ORD>
__global__ void __launch_bounds__(TX * TY) bssn_hi_kernel(BssnArgs a) {
  constexpr int R = ORD / 2 + 1;
  using S = HShape<TX, TY, R>;
  __shared__ double L0[S::TOTAL], L1[S::TOTAL], L2[S::TOTAL];
  double* const bufs[3] = {L0, L1, L2};
  const Geo& G = a.G;
  int bx, by, k;
  if (!plane_tile(a, blockIdx.x, bx, by, k)) return;  // whole workgroup: no barrier yet
  const int tx = (int)threadIdx.x % TX, ty = (int)threadIdx.x / TX;
  const int x0 = bx * TX, y0 = by * TY;
  const int i = x0 + tx, j = y0 + ty;
  const bool active = i < G.n[0] && j < G.n[1];
  AHSrc<TX, TY, R, 3> src;
  src.init(G, a.io.yin, bufs, x0, y0, k, tx, ty);
  T rhs[V_N];
  bssn_rhs_point<T, KO_OFF, ORD>(src, a.W, a.P, rhs);
  if (active)
    bssn_store<STAGE, T>(a.io, G, i + (long long)j * G.sy + (long long)k * G.sz, i, j, k, rhs,
                         a.images != 0, a.P.enforce != 0);
}

template <int STAGE, typename T, int TX, int TY, int NBUF, int KOM>
__global__ void __launch_bounds__(TX * TY) bssn_async_kernel(BssnArgs a) {
  static_assert(NBUF >= 2 && NBUF <= 6, "1 to 5 grid functions in flight");
  using S = LdsShape<TX, TY>;
  // separate arrays, one per buffer (see ASrc); unused ones are not allocated
  __shared__ double L0[S::TOTAL], L1[S::TOTAL], L2[S::TOTAL], L3[S::TOTAL], L4[S::TOTAL],
      L5[S::TOTAL];
  double* const bufs[6] = {L0, L1, L2, L3, L4, L5};
  const Geo& G = a.G;
  int bx, by, k;
  if (!plane_tile(a, blockIdx.x, bx, by, k)) return;  // whole workgroup: no barrier yet
  const int tx = (int)threadIdx.x % TX, ty = (int)threadIdx.x / TX;
  const int x0 = bx * TX, y0 = by * TY;
  const int i = x0 + tx, j = y0 + ty;
  const bool active = i < G.n[0] && j < G.n[1];
  ASrc<TX, TY, NBUF> src;
  src.init(G, a.io.yin, bufs, x0, y0, k, tx, ty);
  T rhs[V_N];
  bssn_rhs_point<T, KOM>(src, a.W, a.P, rhs);
  if (active)
    bssn_store<STAGE, T>(a.io, G, i + (long long)j * G.sy + (long long)k * G.sz, i, j, k, rhs,
                         a.images != 0, a.P.enforce != 0);
}

// CHEMORA_BSSN_TILE=WxH forces the tile of the staged kernels (64x4, 32x8,
// 16x16: 256 threads; 16x8: 128; 16x4, 8x8: 64), and a single width W the
// tile W x (256 / W) (ablation switch, read at every launch)
struct TileShape {
  int w, h;
};
TileShape forced_tile() {
  const TileShape t = [] {
    const char* e = std::getenv("CHEMORA_BSSN_TILE");
    TileShape r{0, 0};
    if (!e) return r;
    int w = 0, h = 0;
    if (std::sscanf(e, "%dx%d", &w, &h) == 2) {
      r = {w, h};
    } else if (std::sscanf(e, "%d", &w) == 1) {
      r = {w, w > 0 ? 256 / w : 0};
    }
    const bool ok = (r.w == 64 && r.h == 4) || (r.w == 32 && r.h == 8) ||
                    (r.w == 16 && (r.h == 16 || r.h == 8 || r.h == 4)) || (r.w == 8 && r.h == 8);
    return ok ? r : TileShape{0, 0};
  }();
  return t;
}

// Kernel choice (measured at 128^3): async staging with three buffers in both
// precisions (FP64 0.757 ms, mixed 0.584 ms; six buffers: 0.764 / 0.758 ms;
// register-prefetched LDS staging: 0.766 / 0.641 ms).  Three buffers
// (66 KB) let two mixed-precision workgroups share a CU, so the mixed
// kernel (245 VGPRs) runs two waves per SIMD.
// CHEMORA_BSSN_KERNEL=global|lds|async overrides it (ablation switch, read at
// every launch).
int kernel_override() {
  const int v = [] {
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
  (void)precision;
  return o >= 0 ? o : 2;
}

// CHEMORA_BSSN_NBUF=6: six staging buffers for the async 32x8 kernel
// instead of three (ablation switch, read at every launch)
int async_nbuf() {
  const int v = [] {
    const char* e = std::getenv("CHEMORA_BSSN_NBUF");
    return (e && std::atoi(e) == 6) ? 6 : 3;
  }();
  return v;
}

// CHEMORA_BSSN_ORDER=plane restores the XCD-contiguous plane order of the
// staged kernels instead of the column walk (ablation switch, read at every
// launch)
bool column_order() {
  const bool v = [] {
    const char* e = std::getenv("CHEMORA_BSSN_ORDER");
    return !(e && std::strcmp(e, "plane") == 0);
  }();
  return v;
}

template <int STAGE, typename T, int KOM>
void launch_shape_k(const BssnArgs& a, dim3 grid, hipStream_t s) {
  int variant = kernel_variant(sizeof(T) == 4 ? CHEMORA_MIXED : CHEMORA_FP64);
  const int nt = a.ltx * a.lty;
  if (variant == 1 && nt != 256) variant = 2;  // the prefetched LDS source needs 256 threads
  if (variant == 0) {
    hipLaunchKernelGGL((bssn_stage_kernel<STAGE, T, KOM, 4>), grid, dim3(256), 0, s, a);
  } else if (variant == 2) {
    if (a.ltx == 32 && async_nbuf() == 3) {
      hipLaunchKernelGGL((bssn_async_kernel<STAGE, T, 32, 8, 3, KOM>), grid, dim3(nt), 0, s, a);
    } else if (a.ltx == 32) {
      hipLaunchKernelGGL((bssn_async_kernel<STAGE, T, 32, 8, 6, KOM>), grid, dim3(nt), 0, s, a);
    } else if (a.ltx == 16 && a.lty == 16) {
      hipLaunchKernelGGL((bssn_async_kernel<STAGE, T, 16, 16, 6, KOM>), grid, dim3(nt), 0, s, a);
    } else if constexpr (KOM == KO_OFF) {  // ablation shapes: without dissipation only
      if (a.ltx == 64)
        hipLaunchKernelGGL((bssn_async_kernel<STAGE, T, 64, 4, 5, KOM>), grid, dim3(nt), 0, s, a);
      else if (a.ltx == 8)
        hipLaunchKernelGGL((bssn_async_kernel<STAGE, T, 8, 8, 5, KOM>), grid, dim3(nt), 0, s, a);
      else if (a.lty == 4)
        hipLaunchKernelGGL((bssn_async_kernel<STAGE, T, 16, 4, 5, KOM>), grid, dim3(nt), 0, s, a);
      else
        hipLaunchKernelGGL((bssn_async_kernel<STAGE, T, 16, 8, 6, KOM>), grid, dim3(nt), 0, s, a);
    }
  } else if (a.ltx == 32) {
    hipLaunchKernelGGL((bssn_lds_kernel<STAGE, T, 32, 8, KOM>), grid, dim3(256), 0, s, a);
  } else if (a.ltx == 16) {
    hipLaunchKernelGGL((bssn_lds_kernel<STAGE, T, 16, 16, KOM>), grid, dim3(256), 0, s, a);
  } else if constexpr (KOM == KO_OFF) {
    hipLaunchKernelGGL((bssn_lds_kernel<STAGE, T, 64, 4, KOM>), grid, dim3(256), 0, s, a);
  }
}

// dissipation on or off: separate instances, so that the default kernels
// keep their register budget
template <int STAGE, typename T>
void launch_shape(const BssnArgs& a, dim3 grid, hipStream_t s) {
  // orders 6 and 8, without dissipation: their own staged kernel (wider
  // halos), or the cached-load kernel (CHEMORA_BSSN_KERNEL=global)
  if (a.P.fd_order == 6 || a.P.fd_order == 8) {
    const bool cached = kernel_variant(sizeof(T) == 4 ? CHEMORA_MIXED : CHEMORA_FP64) == 0;
    if (a.P.fd_order == 6) {
      if (cached)
        hipLaunchKernelGGL((bssn_stage_kernel<STAGE, T, KO_OFF, 6>), grid, dim3(256), 0, s, a);
      else if (a.ltx == 32)
        hipLaunchKernelGGL((bssn_hi_kernel<STAGE, T, 32, 8, 6>), grid, dim3(256), 0, s, a);
      else
        hipLaunchKernelGGL((bssn_hi_kernel<STAGE, T, 16, 16, 6>), grid, dim3(256), 0, s, a);
    } else {
      if (cached)
        hipLaunchKernelGGL((bssn_stage_kernel<STAGE, T, KO_OFF, 8>), grid, dim3(256), 0, s, a);
      else if (a.ltx == 32)
        hipLaunchKernelGGL((bssn_hi_kernel<STAGE, T, 32, 8, 8>), grid, dim3(256), 0, s, a);
      else
        hipLaunchKernelGGL((bssn_hi_kernel<STAGE, T, 16, 16, 8>), grid, dim3(256), 0, s, a);
    }
    return;
  }
  if (a.P.ko_sigma != 0.0)
    launch_shape_k<STAGE, T, KO_ON>(a, grid, s);
  else
    launch_shape_k<STAGE, T, KO_OFF>(a, grid, s);
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
  a.W = make_weights(P.h, P.ko_sigma, P.fd_order);
  a.io = io;
  a.images = images ? 1 : 0;
  a.ltx = G.n[0] >= 24 ? 32 : 16;
  a.lty = 256 / a.ltx;
  // with dissipation only the default tiles exist (forced tiles are an
  // ablation of the dissipation-free kernels)
  if (P.ko_sigma != 0.0 || P.fd_order != 4) {
  } else if (kernel_variant(precision) != 0 && forced_tile().w) {
    a.ltx = forced_tile().w;
    a.lty = forced_tile().h;
  } else if (forced_tile().w && forced_tile().w * forced_tile().h == 256) {
    a.ltx = forced_tile().w;
    a.lty = forced_tile().h;
  }
  a.tiles[0] = (G.n[0] + a.ltx - 1) / a.ltx;
  a.tiles[1] = (G.n[1] + a.lty - 1) / a.lty;
  const long long xy = (long long)a.tiles[0] * a.tiles[1];
  // global kernel: enough workgroups for several rounds per CU, each
  // marching zc planes; LDS kernel: one plane per workgroup
  const bool cached = kernel_variant(precision) == 0;
  const long long want = cached ? 8192 : (long long)1 << 40;
  int zsplit = (int)std::min<long long>((want + xy - 1) / xy, G.n[2]);
  if (zsplit > G.n[2]) zsplit = G.n[2];
  if (zsplit < 1) zsplit = 1;
  a.zc = (G.n[2] + zsplit - 1) / zsplit;
  a.tiles[2] = (G.n[2] + a.zc - 1) / a.zc;
  long long blocks = (long long)a.tiles[0] * a.tiles[1] * a.tiles[2];
  a.cols[0] = a.cols[1] = 0;
  if (!cached && column_order()) {
    const ColumnSplit c = column_split(a.tiles, a.ltx, a.lty);
    if (c.cx > 0) {
      a.cols[0] = c.cx;
      a.cols[1] = c.cy;
      blocks = c.blocks_per_plane * a.tiles[2];
    }
  }
  const dim3 grid((unsigned)blocks);
  hipError_t err = hipSuccess;
  if (kernel_variant(precision) == 2 && launch_bssn_split(stage, precision, a, grid, s, &err))
    return err;
  return precision == CHEMORA_MIXED ? launch_t<float>(stage, a, grid, s)
                                    : launch_t<double>(stage, a, grid, s);
}

}  // namespace chemora
