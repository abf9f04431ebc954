// bssn.hip -- BSSN right-hand side over one block, alone or fused with an
// RK4 substage (Sec. III.D of arXiv:1410.1764: the Einstein equations; Sec. II:
// the time integrator).  The per-point arithmetic is in bssn_point.h.
//
// Mapping: a workgroup of 256 threads covers a tile of ltx x lty points in
// xy (ltx = 64, 32 or 16; x contiguous within a wavefront so that every
// stencil load of a wavefront is a coalesced row segment) and marches zc
// planes along z, one point per thread per plane.  Stencil neighbours come
// from the L1/L2 caches.  Tiles are laid out XCD-contiguously (xcd_tile).
#include "bssn_point.h"

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
  const long long st[3] = {1, G.sy, G.sz};
  for (int k = k0; k < k1; ++k) {
    const long long p = i + (long long)j * G.sy + (long long)k * G.sz;
    T rhs[V_N];
    bssn_rhs_point<T>(a.io.yin + G.off0 + p, G.sv, st, a.W, a.P, rhs);
    bssn_store<STAGE, T>(a.io, G, p, i, j, k, rhs, a.images != 0);
  }
}

template <typename T>
hipError_t launch_t(int stage, const BssnArgs& a, dim3 grid, hipStream_t s) {
  const dim3 block(256);
  switch (stage) {
    case 0: hipLaunchKernelGGL((bssn_stage_kernel<0, T>), grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL((bssn_stage_kernel<1, T>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((bssn_stage_kernel<2, T>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((bssn_stage_kernel<3, T>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((bssn_stage_kernel<4, T>), grid, block, 0, s, a); break;
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
  a.ltx = G.n[0] >= 48 ? 64 : (G.n[0] >= 24 ? 32 : 16);
  a.lty = 256 / a.ltx;
  a.tiles[0] = (G.n[0] + a.ltx - 1) / a.ltx;
  a.tiles[1] = (G.n[1] + a.lty - 1) / a.lty;
  const long long xy = (long long)a.tiles[0] * a.tiles[1];
  const long long want = 8192;  // workgroups: many per CU so that tails are short
  int zsplit = (int)((want + xy - 1) / xy);
  if (zsplit > G.n[2]) zsplit = G.n[2];
  if (zsplit < 1) zsplit = 1;
  a.zc = (G.n[2] + zsplit - 1) / zsplit;
  a.tiles[2] = (G.n[2] + a.zc - 1) / a.zc;
  const dim3 grid((unsigned)(a.tiles[0] * a.tiles[1] * a.tiles[2]));
  return precision == CHEMORA_MIXED ? launch_t<float>(stage, a, grid, s)
                                    : launch_t<double>(stage, a, grid, s);
}

}  // namespace chemora
