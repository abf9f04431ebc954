// batch_stage.h -- the stage kernel of the batched patch path.
// Included by one translation unit per kernel kind (batch_k*.hip), each of
// which instantiates its kind for both precisions and the substages.
//
// One launch runs one RK4 substage over a work list of interior items (one
// (patch, tile) each: right-hand side at the tile's points fused with the
// substage update) and ghost items (a chunk of one patch's ghost points: the
// analytic gauge wave at the output time, written into the output's ghost
// zones).  A staged kind has one tile shape: a kernel holding both shapes
// (selected per patch) needs the registers of both point-code copies at once
// and spills in FP64.
#pragma once

#include <type_traits>

#include "batch_kernel.h"
#include "bssn_zsrc.h"

namespace chemora {
namespace {

// Kernel kinds: 0 = cached loads (tile per patch); staged single-plane
// tiles 1 = 4th order 32x8, 2 = 4th order 16x16, 3 = 6th order 32x8,
// 4 = 8th order 32x8, 5 = 6th order 16x16, 6 = 8th order 16x16;
// 7 = 4th order, z-blocked 32x8x2 tiles of 512 threads (bssn_zsrc.h: the
// staging of the single-grid z-blocked kernels; mixed precision without
// dissipation, where the fused point code fits two waves per SIMD).
template <int KIND>
struct KindShape {
  static constexpr bool ZB = KIND == 7;
  static constexpr bool WIDE = KIND == 1 || KIND == 3 || KIND == 4 || ZB;
  static constexpr int TX = WIDE ? 32 : 16, TY = WIDE ? 8 : 16, TZ = ZB ? 2 : 1;
  static constexpr int NT = ZB ? 512 : kThreads;  // threads per workgroup
  static constexpr int WPE = ZB ? 2 : 1;          // waves per SIMD the registers must allow
  static constexpr int ORD = (KIND == 3 || KIND == 5) ? 6 : ((KIND == 4 || KIND == 6) ? 8 : 4);
  static constexpr bool HI = ORD != 4;
  // kind 0: its first two buffers hold the prolongation ghost boxes only
  static constexpr int TOT = KIND == 0 ? kBatchProlongLds
                             : ZB      ? ZShape<TX, TY, TZ>::TOTAL
                             : HI      ? HShape<TX, TY, ORD / 2 + 1>::TOTAL
                                       : LdsShape<TX, TY>::TOTAL;
  static constexpr int TOT3 = (HI || KIND == 0) ? 1 : TOT;  // third buffer: async kinds only
  static constexpr int TAB = HI ? TOT : 1;   // offset table: the high-order kinds only
};

// A prolongation ghost item: box `box` of the patch's ghost shell, every
// grid function, prolongated from the parent's time levels at time t into
// out (the stage's output).  A and Bb: two LDS buffers of kBatchProlongLds.
// Compiled only into the stage kernel's PAR instances: its code raises the
// register pressure of the whole kernel (FP64 spills of 20-36 B per lane)
// although it never runs beside the point code.
__device__ __forceinline__ void prolong_ghost_item(const Batch& B, const PatchDesc& p, int box,
                                                   double t, double* out, double* A,
                                                   double* Bb) {
  Box x;
  box_geometry(p.pb, p.PC, p.G, p.poff, box, x);
  double wt[kMaxTimeLevels] = {0.0, 0.0, 0.0};
  time_weights(p.ptimes, p.pntimes, t, wt);
  for (int v = 0; v < V_N; ++v) {
    const double* lev[kMaxTimeLevels];
#pragma unroll
    for (int l = 0; l < kMaxTimeLevels; ++l)
      lev[l] = reinterpret_cast<const double*>(B.base + p.plev[l]) + (long long)v * p.PC.sv;
    prolong_box(x, p.PC, p.G, lev, wt, p.pntimes, out + p.G.off0 + (long long)v * p.G.sv, A, Bb);
    __syncthreads();  // A and Bb are reused by the next grid function
  }
}

// one single-plane tile of a staged kind
template <int STAGE, typename T, int KIND, int KOM>
__device__ __forceinline__ void staged_tile(const PatchDesc& p, const StageIO& io, long long tile,
                                            double* const* bufs, int* tab) {
  constexpr int TX = KindShape<KIND>::TX, TY = KindShape<KIND>::TY;
  const Geo& G = p.G;
  int bx, by, k;
  patch_tile(p, tile, bx, by, k);
  const int tx = (int)threadIdx.x % TX, ty = (int)threadIdx.x / TX;
  const int x0 = bx * TX, y0 = by * TY;
  const int i = x0 + tx, j = y0 + ty;
  T rhs[V_N];
  if constexpr (KindShape<KIND>::HI) {
    constexpr int ORD = KindShape<KIND>::ORD;
    HSrc<TX, TY, ORD / 2 + 1> src;
    src.init(G, io.yin, bufs[0], bufs[1], tab, x0, y0, k, tx, ty);
    bssn_rhs_point<T, KO_OFF, ORD>(src, p.W, p.P, rhs);
  } else {
    ASrc<TX, TY, kBatchBufs> src;
    src.init(G, io.yin, bufs, x0, y0, k, tx, ty);
    bssn_rhs_point<T, KOM>(src, p.W, p.P, rhs);
  }
  if (i < G.n[0] && j < G.n[1])
    bssn_store<STAGE, T>(io, G, i + (long long)j * G.sy + (long long)k * G.sz, i, j, k, rhs,
                         false, p.P.enforce != 0);
}

// whether the kernel instance of type T and kind KIND is persistent (the
// host sizes the grid to match: batch_persistent_host)
template <typename T, int KIND>
constexpr bool batch_persistent() {
  return std::is_same<T, double>::value && KIND <= 2;
}

// one 32 x 8 x 2 tile of the z-blocked kind: thread (tx, ty, pz) evaluates
// plane k0 + pz
template <int STAGE, typename T, int KOM>
__device__ __forceinline__ void zblocked_tile(const PatchDesc& p, const StageIO& io,
                                              long long tile, double* const* bufs) {
  using K = KindShape<7>;
  const Geo& G = p.G;
  int bx, by, bz;
  patch_tile(p, tile, bx, by, bz);
  const int t = (int)threadIdx.x;
  const int tx = t % K::TX, ty = (t / K::TX) % K::TY, pz = t / (K::TX * K::TY);
  const int x0 = bx * K::TX, y0 = by * K::TY, k0 = bz * K::TZ;
  const int i = x0 + tx, j = y0 + ty, k = k0 + pz;
  ZSrc<K::TX, K::TY, K::TZ, kBatchBufs, RhsOrder> src;
  src.init(G, io.yin, bufs, x0, y0, k0, tx, ty, pz);
  T rhs[V_N];
  bssn_rhs_point<T, KOM>(src, p.W, p.P, rhs);
  if (i < G.n[0] && j < G.n[1] && k < G.n[2])
    bssn_store<STAGE, T>(io, G, i + (long long)j * G.sy + (long long)k * G.sz, i, j, k, rhs,
                         false, p.P.enforce != 0);
}

// KOM: Kreiss-Oliger dissipation compiled in (KO_ON: patches with sigma = 0
// add an exact zero) or out (KO_OFF: no patch dissipates)
// PAR: some patch of the batch has a coarse parent (prolongation ghost
// items compiled in; 4th-order kinds only)
template <int STAGE, typename T, int KIND, int KOM, bool PAR>
__global__ void __launch_bounds__(KindShape<KIND>::NT)
__attribute__((amdgpu_waves_per_eu(KindShape<KIND>::WPE))) batch_stage_kernel(Batch B) {
  constexpr int NT = KindShape<KIND>::NT;
  __shared__ int s_patch;
  constexpr int TOT = KindShape<KIND>::TOT;
  // separate arrays, one per staging buffer (see bssn_lds.h); a tiny
  // placeholder each for kind 0
  __shared__ double L0[TOT], L1[TOT], L2[KindShape<KIND>::TOT3];
  __shared__ int TB[KindShape<KIND>::TAB];
  double* bufs[3] = {L0, L1, L2};
  __shared__ long long s_lo, s_hi;  // item range of s_patch (interior or ghost)
  // The current patch's descriptor lives in LDS: under register pressure the
  // compiler re-reads descriptor fields (weights, strides) inside the point
  // code; from global memory every such read would be followed by a vmcnt
  // wait that also drains the stencil copies in flight, from LDS it waits
  // on lgkmcnt only.
  __shared__ PatchDesc s_pd;
  __shared__ int s_changed;
  const double tnow = *B.clock;
  // XCD x (blockIdx.x % 8) takes share x of the interior items and share x
  // of the ghost items, in list order; its gridDim.x / 8 blocks stride it
  const int x = (int)blockIdx.x % kNumXcd;
  const long long R = gridDim.x / kNumXcd;
  const long long ni = B.n_interior, ng = B.n_total - B.n_interior;
  const long long i0 = ni * x / kNumXcd, i1 = ni * (x + 1) / kNumXcd;
  const long long g0 = ng * x / kNumXcd, g1 = ng * (x + 1) / kNumXcd;
  const long long share = (i1 - i0) + (g1 - g0);
  if (threadIdx.x == 0) {
    s_lo = 0;
    s_hi = -1;
  }
  // Persistent (a workgroup strides its XCD's share) only where that
  // measured faster: FP64 at 4th order, whose point code holds one wave per
  // SIMD either way.  Elsewhere the grid gives every item of a share its own
  // workgroup (the hardware hands them out in order), so the item loop runs
  // once -- provably so for the compiler, which would otherwise hoist
  // thread-invariant values out of the loop and hold them through the point
  // code: mixed kinds 1/2 took 256 VGPRs + 96 AGPRs (one wave per SIMD)
  // against 241 VGPRs (two), the z-blocked kind spilled ~300 B per lane and
  // the FP64 high-order kinds 144-548 B.
  const long long step = batch_persistent<T, KIND>() ? R : share;
  for (long long t = blockIdx.x / kNumXcd; t < share; t += step) {
    const bool interior = t < i1 - i0;
    const long long item = interior ? i0 + t : ni + g0 + (t - (i1 - i0));
    __syncthreads();  // the previous item is finished by every wave
    if (threadIdx.x == 0) {
      s_changed = 0;
      if (!(item >= s_lo && item < s_hi)) {
        // consecutive items of a block mostly stay in one patch: search only
        // when the item leaves the current patch's range
        const int q = interior ? find_patch(B.prefix, B.np, item)
                               : find_patch(B.gprefix, B.np, item - ni);
        s_patch = q;
        s_lo = interior ? B.prefix[q] : ni + B.gprefix[q];
        s_hi = interior ? B.prefix[q + 1] : ni + B.gprefix[q + 1];
        s_changed = 1;
      }
    }
    __syncthreads();
    if (s_changed) {  // the same value in every thread
      static_assert(sizeof(PatchDesc) % 8 == 0, "descriptor copied in 8-byte words");
      const unsigned long long* from =
          reinterpret_cast<const unsigned long long*>(B.pd + s_patch);
      unsigned long long* to = reinterpret_cast<unsigned long long*>(&s_pd);
      for (int w = (int)threadIdx.x; w < (int)(sizeof(PatchDesc) / 8); w += NT)
        to[w] = from[w];
      __syncthreads();
    }
    const PatchDesc& p = s_pd;
    const Geo& G = p.G;
    StageIO io;
    stage_buffers(B, p, B.stage_io, io, B.dt);
    if (interior) {
      const long long tile = item - B.prefix[s_patch];
      if constexpr (KindShape<KIND>::ZB) {
        zblocked_tile<STAGE, T, KOM>(p, io, tile, bufs);
      } else if constexpr (KIND != 0) {
        staged_tile<STAGE, T, KIND, KOM>(p, io, tile, bufs, TB);
      } else {
        int tx, ty, tzi;
        patch_tile(p, tile, tx, ty, tzi);
        const int lx = (int)threadIdx.x % p.ltx, ly = (int)threadIdx.x / p.ltx;
        const int i = tx * p.ltx + lx, j = ty * p.lty + ly;
        if (ly < p.lty && i < G.n[0] && j < G.n[1]) {
          const int k0 = tzi * p.tz, k1 = min(k0 + p.tz, G.n[2]);
          for (int k = k0; k < k1; ++k) {
            const long long q = i + (long long)j * G.sy + (long long)k * G.sz;
            T rhs[V_N];
            GSrc src{io.yin + G.off0 + q, G.sv, G.sy, G.sz};
            bssn_rhs_point<T, KOM>(src, p.W, p.P, rhs);
            bssn_store<STAGE, T>(io, G, q, i, j, k, rhs, false, p.P.enforce != 0);
          }
        }
      }
    } else {
      const long long chunk = item - B.n_interior - B.gprefix[s_patch];
      const double t = tnow + B.t_out * B.dt;
      if constexpr (PAR && !KindShape<KIND>::HI) {
        static_assert(KindShape<KIND>::TOT >= kBatchProlongLds, "LDS for prolongation boxes");
        if (p.parent) {  // the same value in every thread
          prolong_ghost_item(B, p, (int)chunk, t, io.out, L0, L1);
          continue;
        }
      }
      for (long long gq = chunk * kGhostChunk + threadIdx.x;
           gq < min((chunk + 1) * kGhostChunk, p.ghosts); gq += NT) {
        int ijk[3];
        ghost_ijk(G, gq, ijk);
        const int a = p.P.gw_axis;
        const double xa = p.P.origin[a] + ijk[a] * p.P.h[a];
        gw_store(p.P, xa, t, io.out + G.off0 + ijk[0] + (long long)ijk[1] * G.sy +
                                  (long long)ijk[2] * G.sz, G.sv);
      }
    }
  }
}

template <typename T, int KIND, int KOM, bool PAR>
hipError_t launch_stage_t(int stage, const Batch& b, unsigned grid, hipStream_t st) {
  const dim3 g(grid), blk(KindShape<KIND>::NT);
  switch (stage) {
    case 0: hipLaunchKernelGGL((batch_stage_kernel<0, T, KIND, KOM, PAR>), g, blk, 0, st, b); break;
    case 1: hipLaunchKernelGGL((batch_stage_kernel<1, T, KIND, KOM, PAR>), g, blk, 0, st, b); break;
    case 2: hipLaunchKernelGGL((batch_stage_kernel<2, T, KIND, KOM, PAR>), g, blk, 0, st, b); break;
    case 3: hipLaunchKernelGGL((batch_stage_kernel<3, T, KIND, KOM, PAR>), g, blk, 0, st, b); break;
    default: hipLaunchKernelGGL((batch_stage_kernel<4, T, KIND, KOM, PAR>), g, blk, 0, st, b); break;
  }
  return hipGetLastError();
}

template <typename T, int KIND, int KOM>
hipError_t launch_stage_p(bool par, int stage, const Batch& b, unsigned grid, hipStream_t st) {
  if constexpr (!KindShape<KIND>::HI) {
    if (par) return launch_stage_t<T, KIND, KOM, true>(stage, b, grid, st);
  }
  return launch_stage_t<T, KIND, KOM, false>(stage, b, grid, st);
}

// KO_ON and PAR instances exist for the 4th-order kinds only (the high
// orders run without dissipation and without parents)
template <int KIND>
hipError_t launch_stage_kind(int precision, bool ko, bool par, int stage, const Batch& b,
                             unsigned grid, hipStream_t st) {
  if constexpr (KindShape<KIND>::ZB) {  // mixed precision without dissipation only
    if (precision != CHEMORA_MIXED || ko) return hipErrorInvalidValue;
    return launch_stage_p<float, KIND, KO_OFF>(par, stage, b, grid, st);
  } else {
    if constexpr (!KindShape<KIND>::HI) {
      if (ko)
        return precision == CHEMORA_MIXED
                   ? launch_stage_p<float, KIND, KO_ON>(par, stage, b, grid, st)
                   : launch_stage_p<double, KIND, KO_ON>(par, stage, b, grid, st);
    }
    return precision == CHEMORA_MIXED
               ? launch_stage_p<float, KIND, KO_OFF>(par, stage, b, grid, st)
               : launch_stage_p<double, KIND, KO_OFF>(par, stage, b, grid, st);
  }
}

template <typename T, int KIND, int KOM, bool PAR>
int per_cu_t() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_stage_kernel<1, T, KIND, KOM, PAR>,
                                                   KindShape<KIND>::NT, 0) != hipSuccess || n < 1)
    n = 1;
  return n;
}

template <typename T, int KIND, int KOM>
int per_cu_p(bool par) {
  if constexpr (!KindShape<KIND>::HI) {
    if (par) return per_cu_t<T, KIND, KOM, true>();
  }
  return per_cu_t<T, KIND, KOM, false>();
}

template <int KIND>
int per_cu_kind(int precision, bool ko, bool par) {
  if constexpr (KindShape<KIND>::ZB) {
    return per_cu_p<float, KIND, KO_OFF>(par);
  } else {
    if constexpr (!KindShape<KIND>::HI) {
      if (ko) return precision == CHEMORA_MIXED ? per_cu_p<float, KIND, KO_ON>(par)
                                                : per_cu_p<double, KIND, KO_ON>(par);
    }
    return precision == CHEMORA_MIXED ? per_cu_p<float, KIND, KO_OFF>(par)
                                      : per_cu_p<double, KIND, KO_OFF>(par);
  }
}

}  // namespace
}  // namespace chemora
