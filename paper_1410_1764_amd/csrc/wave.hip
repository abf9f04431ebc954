// wave.hip -- scalar wave right-hand side, eq. (1) of arXiv:1410.1764 in its
// two-variable reading (du/dt = rho, drho/dt = Laplacian u), with 4th-order
// centred differences (Sec. III.B.2), alone or fused with an RK4 substage.
//
// Memory-bound design (HBM roofline): one workgroup = a 64 x 4 xy tile, one
// wavefront per x row of 64 contiguous doubles (coalesced), marching along z.
// u along z lives in a 5-deep register queue; the current xy plane of u goes
// through LDS with a 2-point halo.  Each value of u is read from memory once
// per plane by one thread (its centre) plus the halo ring.
//
// Precision: the 2nd-derivative stencil is written on neighbour differences,
// s_a = (f(+a) - f(0)) + (f(-a) - f(0)) (a = 1, 2), d2f = (16 s_1 - s_2) / (12 h^2).
// The differences are always formed in double; the weights and the sum are
// done in T (double, or float for the mixed path).  The stage update is
// always double.
#include <cstdlib>

#include "internal.h"

namespace chemora {
namespace {

constexpr int TX = 64, TY = 4, R = 2;

struct WaveArgs {
  Geo G;
  StageIO io;
  double w2[3];  // 1 / (12 h^2)
  int zc;        // z-planes per workgroup
  int tiles[3];  // workgroups along x, y, z
  int images;    // write periodic images of the stage output
};

// Barrier between the LDS tile's writes and reads: the tile only needs the
// LDS writes done (lgkmcnt(0)); __syncthreads() would also wait for every
// global access in flight, including the next plane's prefetched operands.
// The empty asm statements keep the compiler from moving memory accesses
// across it.
__device__ __forceinline__ void tile_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt((15) | (7 << 4) | (0 << 8) | (3 << 14));  // lgkmcnt(0) only
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Pointwise operands of one plane: rho at the point, and for the substage
// update y_n (u, rho) and the accumulator (u, rho).  y_n and the accumulator
// are read once and the accumulator written once per substage, with
// nontemporal loads and stores: they then do not displace the lines of u
// that neighbouring workgroups' stencils still read from L2.
struct Pointwise {
  double rho, u0, r0, au, ar;
};

template <int STAGE>
__device__ __forceinline__ Pointwise load_pointwise(const WaveArgs& a, long long p) {
  const Geo& G = a.G;
  Pointwise w;
  w.rho = a.io.yin[G.off0 + p + G.sv];
  w.u0 = w.r0 = w.au = w.ar = 0.0;
  if (STAGE >= 2) {
    w.u0 = __builtin_nontemporal_load(&a.io.y0[G.off0 + p]);
    w.r0 = __builtin_nontemporal_load(&a.io.y0[G.off0 + p + G.sv]);
    w.au = __builtin_nontemporal_load(&a.io.acc[G.off0 + p]);
    w.ar = __builtin_nontemporal_load(&a.io.acc[G.off0 + p + G.sv]);
  }
  return w;
}

// The z-march is software-pipelined: a plane's pointwise operands are
// loaded during the previous plane, before its stores, so that they are in
// flight across the tile barriers instead of being waited for each plane.
template <int STAGE, typename T>
__global__ void __launch_bounds__(TX * TY) wave_stage_kernel(WaveArgs a) {
  __shared__ double tile[TY + 2 * R][TX + 2 * R];
  const Geo& G = a.G;
  const int nb = a.tiles[0] * a.tiles[1] * a.tiles[2];
  const int b = xcd_tile(blockIdx.x, nb);
  const int bx = b % a.tiles[0], by = (b / a.tiles[0]) % a.tiles[1], bz = b / (a.tiles[0] * a.tiles[1]);
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int i = bx * TX + tx, j = by * TY + ty;
  const int k0 = bz * a.zc;
  const int k1 = min(k0 + a.zc, G.n[2]);
  const bool comp = i < G.n[0] && j < G.n[1];
  const bool col_ok = i < G.n[0] + R && j < G.n[1] + R;
  const double* U = a.io.yin + G.off0;
  const long long col = i + (long long)j * G.sy;
  const long long sz = G.sz;

  double q0 = 0, q1 = 0, q2 = 0, q3 = 0, q4 = 0;  // u at k-2 .. k+2
  if (col_ok) {
    q0 = U[col + (k0 - 2) * sz];
    q1 = U[col + (k0 - 1) * sz];
    q2 = U[col + k0 * sz];
    q3 = U[col + (k0 + 1) * sz];
  }
  Pointwise pw{0.0, 0.0, 0.0, 0.0, 0.0};
  if (comp && k0 < k1) pw = load_pointwise<STAGE>(a, col + k0 * sz);
  const T w2x = (T)a.w2[0], w2y = (T)a.w2[1], w2z = (T)a.w2[2];

  for (int k = k0; k < k1; ++k) {
    const long long pk = col + k * sz;
    if (col_ok) q4 = U[pk + 2 * sz];
    tile_barrier();
    tile[ty + R][tx + R] = q2;
    if (tx < R && j < G.n[1] + R) tile[ty + R][tx] = U[pk - R];
    if (tx >= TX - R && i < G.n[0] && j < G.n[1] + R) tile[ty + R][tx + 2 * R] = U[pk + R];
    if (ty < R && i < G.n[0] + R) tile[ty][tx + R] = U[pk - (long long)R * G.sy];
    if (ty >= TY - R && j < G.n[1] && i < G.n[0] + R)
      tile[ty + 2 * R][tx + R] = U[pk + (long long)R * G.sy];
    tile_barrier();
    if (comp) {
      const double c = q2;
      const double sx1 = (tile[ty + R][tx + R + 1] - c) + (tile[ty + R][tx + R - 1] - c);
      const double sx2 = (tile[ty + R][tx + R + 2] - c) + (tile[ty + R][tx + R - 2] - c);
      const double sy1 = (tile[ty + R + 1][tx + R] - c) + (tile[ty + R - 1][tx + R] - c);
      const double sy2 = (tile[ty + R + 2][tx + R] - c) + (tile[ty + R - 2][tx + R] - c);
      const double sz1 = (q3 - c) + (q1 - c);
      const double sz2 = (q4 - c) + (q0 - c);
      const T lap = ((T)16 * (T)sx1 - (T)sx2) * w2x + ((T)16 * (T)sy1 - (T)sy2) * w2y +
                    ((T)16 * (T)sz1 - (T)sz2) * w2z;
      const Pointwise cur = pw;
      if (k + 1 < k1) pw = load_pointwise<STAGE>(a, pk + sz);  // before this plane's stores
      const double ku = cur.rho, kr = (double)lap;
      const long long p = pk;
      double* out = a.io.out + G.off0;
      if (STAGE == 0) {
        __builtin_nontemporal_store(ku, &out[p]);
        __builtin_nontemporal_store(kr, &out[p + G.sv]);
      } else {
        double* acc = a.io.acc + G.off0;
        const double u0 = STAGE == 1 ? c : cur.u0, r0 = STAGE == 1 ? cur.rho : cur.r0;
        double nu, nr;
        if (STAGE == 1) {
          __builtin_nontemporal_store(ku, &acc[p]);
          __builtin_nontemporal_store(kr, &acc[p + G.sv]);
          nu = u0 + a.io.cdt * ku;
          nr = r0 + a.io.cdt * kr;
        } else if (STAGE == 2 || STAGE == 3) {
          __builtin_nontemporal_store(cur.au + 2.0 * ku, &acc[p]);
          __builtin_nontemporal_store(cur.ar + 2.0 * kr, &acc[p + G.sv]);
          nu = u0 + a.io.cdt * ku;
          nr = r0 + a.io.cdt * kr;
        } else {
          nu = u0 + a.io.cdt * (cur.au + ku);
          nr = r0 + a.io.cdt * (cur.ar + kr);
        }
        if (a.images) {
          store_with_images(out, G, i, j, k, nu, true);
          store_with_images(out + G.sv, G, i, j, k, nr, true);
        } else {  // read by the next substage only after this launch: nontemporal
          __builtin_nontemporal_store(nu, &out[p]);
          __builtin_nontemporal_store(nr, &out[p + G.sv]);
        }
      }
    }
    q0 = q1;
    q1 = q2;
    q2 = q3;
    q3 = q4;
  }
}

template <typename T>
hipError_t launch_t(int stage, const WaveArgs& a, dim3 grid, hipStream_t s) {
  const dim3 block(TX * TY);
  switch (stage) {
    case 0: hipLaunchKernelGGL((wave_stage_kernel<0, T>), grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL((wave_stage_kernel<1, T>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((wave_stage_kernel<2, T>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((wave_stage_kernel<3, T>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((wave_stage_kernel<4, T>), grid, block, 0, s, a); break;
  }
  return hipGetLastError();
}

// workgroups the z-split aims for (CHEMORA_WAVE_WGS overrides; ablation
// switch, read at every launch)
long long wave_workgroups() {
  const long long v = [] {
    const char* e = std::getenv("CHEMORA_WAVE_WGS");
    const long long n = e ? std::atoll(e) : 0;
    return n >= 256 && n <= (1 << 20) ? n : 16384LL;
  }();
  return v;
}

}  // namespace

hipError_t launch_wave_stage(const Geo& G, const double h[3], int stage, int precision,
                             bool images, const StageIO& io, hipStream_t s) {
  WaveArgs a;
  a.G = G;
  a.io = io;
  for (int d = 0; d < 3; ++d) a.w2[d] = 1.0 / (12.0 * h[d] * h[d]);
  a.images = images ? 1 : 0;
  a.tiles[0] = (G.n[0] + TX - 1) / TX;
  a.tiles[1] = (G.n[1] + TY - 1) / TY;
  // enough workgroups to fill 256 CUs many times over (measured at 256^3: 16384
  // workgroups of 4 planes, 1.17 ms per RK4 step, against 1.21 ms for 4096 of 16)
  const long long xy = (long long)a.tiles[0] * a.tiles[1];
  const long long want = wave_workgroups();
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
