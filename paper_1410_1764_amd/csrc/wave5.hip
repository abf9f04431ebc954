// wave5.hip -- the scalar wave equation in the first-order form the paper
// writes down (eq. (1) of arXiv:1410.1764; Fig. 1, calculation "RHS"):
//   du/dt = rho,  drho/dt = d_i v_i,  dv_i/dt = d_i rho
// with the 4th-order centred first derivative (weights 8, -1 over 12 h on
// neighbour differences), alone or fused with an RK4 substage; and Fig. 1's
// "Energy" calculation eps = (rho^2 + v_i v_i)/2 with its grid total.
//
// Memory-bound design: a workgroup covers a 64 x 4 xy tile (one wavefront
// per contiguous x row) and marches along z; rho and v3 along z live in
// 5-deep register queues, x and y neighbours come through L1.
#include "internal.h"

namespace chemora {
namespace {

constexpr int TX = 64, TY = 4;

struct W5Args {
  Geo G;
  StageIO io;
  double w1[3];  // 1 / (12 h)
  int zc;
  int tiles[3];
  int images;
};

template <int STAGE, typename T>
__global__ void __launch_bounds__(TX * TY) wave5_stage_kernel(W5Args a) {
  const Geo& G = a.G;
  const int nb = a.tiles[0] * a.tiles[1] * a.tiles[2];
  const int b = xcd_tile(blockIdx.x, nb);
  const int bx = b % a.tiles[0], by = (b / a.tiles[0]) % a.tiles[1];
  const int bz = b / (a.tiles[0] * a.tiles[1]);
  const int i = bx * TX + (int)threadIdx.x % TX, j = by * TY + (int)threadIdx.x / TX;
  if (i >= G.n[0] || j >= G.n[1]) return;  // no LDS, no barriers in this kernel
  const int k0 = bz * a.zc, k1 = min(k0 + a.zc, G.n[2]);
  const long long sv = G.sv, sy = G.sy, sz = G.sz;
  const double* Y = a.io.yin + G.off0;
  const double* R = Y + sv;       // rho
  const double* V1 = Y + 2 * sv;  // v1
  const double* V2 = Y + 3 * sv;
  const double* V3 = Y + 4 * sv;
  const long long col = i + (long long)j * sy;
  // z queues at k-2 .. k+2
  double r0 = R[col + (k0 - 2) * sz], r1 = R[col + (k0 - 1) * sz], r2 = R[col + k0 * sz],
         r3 = R[col + (k0 + 1) * sz], r4;
  double w0 = V3[col + (k0 - 2) * sz], w1 = V3[col + (k0 - 1) * sz], w2 = V3[col + k0 * sz],
         w3 = V3[col + (k0 + 1) * sz], w4;
  const T cx = (T)a.w1[0], cy = (T)a.w1[1], cz = (T)a.w1[2];
  for (int k = k0; k < k1; ++k) {
    const long long p = col + k * sz;
    r4 = R[p + 2 * sz];
    w4 = V3[p + 2 * sz];
    auto d1 = [](double m2, double m1, double p1, double p2, T c) {
      return ((T)8 * (T)(p1 - m1) - (T)(p2 - m2)) * c;
    };
    const T drx = d1(R[p - 2], R[p - 1], R[p + 1], R[p + 2], cx);
    const T dry = d1(R[p - 2 * sy], R[p - sy], R[p + sy], R[p + 2 * sy], cy);
    const T drz = d1(r0, r1, r3, r4, cz);
    const T div = d1(V1[p - 2], V1[p - 1], V1[p + 1], V1[p + 2], cx) +
                  d1(V2[p - 2 * sy], V2[p - sy], V2[p + sy], V2[p + 2 * sy], cy) +
                  d1(w0, w1, w3, w4, cz);
    const double kv[5] = {r2, (double)div, (double)drx, (double)dry, (double)drz};
    double* out = a.io.out + G.off0;
    if (STAGE == 0) {
#pragma unroll
      for (int v = 0; v < 5; ++v) __builtin_nontemporal_store(kv[v], &out[p + v * sv]);
    } else {
      // every pointwise load before the first store (see bssn_store); y_n
      // and the accumulator are read once and the accumulator written once
      // per substage: nontemporal, so that they do not displace the stencil
      // lines neighbouring workgroups still read
      double y0[5], ac[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        y0[v] = STAGE == 1 ? Y[p + v * sv]
                           : __builtin_nontemporal_load(&a.io.y0[G.off0 + p + v * sv]);
        ac[v] = STAGE == 1 ? 0.0 : __builtin_nontemporal_load(&a.io.acc[G.off0 + p + v * sv]);
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const long long q = p + v * sv;
        double nv;
        if (STAGE == 1) {
          __builtin_nontemporal_store(kv[v], &a.io.acc[G.off0 + q]);
          nv = y0[v] + a.io.cdt * kv[v];
        } else if (STAGE == 2 || STAGE == 3) {
          __builtin_nontemporal_store(ac[v] + 2.0 * kv[v], &a.io.acc[G.off0 + q]);
          nv = y0[v] + a.io.cdt * kv[v];
        } else {
          nv = y0[v] + a.io.cdt * (ac[v] + kv[v]);
        }
        if (a.images)
          store_with_images(out + v * sv, G, i, j, k, nv, true);
        else  // read by the next substage only after this launch: nontemporal
          __builtin_nontemporal_store(nv, &out[q]);
      }
    }
    r0 = r1;
    r1 = r2;
    r2 = r3;
    r3 = r4;
    w0 = w1;
    w1 = w2;
    w2 = w3;
    w3 = w4;
  }
}

template <typename T>
hipError_t launch_t(int stage, const W5Args& a, dim3 grid, hipStream_t s) {
  const dim3 block(TX * TY);
  switch (stage) {
    case 0: hipLaunchKernelGGL((wave5_stage_kernel<0, T>), grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL((wave5_stage_kernel<1, T>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((wave5_stage_kernel<2, T>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((wave5_stage_kernel<3, T>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((wave5_stage_kernel<4, T>), grid, block, 0, s, a); break;
  }
  return hipGetLastError();
}

void plan(const Geo& G, int want, int& zc, int tiles[3]) {
  tiles[0] = (G.n[0] + TX - 1) / TX;
  tiles[1] = (G.n[1] + TY - 1) / TY;
  const long long xy = (long long)tiles[0] * tiles[1];
  int zsplit = (int)((want + xy - 1) / xy);
  if (zsplit > G.n[2]) zsplit = G.n[2];
  if (zsplit < 1) zsplit = 1;
  zc = (G.n[2] + zsplit - 1) / zsplit;
  tiles[2] = (G.n[2] + zc - 1) / zc;
}

// ---- energy: eps = (rho^2 + v.v)/2 and its sum, in a fixed order
constexpr int ET = 256;

__global__ void __launch_bounds__(ET) energy_kernel(Geo G, const double* y, double* eps,
                                                    double* partial, int zc, int t0, int t1,
                                                    int t2) {
  __shared__ double red[ET];
  const int nb = t0 * t1 * t2;
  const int b = xcd_tile(blockIdx.x, nb);
  const int bx = b % t0, by = (b / t0) % t1, bz = b / (t0 * t1);
  const int i = bx * TX + (int)threadIdx.x % TX, j = by * TY + (int)threadIdx.x / TX;
  double s = 0.0;
  if (i < G.n[0] && j < G.n[1]) {
    const int k0 = bz * zc, k1 = min(k0 + zc, G.n[2]);
    for (int k = k0; k < k1; ++k) {
      const long long p = G.off0 + i + (long long)j * G.sy + (long long)k * G.sz;
      const double r = y[p + G.sv], v1 = y[p + 2 * G.sv], v2 = y[p + 3 * G.sv],
                   v3 = y[p + 4 * G.sv];
      const double e = 0.5 * (r * r + (v1 * v1 + v2 * v2 + v3 * v3));
      if (eps) eps[p] = e;
      s += e;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = ET / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[b] = red[0];
}

__global__ void __launch_bounds__(ET) energy_total_kernel(const double* partial, int nb,
                                                          double cell, double* total) {
  __shared__ double red[ET];
  double s = 0.0;
  for (int t = threadIdx.x; t < nb; t += ET) s += partial[t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = ET / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = red[0] * cell;
}

}  // namespace

hipError_t launch_wave5_stage(const Geo& G, const double h[3], int stage, int precision,
                              bool images, const StageIO& io, hipStream_t s) {
  W5Args a;
  a.G = G;
  a.io = io;
  for (int d = 0; d < 3; ++d) a.w1[d] = 1.0 / (12.0 * h[d]);
  a.images = images ? 1 : 0;
  plan(G, 4096, a.zc, a.tiles);
  const dim3 grid((unsigned)(a.tiles[0] * a.tiles[1] * a.tiles[2]));
  return precision == CHEMORA_MIXED ? launch_t<float>(stage, a, grid, s)
                                    : launch_t<double>(stage, a, grid, s);
}

long long energy_partial_count(const Geo& G) {
  int zc, tiles[3];
  plan(G, 2048, zc, tiles);
  return (long long)tiles[0] * tiles[1] * tiles[2];
}

hipError_t launch_wave5_energy(const Geo& G, const double h[3], const double* y, double* eps,
                               double* total, double* partial, hipStream_t s) {
  int zc, tiles[3];
  plan(G, 2048, zc, tiles);
  const int nb = tiles[0] * tiles[1] * tiles[2];
  hipLaunchKernelGGL(energy_kernel, dim3(nb), dim3(ET), 0, s, G, y, eps, partial, zc, tiles[0],
                     tiles[1], tiles[2]);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(energy_total_kernel, dim3(1), dim3(ET), 0, s, partial, nb,
                     h[0] * h[1] * h[2], total);
  return hipGetLastError();
}

}  // namespace chemora
