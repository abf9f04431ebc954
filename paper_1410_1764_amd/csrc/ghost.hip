// ghost.hip -- ghost-zone kernels (the driver owns ghost zones, Sec. II of
// arXiv:1410.1764): periodic images, and the analytic gauge wave.
//
// Ghost points are enumerated compactly (no thread is spent on interior
// points) in three segments:
//   Z: the 2g z-planes outside [0, n_z), full extended xy extent;
//   Y: z in [0, n_z), the 2g y-rows outside [0, n_y), full extended x extent;
//   X: z in [0, n_z), y in [0, n_y), the 2g x-columns outside [0, n_x).
// Threads in one x row of the Z and Y segments touch consecutive addresses.
#include "internal.h"

namespace chemora {
namespace {

__device__ __forceinline__ void ghost_point(const Geo& G, long long t, int& i, int& j, int& k) {
  const int g = G.g, e0 = G.n[0] + 2 * g, e1 = G.n[1] + 2 * g;
  const long long cz = 2LL * g * e1 * e0;
  const long long cy = (long long)G.n[2] * 2 * g * e0;
  if (t < cz) {
    i = (int)(t % e0) - g;
    long long r = t / e0;
    j = (int)(r % e1) - g;
    const int p = (int)(r / e1);  // 0 .. 2g-1
    k = p < g ? p - g : G.n[2] + (p - g);
  } else if (t < cz + cy) {
    t -= cz;
    i = (int)(t % e0) - g;
    long long r = t / e0;
    const int p = (int)(r % (2 * g));
    j = p < g ? p - g : G.n[1] + (p - g);
    k = (int)(r / (2 * g));
  } else {
    t -= cz + cy;
    const int p = (int)(t % (2 * g));
    i = p < g ? p - g : G.n[0] + (p - g);
    long long r = t / (2 * g);
    j = (int)(r % G.n[1]);
    k = (int)(r / G.n[1]);
  }
}

__device__ __forceinline__ long long ghost_count(const Geo& G) {
  const int g = G.g, e0 = G.n[0] + 2 * g, e1 = G.n[1] + 2 * g;
  return 2LL * g * e1 * e0 + (long long)G.n[2] * 2 * g * e0 + (long long)G.n[2] * G.n[1] * 2 * g;
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__global__ void __launch_bounds__(256) fill_periodic_kernel(Geo G, double* state) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ghost_count(G)) return;
  int i, j, k;
  ghost_point(G, t, i, j, k);
  double* f = state + G.off0 + (long long)blockIdx.y * G.sv;
  const long long src = wrap(i, G.n[0]) + (long long)wrap(j, G.n[1]) * G.sy +
                        (long long)wrap(k, G.n[2]) * G.sz;
  f[i + (long long)j * G.sy + (long long)k * G.sz] = f[src];
}

// BSSN variables of the gauge wave ds^2 = -H dt^2 + H dx_a^2 + dx_b^2 + dx_c^2,
// H = 1 - A sin(2 pi (x_a - t)/d), zero shift (exact under harmonic slicing):
// chi = H^-1/3, gt_aa = H^2/3, gt_bb = H^-1/3, K = -(pi A/d) cos H^-3/2,
// At_aa = -(2 pi A/3d) cos H^-5/6, At_bb = (pi A/3d) cos H^-11/6,
// Gamt^a = -(4 pi A/3d) cos H^-5/3, alpha = sqrt(H); everything else 0.
__device__ __forceinline__ void gaugewave_values(const BssnPar& P, double xa, double t,
                                                 double v[24]) {
  const double pi = 3.141592653589793;
  const double A = P.gw_A, d = P.gw_d;
  const int a = P.gw_axis;
  double s, c;
  sincos(2.0 * pi * (xa - t) / d, &s, &c);
  const double H = 1.0 - A * s;
  const double L = log(H);
  const double Hm13 = exp(-L / 3.0);
  for (int q = 0; q < 24; ++q) v[q] = 0.0;
  v[0] = Hm13;
  const int diag[3] = {1, 4, 6};  // gt11, gt22, gt33
  for (int b = 0; b < 3; ++b) {
    if (b == a) {
      v[diag[b]] = exp(2.0 * L / 3.0);
      v[7 + diag[b]] = -(2.0 * pi * A / (3.0 * d)) * c * exp(-5.0 * L / 6.0);
    } else {
      v[diag[b]] = Hm13;
      v[7 + diag[b]] = (pi * A / (3.0 * d)) * c * exp(-11.0 * L / 6.0);
    }
  }
  v[7] = -(pi * A / d) * c * exp(-1.5 * L);
  const double gam = -(4.0 * pi * A / (3.0 * d)) * c * exp(-5.0 * L / 3.0);
#pragma unroll
  for (int b = 0; b < 3; ++b) v[14 + b] = b == a ? gam : 0.0;  // constant indices
  v[17] = sqrt(H);
}

__global__ void __launch_bounds__(256) fill_gaugewave_kernel(Geo G, BssnPar P, double t,
                                                             double* state) {
  const long long tt = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tt >= ghost_count(G)) return;
  int ijk[3];
  ghost_point(G, tt, ijk[0], ijk[1], ijk[2]);
  const int a = P.gw_axis;
  const double xa = P.origin[a] + ijk[a] * P.h[a];
  double v[24];
  gaugewave_values(P, xa, t, v);
  double* f = state + G.off0 + ijk[0] + (long long)ijk[1] * G.sy + (long long)ijk[2] * G.sz;
#pragma unroll
  for (int q = 0; q < 24; ++q) f[q * G.sv] = v[q];
}

long long host_ghost_count(const Geo& G) {
  const int g = G.g;
  const long long e0 = G.n[0] + 2 * g, e1 = G.n[1] + 2 * g;
  return 2LL * g * e1 * e0 + (long long)G.n[2] * 2 * g * e0 + (long long)G.n[2] * G.n[1] * 2 * g;
}

}  // namespace

hipError_t launch_fill_periodic(const Geo& G, int nvar, double* state, hipStream_t s) {
  const long long cnt = host_ghost_count(G);
  if (cnt == 0 || nvar == 0) return hipSuccess;
  dim3 grid((unsigned)((cnt + 255) / 256), (unsigned)nvar);
  hipLaunchKernelGGL(fill_periodic_kernel, grid, dim3(256), 0, s, G, state);
  return hipGetLastError();
}

hipError_t launch_fill_gaugewave(const Geo& G, const BssnPar& P, double t, double* state,
                                 hipStream_t s) {
  const long long cnt = host_ghost_count(G);
  if (cnt == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_gaugewave_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                     G, P, t, state);
  return hipGetLastError();
}

}  // namespace chemora
