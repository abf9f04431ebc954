// bssn_zsrc.h -- z-blocked LDS staging for the 4th-order BSSN point code:
// a workgroup of TX*TY*TZ threads evaluates TZ consecutive z-planes of a
// TX x TY tile (one point per thread), so the staged neighbourhood of each
// grid function serves TZ planes.  For 32 x 8 x 2 that is 7.2 staged values
// per point and grid function, against 10.8 for one plane of 32 x 8: the
// z neighbours of one output plane are the other plane's own data.
//
// Staged planes of one grid function, for output planes k0 .. k0+TZ-1:
//   A: plane k0-3, the tile only (z-lopsided and dissipation reach);
//   R: planes k0-2 .. k0+TZ+1, each the tile with a 3-point halo in x and y
//      (one width for every plane, so that stencil offsets are constants);
//   C: plane k0+TZ+2, the tile only.
// The copies are gfx950's asynchronous global_load_lds_dwordx4, as in ASrc
// (bssn_lds.h): NBUF separate buffers, NBUF-1 grid functions in flight,
// hand-off = vmcnt wait + barrier.
#pragma once

#include "bssn_lds.h"

namespace chemora {

template <int TX, int TY, int TZ>
struct ZShape {
  static constexpr int NT = TX * TY * TZ;
  static constexpr int W = TX + 6, H = TY + 6, PL = W * H;
  static constexpr int NR = TZ + 4;  // R planes: dz = -2 .. TZ+1 from k0
  static constexpr int N3 = TX * TY;
  static constexpr int TOTAL = N3 + NR * PL + N3;
};

// Accessor for the thread at tile position (tx, ty), block plane pz.
// r: its window's low corner (tx-3, ty-3) in the R plane of dz = -2;
// m3 / p3: its own point in the planes 3 below and 3 above.
template <int TX, int TY, int TZ>
struct ZAcc {
  using S = ZShape<TX, TY, TZ>;
  const double* r;
  const double* m3;
  const double* p3;
  __device__ __forceinline__ double operator()(int dx, int dy, int dz) const {
    if (dz == 3) return p3[0];
    if (dz == -3) return m3[0];
    return r[(dz + 2) * S::PL + (dy + 3) * S::W + dx + 3];
  }
  // +-(dx,dy,dz): in-plane (x or y axis) or the z axis at distance 3
  __device__ __forceinline__ double sel(bool up, int dx, int dy, int dz) const {
    if (dz == 0) {
      const int c = 2 * S::PL + 3 * S::W + 3, o = dy * S::W + dx;
      return r[up ? c + o : c - o];
    }
    return up ? p3[0] : m3[0];
  }
};

template <int TX, int TY, int TZ, int NBUF, typename ORDER>
struct ZSrc {
  using S = ZShape<TX, TY, TZ>;
  static constexpr int PAIRS = S::TOTAL / 2;
  static constexpr int PSLOTS = (PAIRS + S::NT - 1) / S::NT;
  static constexpr int D = NBUF - 1;
  static_assert(S::N3 % 2 == 0 && S::W % 2 == 0 && TX % 2 == 0, "pairs must not straddle rows");
  static_assert(S::NT % 64 == 0, "whole wavefronts");
  double* buf[NBUF];
  const char* Yb;        // stage input allocation (byte address)
  const double* Yc;      // centre value of variable 0 at the thread's (clamped) point
  long long sv;          // elements between grid functions
  unsigned off[PSLOTS];  // byte offset from Yb of each pair slot (variable 0)
  int ro, m3o, p3o;      // the thread's offsets inside one buffer
  int seq;
  int wbase;             // 64 * wave index

  // tile origin (x0, y0), first plane k0, thread position (tx, ty, pz)
  __device__ __forceinline__ void init(const Geo& G, const double* yin, double* const* shared,
                                       int x0, int y0, int k0, int tx, int ty, int pz) {
#pragma unroll
    for (int b = 0; b < NBUF; ++b) buf[b] = shared[b];
    Yb = reinterpret_cast<const char*>(yin);
    sv = G.sv;
    const int tid = (pz * TY + ty) * TX + tx;
    wbase = tid & ~63;
#pragma unroll
    for (int m = 0; m < PSLOTS; ++m) {
      int p = tid + m * S::NT;
      if (p >= PAIRS) p = 0;  // masked off at issue
      const int t = 2 * p;
      int px, py, dz;
      if (t < S::N3) {
        dz = -3;
        py = t / TX;
        px = t % TX;
      } else if (t < S::N3 + S::NR * S::PL) {
        const int q = t - S::N3, rp = q / S::PL, e = q % S::PL;
        dz = rp - 2;
        py = e / S::W - 3;
        px = e % S::W - 3;
      } else {
        const int e = t - S::N3 - S::NR * S::PL;
        dz = TZ + 2;
        py = e / TX;
        px = e % TX;
      }
      // pair start in [-g-1, n+g-1] keeps both doubles inside the padded
      // row; rows and planes clamped into the block (ragged tiles)
      int gx = x0 + px, gy = y0 + py, gz = k0 + dz;
      gx = gx < -G.g - 1 ? -G.g - 1 : (gx > G.n[0] + G.g - 1 ? G.n[0] + G.g - 1 : gx);
      gy = gy < -G.g ? -G.g : (gy > G.n[1] + G.g - 1 ? G.n[1] + G.g - 1 : gy);
      gz = gz < -G.g ? -G.g : (gz > G.n[2] + G.g - 1 ? G.n[2] + G.g - 1 : gz);
      off[m] = (unsigned)(8 * (G.off0 + gx + (long long)gy * G.sy + (long long)gz * G.sz));
    }
    ro = S::N3 + pz * S::PL + ty * S::W + tx;
    m3o = pz == 0 ? ty * TX + tx : S::N3 + (pz - 1) * S::PL + (ty + 3) * S::W + tx + 3;
    p3o = pz == TZ - 1 ? S::N3 + S::NR * S::PL + ty * TX + tx
                       : S::N3 + (pz + 5) * S::PL + (ty + 3) * S::W + tx + 3;
    const int ci = x0 + tx < G.n[0] ? x0 + tx : G.n[0] - 1;
    const int cj = y0 + ty < G.n[1] ? y0 + ty : G.n[1] - 1;
    const int ck = k0 + pz < G.n[2] ? k0 + pz : G.n[2] - 1;
    Yc = yin + G.off0 + ci + (long long)cj * G.sy + (long long)ck * G.sz;
    seq = 0;
  }

  // start copying grid function ORDER::at(s) into buffer s % NBUF
  __device__ __forceinline__ void issue(int s) {
    const char* base = Yb + (long long)ORDER::at(s) * sv * 8;
    double* dst = buf[s % NBUF];
    const int lane = (int)threadIdx.x & 63;
#pragma unroll
    for (int m = 0; m < PSLOTS; ++m) {
      if (m < PSLOTS - 1 || wbase + lane + m * S::NT < PAIRS) {
        __builtin_amdgcn_global_load_lds((gbl_void_t*)(base + off[m]),
                                         (lds_void_t*)(dst + 2 * (m * S::NT + wbase)), 16, 0, 0);
      }
    }
  }

  __device__ __forceinline__ double center(int v) const { return Yc[v * sv]; }
  // the centre value of a grid function this kernel does not stage: read once
  // per point, so with a nontemporal load that does not displace staged lines
  __device__ __forceinline__ double center_nt(int v) const {
    return __builtin_nontemporal_load(&Yc[v * sv]);
  }

  template <int YOUNGER>
  __device__ __forceinline__ void wait_and_sync() {
    wait_vm_lgkm0<YOUNGER * (PSLOTS - 1)>();
    fence_memory();
    __builtin_amdgcn_s_barrier();
    fence_memory();
  }

  __device__ __forceinline__ ZAcc<TX, TY, TZ> acquire(int /*v*/) {
    if (seq == 0) {
      // issued after the point's centre loads (kept older by the fence), so
      // that waiting for a centre value never drains the copies
      fence_memory();
#pragma unroll
      for (int s = 0; s < D; ++s) issue(s);
    }
    const int last = seq + D - 1 < ORDER::N - 1 ? seq + D - 1 : ORDER::N - 1;
    switch (last - seq) {  // folds to one case once seq is known
      case 0: wait_and_sync<0>(); break;
      case 1: wait_and_sync<1>(); break;
      case 2: wait_and_sync<2>(); break;
      case 3: wait_and_sync<3>(); break;
      default: wait_and_sync<4>(); break;
    }
    if (seq + D < ORDER::N) issue(seq + D);
    double* b = buf[seq % NBUF];
    ++seq;
    return ZAcc<TX, TY, TZ>{b + ro, b + m3o, b + p3o};
  }
};

}  // namespace chemora
