// bssn_lds.h -- LDS-staged source for the BSSN point code (bssn_point.h).
//
// A workgroup of TX*TY threads evaluates one TX x TY tile of a z-plane (one
// point per thread).  The 24 grid functions are
// differentiated one after another (kRhsOrder); for each one the workgroup
// stages the tile's stencil neighbourhood in LDS with one cooperative burst
// of loads, and every thread then reads its ~70 stencil values from LDS
// (low latency, no L1 traffic) instead of from the caches.
//
// Neighbourhood of a TX x TY tile at plane k (union of the stencils of its
// points): plane k with a 3-point halo in x and y (axis and lopsided
// stencils, xy mixed derivatives); planes k+-1 and k+-2 with a 2-point halo
// (xz and yz mixed derivatives, z axis); planes k+-3 without halo (z
// lopsided).  For 64 x 4 that is 700 + 4*544 + 2*256 = 3388 doubles.
//
// Double buffering: while the threads differentiate grid function s from
// one buffer, the loads of grid function s+1 are already in flight into
// registers; acquire(s+1) writes them to the other buffer and synchronises.
// One barrier per grid function.  Out-of-grid tile points (ragged tiles)
// read clamped addresses; their results are never stored.
#pragma once

#include "bssn_point.h"

namespace chemora {

template <int TX, int TY>
struct LdsShape {
  static constexpr int NT = TX * TY;
  static constexpr int W0 = TX + 6, H0 = TY + 6;  // plane k, halo 3
  static constexpr int W1 = TX + 4, H1 = TY + 4;  // planes k+-1, k+-2, halo 2
  static constexpr int N0 = W0 * H0, N1 = W1 * H1, N3 = TX * TY;
  // segments in order: k | k+1 | k-1 | k+2 | k-2 | k+3 | k-3
  static constexpr int TOTAL = N0 + 4 * N1 + 2 * N3;
  static constexpr int SLOTS = (TOTAL + NT - 1) / NT;
};

// Accessor into one staged buffer for the thread at tile position (tx, ty).
// The bases point at the low corner of the thread's window, so that every
// stencil offset is a non-negative constant (ds_read takes an unsigned
// immediate offset; a negative one would cost an address register each).
template <int TX, int TY>
struct LAcc {
  using S = LdsShape<TX, TY>;
  const double* b0;  // plane k at (tx - 3, ty - 3)
  const double* b1;  // plane k+1 at (tx - 2, ty - 2); k-1, k+2, k-2 follow at N1 strides
  const double* b3;  // plane k+3 at (tx, ty); k-3 follows at N3
  __device__ __forceinline__ double operator()(int dx, int dy, int dz) const {
    if (dz == 0) return b0[(dy + 3) * S::W0 + dx + 3];
    if (dz == 3) return b3[0];
    if (dz == -3) return b3[S::N3];
    const int seg = dz == 1 ? 0 : (dz == -1 ? 1 : (dz == 2 ? 2 : 3));
    return b1[seg * S::N1 + (dy + 2) * S::W1 + dx + 2];
  }
  // +-(dx,dy,dz): in-plane (x or y axis) or the z axis at distance 3
  __device__ __forceinline__ double sel(bool up, int dx, int dy, int dz) const {
    if (dz == 0) {
      const int c = 3 * S::W0 + 3, o = dy * S::W0 + dx;
      return b0[up ? c + o : c - o];
    }
    return b3[up ? 0 : S::N3];
  }
};

template <int TX, int TY>
struct LSrc {
  using S = LdsShape<TX, TY>;
  double* lds0;      // buffer for even-numbered grid functions (TOTAL doubles)
  double* lds1;      // buffer for odd-numbered ones
  const double* Yt;  // yin + off0: tile addressing base (variable 0)
  const double* Yc;  // centre value of variable 0 at the thread's (clamped) point
  long long sv;
  int off[S::SLOTS];     // element offset of each staged slot (variable 0)
  double reg[S::SLOTS];  // loads in flight for the next grid function
  int b0o, b1o, b3o;     // the thread's element offsets inside one buffer
  int seq;               // grid functions acquired at this point so far

  // tile origin (x0, y0), plane k, thread position (tx, ty)
  __device__ __forceinline__ void init(const Geo& G, const double* yin, double* buf0,
                                       double* buf1, int x0, int y0, int k, int tx, int ty) {
    lds0 = buf0;
    lds1 = buf1;
    Yt = yin + G.off0;
    sv = G.sv;
    const int tid = ty * TX + tx;
#pragma unroll
    for (int m = 0; m < S::SLOTS; ++m) {
      int t = tid + m * S::NT;
      if (t >= S::TOTAL) t = 0;  // beyond the buffer: load slot 0 again, never stored
      int px, py, dz;
      if (t < S::N0) {
        dz = 0;
        py = t / S::W0 - 3;
        px = t % S::W0 - 3;
      } else if (t < S::N0 + 4 * S::N1) {
        const int r = t - S::N0, s = r / S::N1, q = r % S::N1;
        dz = (s == 0) ? 1 : (s == 1 ? -1 : (s == 2 ? 2 : -2));
        py = q / S::W1 - 2;
        px = q % S::W1 - 2;
      } else {
        const int r = t - S::N0 - 4 * S::N1, s = r / S::N3, q = r % S::N3;
        dz = s == 0 ? 3 : -3;
        py = q / TX;
        px = q % TX;
      }
      int gx = x0 + px, gy = y0 + py;
      gx = gx < -G.g ? -G.g : (gx > G.n[0] + G.g - 1 ? G.n[0] + G.g - 1 : gx);
      gy = gy < -G.g ? -G.g : (gy > G.n[1] + G.g - 1 ? G.n[1] + G.g - 1 : gy);
      off[m] = gx + gy * G.sy + (k + dz) * G.sz;
    }
    b0o = ty * S::W0 + tx;
    b1o = S::N0 + ty * S::W1 + tx;
    b3o = S::N0 + 4 * S::N1 + ty * TX + tx;
    const int ci = x0 + tx < G.n[0] ? x0 + tx : G.n[0] - 1;
    const int cj = y0 + ty < G.n[1] ? y0 + ty : G.n[1] - 1;
    Yc = Yt + ci + (long long)cj * G.sy + (long long)k * G.sz;
    seq = 0;
  }

  __device__ __forceinline__ void prefetch(int v) {
    const double* base = Yt + v * sv;
#pragma unroll
    for (int m = 0; m < S::SLOTS; ++m) reg[m] = base[off[m]];
  }

  __device__ __forceinline__ double center(int v) const { return Yc[v * sv]; }

  // the staged neighbourhood of grid function kRhsOrder[seq] (== v)
  __device__ __forceinline__ LAcc<TX, TY> acquire(int /*v*/) {
    double* buf = (seq & 1) ? lds1 : lds0;
    const int tid = (int)threadIdx.x;
#pragma unroll
    for (int m = 0; m < S::SLOTS; ++m) {
      const int t = tid + m * S::NT;
      if (m < S::SLOTS - 1 || t < S::TOTAL) buf[t] = reg[m];
    }
    __syncthreads();
    if (seq + 1 < V_N) prefetch(kRhsOrder[seq + 1]);
    ++seq;
    return LAcc<TX, TY>{buf + b0o, buf + b1o, buf + b3o};
  }
};

// ---------------------------------------------------------------------------
// Staging for the 6th- and 8th-order operators (stencil radius R = order/2 + 1,
// the reach of the lopsided stencil).  Neighbourhood of a TX x TY tile at
// plane k: plane k with an R-point halo in x and y (axis and lopsided
// stencils, xy mixed derivatives); planes k+-1 .. k+-(R-1) with an
// (R-1)-point halo (xz and yz mixed derivatives, z axis); planes k+-R without
// halo (z lopsided).  Two buffers, one barrier per grid function: the
// workgroup loads grid function s into one buffer while no thread can still
// be reading the grid function two before it.  The element offsets of the
// staged points are computed once per workgroup into an LDS table, so the
// per-variable copy is a table lookup, a load and an LDS store per slot.
template <int TX, int TY, int R>
struct HShape {
  static constexpr int NT = TX * TY;
  static constexpr int W0 = TX + 2 * R, H0 = TY + 2 * R;
  static constexpr int W1 = TX + 2 * (R - 1), H1 = TY + 2 * (R - 1);
  static constexpr int N0 = W0 * H0, N1 = W1 * H1, N3 = TX * TY;
  static constexpr int NMID = 2 * (R - 1);  // planes k+1 .. k+R-1, then k-1 .. k-(R-1)
  static constexpr int TOTAL = N0 + NMID * N1 + 2 * N3;
  static constexpr int SLOTS = (TOTAL + NT - 1) / NT;
  __host__ __device__ static constexpr int seg(int dz) { return dz > 0 ? dz - 1 : R - 2 - dz; }
};

template <int TX, int TY, int R>
struct HAcc {
  using S = HShape<TX, TY, R>;
  const double* b0;  // plane k at (tx - R, ty - R)
  const double* b1;  // first middle plane at (tx - R + 1, ty - R + 1)
  const double* b3;  // plane k+R at (tx, ty); k-R follows at N3
  __device__ __forceinline__ double operator()(int dx, int dy, int dz) const {
    if (dz == 0) return b0[(dy + R) * S::W0 + dx + R];
    if (dz == R) return b3[0];
    if (dz == -R) return b3[S::N3];
    return b1[S::seg(dz) * S::N1 + (dy + R - 1) * S::W1 + dx + R - 1];
  }
  // +-(dx,dy,dz) along one axis (lopsided stencils)
  __device__ __forceinline__ double sel(bool up, int dx, int dy, int dz) const {
    if (dz == 0) {
      const int c = R * S::W0 + R, o = dy * S::W0 + dx;
      return b0[up ? c + o : c - o];
    }
    if (dz == R || dz == -R) return b3[(up == (dz > 0)) ? 0 : S::N3];
    const int c = (R - 1) * S::W1 + R - 1;
    return b1[(up ? S::seg(dz) : S::seg(-dz)) * S::N1 + c];
  }
};

template <int TX, int TY, int R>
struct HSrc {
  using S = HShape<TX, TY, R>;
  double* lds0;
  double* lds1;
  const int* otab;   // element offset (variable 0) of every staged point
  const double* Yt;  // yin + off0
  const double* Yc;  // centre value of variable 0 at the thread's (clamped) point
  long long sv;
  int b0o, b1o, b3o;
  int seq;

  // fills the offset table (all threads) and synchronises
  __device__ __forceinline__ void init(const Geo& G, const double* yin, double* buf0,
                                       double* buf1, int* tab, int x0, int y0, int k, int tx,
                                       int ty) {
    lds0 = buf0;
    lds1 = buf1;
    otab = tab;
    Yt = yin + G.off0;
    sv = G.sv;
    for (int t = ty * TX + tx; t < S::TOTAL; t += S::NT) {
      int px, py, dz;
      if (t < S::N0) {
        dz = 0;
        py = t / S::W0 - R;
        px = t % S::W0 - R;
      } else if (t < S::N0 + S::NMID * S::N1) {
        const int r = t - S::N0, sgm = r / S::N1, q = r % S::N1;
        dz = sgm < R - 1 ? sgm + 1 : -(sgm - (R - 1) + 1);
        py = q / S::W1 - (R - 1);
        px = q % S::W1 - (R - 1);
      } else {
        const int r = t - S::N0 - S::NMID * S::N1, sgm = r / S::N3, q = r % S::N3;
        dz = sgm == 0 ? R : -R;
        py = q / TX;
        px = q % TX;
      }
      int gx = x0 + px, gy = y0 + py;
      gx = gx < -G.g ? -G.g : (gx > G.n[0] + G.g - 1 ? G.n[0] + G.g - 1 : gx);
      gy = gy < -G.g ? -G.g : (gy > G.n[1] + G.g - 1 ? G.n[1] + G.g - 1 : gy);
      tab[t] = gx + gy * G.sy + (k + dz) * G.sz;
    }
    b0o = ty * S::W0 + tx;
    b1o = S::N0 + ty * S::W1 + tx;
    b3o = S::N0 + S::NMID * S::N1 + ty * TX + tx;
    const int ci = x0 + tx < G.n[0] ? x0 + tx : G.n[0] - 1;
    const int cj = y0 + ty < G.n[1] ? y0 + ty : G.n[1] - 1;
    Yc = Yt + ci + (long long)cj * G.sy + (long long)k * G.sz;
    seq = 0;
    __syncthreads();
  }

  __device__ __forceinline__ double center(int v) const { return Yc[v * sv]; }

  __device__ __forceinline__ HAcc<TX, TY, R> acquire(int v) {
    double* buf = (seq & 1) ? lds1 : lds0;
    const double* base = Yt + (long long)v * sv;
    const int tid = (int)threadIdx.x;
    double r[S::SLOTS];
#pragma unroll
    for (int m = 0; m < S::SLOTS; ++m) {
      const int t = tid + m * S::NT;
      r[m] = (m < S::SLOTS - 1 || t < S::TOTAL) ? base[otab[t]] : 0.0;
    }
#pragma unroll
    for (int m = 0; m < S::SLOTS; ++m) {
      const int t = tid + m * S::NT;
      if (m < S::SLOTS - 1 || t < S::TOTAL) buf[t] = r[m];
    }
    __syncthreads();
    ++seq;
    return HAcc<TX, TY, R>{buf + b0o, buf + b1o, buf + b3o};
  }
};

}  // namespace chemora

namespace chemora {

// ---------------------------------------------------------------------------
// Asynchronous staging (gfx950 global_load_lds_dwordx4): every lane copies
// two consecutive doubles straight from global memory into LDS, so the
// copies of the next D grid functions are in flight while the current one
// is differentiated, without holding any of them in registers.  Buffers
// are NBUF = D + 1 separate LDS arrays: the compiler then knows that a read
// of one buffer does not depend on a copy into another and inserts no wait
// for it.  The hand-off per grid function is: wait until this wave's copies
// of it have landed (vmcnt), barrier (all waves' copies landed, and every
// wave has finished reading the buffer the next copy will overwrite), issue
// the copy D grid functions ahead into that buffer.  __syncthreads() is not
// used for it: its fence waits for all outstanding copies.
//
// Pairs never straddle a row (every row length is even) and may read one
// column past the ghost zone, which every row's padding provides.

typedef __attribute__((address_space(3))) void lds_void_t;
typedef const __attribute__((address_space(1))) void gbl_void_t;

// s_waitcnt vmcnt(n) lgkmcnt(0), expcnt untouched (gfx9 encoding)
template <int N>
__device__ __forceinline__ void wait_vm_lgkm0() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (0 << 8) | (((N >> 4) & 3) << 14));
}

template <int TX, int TY, int NBUF, typename ORDER = RhsOrder>
struct ASrc {
  using S = LdsShape<TX, TY>;
  static constexpr int PAIRS = S::TOTAL / 2;
  static constexpr int PSLOTS = (PAIRS + S::NT - 1) / S::NT;
  static constexpr int D = NBUF - 1;
  static_assert(S::TOTAL % 2 == 0 && S::W0 % 2 == 0 && S::W1 % 2 == 0 && TX % 2 == 0,
                "pairs must not straddle rows");
  double* buf[NBUF];
  const char* Yb;        // state allocation (byte address)
  const double* Yc;      // centre value of variable 0 at the thread's (clamped) point
  long long sv;          // elements between grid functions
  unsigned off[PSLOTS];  // byte offset from Yb of each pair slot (variable 0)
  int b0o, b1o, b3o;
  int seq;
  int wbase;             // 64 * wave index

  __device__ __forceinline__ void init(const Geo& G, const double* yin, double* const* shared,
                                       int x0, int y0, int k, int tx, int ty) {
#pragma unroll
    for (int b = 0; b < NBUF; ++b) buf[b] = shared[b];
    Yb = reinterpret_cast<const char*>(yin);
    sv = G.sv;
    const int tid = ty * TX + tx;
    wbase = tid & ~63;
#pragma unroll
    for (int m = 0; m < PSLOTS; ++m) {
      int p = tid + m * S::NT;
      if (p >= PAIRS) p = 0;  // masked off at issue
      const int t = 2 * p;
      int px, py, dz;
      if (t < S::N0) {
        dz = 0;
        py = t / S::W0 - 3;
        px = t % S::W0 - 3;
      } else if (t < S::N0 + 4 * S::N1) {
        const int r = t - S::N0, s = r / S::N1, q = r % S::N1;
        dz = (s == 0) ? 1 : (s == 1 ? -1 : (s == 2 ? 2 : -2));
        py = q / S::W1 - 2;
        px = q % S::W1 - 2;
      } else {
        const int r = t - S::N0 - 4 * S::N1, s = r / S::N3, q = r % S::N3;
        dz = s == 0 ? 3 : -3;
        py = q / TX;
        px = q % TX;
      }
      // pair start in [-g-1, n+g-1] keeps both doubles inside the padded row
      int gx = x0 + px, gy = y0 + py;
      gx = gx < -G.g - 1 ? -G.g - 1 : (gx > G.n[0] + G.g - 1 ? G.n[0] + G.g - 1 : gx);
      gy = gy < -G.g ? -G.g : (gy > G.n[1] + G.g - 1 ? G.n[1] + G.g - 1 : gy);
      off[m] = (unsigned)(8 * (G.off0 + gx + (long long)gy * G.sy + (long long)(k + dz) * G.sz));
    }
    b0o = ty * S::W0 + tx;
    b1o = S::N0 + ty * S::W1 + tx;
    b3o = S::N0 + 4 * S::N1 + ty * TX + tx;
    const int ci = x0 + tx < G.n[0] ? x0 + tx : G.n[0] - 1;
    const int cj = y0 + ty < G.n[1] ? y0 + ty : G.n[1] - 1;
    Yc = yin + G.off0 + ci + (long long)cj * G.sy + (long long)k * G.sz;
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

  // copies issued after those of grid function s, counted per wave (full
  // instructions only: waiting for fewer younger copies is always safe)
  template <int YOUNGER>
  __device__ __forceinline__ void wait_and_sync() {
    wait_vm_lgkm0<YOUNGER * (PSLOTS - 1)>();
    fence_memory();
    __builtin_amdgcn_s_barrier();
    fence_memory();
  }

  __device__ __forceinline__ LAcc<TX, TY> acquire(int /*v*/) {
    if (seq == 0) {
      // prologue: issued after the point's centre loads (kept older by the
      // fence), so that waiting for a centre value never drains the copies
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
      case 4: wait_and_sync<4>(); break;
      default: wait_and_sync<5>(); break;
    }
    if (seq + D < ORDER::N) issue(seq + D);
    double* b = buf[seq % NBUF];
    ++seq;
    return LAcc<TX, TY>{b + b0o, b + b1o, b + b3o};
  }
};

// Asynchronous staging of the 6th- and 8th-order neighbourhood (HShape):
// the same copy scheme as ASrc (each lane copies a pair of doubles straight
// into LDS; NBUF separate buffers, NBUF - 1 grid functions in flight; the
// hand-off is a vmcnt wait plus a barrier), with HShape's plane layout and
// accessor.  Pairs never straddle a row: every row length is even.
template <int TX, int TY, int R, int NBUF>
struct AHSrc {
  using S = HShape<TX, TY, R>;
  static constexpr int PAIRS = S::TOTAL / 2;
  static constexpr int PSLOTS = (PAIRS + S::NT - 1) / S::NT;
  static constexpr int D = NBUF - 1;
  static_assert(S::TOTAL % 2 == 0 && S::W0 % 2 == 0 && S::W1 % 2 == 0 && TX % 2 == 0 &&
                    S::N0 % 2 == 0 && S::N1 % 2 == 0,
                "pairs must not straddle rows");
  double* buf[NBUF];
  const char* Yb;        // state allocation (byte address)
  const double* Yc;      // centre value of variable 0 at the thread's (clamped) point
  long long sv;          // elements between grid functions
  unsigned off[PSLOTS];  // byte offset from Yb of each pair slot (variable 0)
  int b0o, b1o, b3o;
  int seq;
  int wbase;             // 64 * wave index

  __device__ __forceinline__ void init(const Geo& G, const double* yin, double* const* shared,
                                       int x0, int y0, int k, int tx, int ty) {
#pragma unroll
    for (int b = 0; b < NBUF; ++b) buf[b] = shared[b];
    Yb = reinterpret_cast<const char*>(yin);
    sv = G.sv;
    const int tid = ty * TX + tx;
    wbase = tid & ~63;
#pragma unroll
    for (int m = 0; m < PSLOTS; ++m) {
      int p = tid + m * S::NT;
      if (p >= PAIRS) p = 0;  // masked off at issue
      const int t = 2 * p;
      int px, py, dz;
      if (t < S::N0) {
        dz = 0;
        py = t / S::W0 - R;
        px = t % S::W0 - R;
      } else if (t < S::N0 + S::NMID * S::N1) {
        const int r = t - S::N0, sgm = r / S::N1, q = r % S::N1;
        dz = sgm < R - 1 ? sgm + 1 : -(sgm - (R - 1) + 1);
        py = q / S::W1 - (R - 1);
        px = q % S::W1 - (R - 1);
      } else {
        const int r = t - S::N0 - S::NMID * S::N1, sgm = r / S::N3, q = r % S::N3;
        dz = sgm == 0 ? R : -R;
        py = q / TX;
        px = q % TX;
      }
      // pair start in [-g-1, n+g-1] keeps both doubles inside the padded row
      int gx = x0 + px, gy = y0 + py;
      gx = gx < -G.g - 1 ? -G.g - 1 : (gx > G.n[0] + G.g - 1 ? G.n[0] + G.g - 1 : gx);
      gy = gy < -G.g ? -G.g : (gy > G.n[1] + G.g - 1 ? G.n[1] + G.g - 1 : gy);
      off[m] = (unsigned)(8 * (G.off0 + gx + (long long)gy * G.sy + (long long)(k + dz) * G.sz));
    }
    b0o = ty * S::W0 + tx;
    b1o = S::N0 + ty * S::W1 + tx;
    b3o = S::N0 + S::NMID * S::N1 + ty * TX + tx;
    const int ci = x0 + tx < G.n[0] ? x0 + tx : G.n[0] - 1;
    const int cj = y0 + ty < G.n[1] ? y0 + ty : G.n[1] - 1;
    Yc = yin + G.off0 + ci + (long long)cj * G.sy + (long long)k * G.sz;
    seq = 0;
  }

  // start copying grid function kRhsOrder[s] into buffer s % NBUF
  __device__ __forceinline__ void issue(int s) {
    const char* base = Yb + (long long)RhsOrder::at(s) * sv * 8;
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

  template <int YOUNGER>
  __device__ __forceinline__ void wait_and_sync() {
    wait_vm_lgkm0<YOUNGER * (PSLOTS - 1)>();
    fence_memory();
    __builtin_amdgcn_s_barrier();
    fence_memory();
  }

  __device__ __forceinline__ HAcc<TX, TY, R> acquire(int /*v*/) {
    if (seq == 0) {
      fence_memory();
#pragma unroll
      for (int s = 0; s < D; ++s) issue(s);
    }
    const int last = seq + D - 1 < RhsOrder::N - 1 ? seq + D - 1 : RhsOrder::N - 1;
    switch (last - seq) {  // folds to one case once seq is known
      case 0: wait_and_sync<0>(); break;
      case 1: wait_and_sync<1>(); break;
      case 2: wait_and_sync<2>(); break;
      case 3: wait_and_sync<3>(); break;
      case 4: wait_and_sync<4>(); break;
      default: wait_and_sync<5>(); break;
    }
    if (seq + D < RhsOrder::N) issue(seq + D);
    double* b = buf[seq % NBUF];
    ++seq;
    return HAcc<TX, TY, R>{b + b0o, b + b1o, b + b3o};
  }
};

}  // namespace chemora
