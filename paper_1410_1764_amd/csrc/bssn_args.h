// bssn_args.h -- launch arguments of the single-block BSSN kernels and the
// tile each workgroup takes (shared by the fused and the split kernels).
#pragma once

#include "bssn_lds.h"

namespace chemora {

struct BssnArgs {
  Geo G;
  BssnPar P;
  Weights W;
  StageIO io;
  int ltx, lty, zc;
  int tiles[3];
  int cols[2];  // column split of the staged kernels (column_tile); 0: xcd_tile order
  int images;
};

// tile of workgroup b in the single-plane (staged) kernels
__device__ __forceinline__ bool plane_tile(const BssnArgs& a, int b, int& bx, int& by, int& bz) {
  if (a.cols[0] > 0) return column_tile(b, a.tiles, a.cols[0], a.cols[1], bx, by, bz);
  const int t = xcd_tile(b, a.tiles[0] * a.tiles[1] * a.tiles[2]);
  bx = t % a.tiles[0];
  by = (t / a.tiles[0]) % a.tiles[1];
  bz = t / (a.tiles[0] * a.tiles[1]);
  return true;
}

// Launches the two-kernel (split) form of a substage when it applies to
// the arguments (fd_order 4, 32 x 8 staged tiles); returns false otherwise
// without launching anything.
bool launch_bssn_split(int stage, int precision, const BssnArgs& a, dim3 grid, hipStream_t s,
                       hipError_t* err);

}  // namespace chemora
