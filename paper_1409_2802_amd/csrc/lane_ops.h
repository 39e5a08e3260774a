// Cross-lane helpers for 64-wide wavefronts: DPP all-reductions within rows
// of 16 lanes and uniform reads of one lane's double.
#pragma once

#include <hip/hip_runtime.h>

namespace ffc {

// DPP move of a double (two 32-bit halves) with row control CTRL.
template <int CTRL>
__device__ inline double dpp_mov(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// All-reduce of a double within each row of 16 lanes by DPP moves (quad
// swaps, half-row mirror, row mirror). Every step combines two values in the
// same order on both partners, so all 16 lanes end with bitwise-identical
// results.
__device__ inline double row16_sum(double x) {
  x += dpp_mov<0xB1>(x);    // quad_perm [1,0,3,2]
  x += dpp_mov<0x4E>(x);    // quad_perm [2,3,0,1]
  x += dpp_mov<0x141>(x);   // row_half_mirror
  x += dpp_mov<0x140>(x);   // row_mirror
  return x;
}

__device__ inline double row16_max(double x) {
  x = fmax(x, dpp_mov<0xB1>(x));
  x = fmax(x, dpp_mov<0x4E>(x));
  x = fmax(x, dpp_mov<0x141>(x));
  x = fmax(x, dpp_mov<0x140>(x));
  return x;
}

// Lane l's value, wavefront-uniform (l must be uniform).
__device__ inline double readlane_d(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                          __builtin_amdgcn_readlane(__double2loint(x), l));
}

// Sum over the whole wavefront in a fixed order (rows of 16 by DPP, then the
// four row sums in lane order), the same value in every lane.
__device__ inline double wave_sum_dpp(double x) {
  x = row16_sum(x);
  return ((readlane_d(x, 0) + readlane_d(x, 16)) + readlane_d(x, 32)) + readlane_d(x, 48);
}

}  // namespace ffc
