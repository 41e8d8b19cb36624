// Cross-lane helpers for 64-wide wavefronts (device code only).
#pragma once

#include <hip/hip_runtime.h>

namespace strom {

// Value of a double in lane k (k uniform across the wave): two v_readlane, no LDS round trip.
__device__ __forceinline__ double readlane_d(double v, int k) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
  return __hiloint2double(hi, lo);
}

// One DPP move of a double (both halves) within rows of 16 lanes.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over each row of 16 lanes, left in every lane of the row: exchanges with lane ^ 1 and
// lane ^ 2 (quad permutes), then the half-row and row mirrors.  Both partners of every
// exchange add the same two values, so all 16 lanes hold the identical total.  Must run
// with the whole wave active.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return v;
}

}  // namespace strom
