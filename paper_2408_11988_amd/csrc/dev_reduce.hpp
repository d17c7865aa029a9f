// FP64 sums over aligned lane groups of a wavefront, with every lane of a
// group receiving its group's sum. Inside a row of 16 lanes the partners come
// through DPP, a VALU operand modifier that does not use the LDS crossbar:
// quad permutations pair lanes 1 and 2 apart, then the half-row mirror
// (lane l with 7 - l inside 8) and the row mirror (l with 15 - l inside 16)
// pair the quads and the half rows. Only the 32- and 64-lane steps use
// cross-lane shuffles. The order of the additions is fixed.
#pragma once

#include "common.hpp"

namespace tss {

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

template <int GL>
__device__ __forceinline__ double group_sum_f64(double x) {
  static_assert(GL >= 1 && GL <= 64 && (GL & (GL - 1)) == 0, "group width must be a power of two <= 64");
  if constexpr (GL >= 2) x += dpp_f64<0xB1>(x);    // quad_perm [1,0,3,2]
  if constexpr (GL >= 4) x += dpp_f64<0x4E>(x);    // quad_perm [2,3,0,1]
  if constexpr (GL >= 8) x += dpp_f64<0x141>(x);   // row_half_mirror
  if constexpr (GL >= 16) x += dpp_f64<0x140>(x);  // row_mirror
  if constexpr (GL >= 32) x += __shfl_xor(x, 16, kWave);
  if constexpr (GL >= 64) x += __shfl_xor(x, 32, kWave);
  return x;
}

}  // namespace tss
