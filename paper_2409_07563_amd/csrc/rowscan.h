// DPP row operations (16-lane rows) shared by the time-parallel kernels:
// prefix sums over the lanes of one row.  Lanes whose source lies outside the
// row read 0 (bound_ctrl), which is the identity of the sums.
#pragma once

#include "common.h"

namespace mppi {

template <int CTRL>
__device__ __forceinline__ float row_dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ int row_dpp_int(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;

// inclusive prefix sum over the row (Hillis-Steele)
__device__ __forceinline__ float row_scan(float v) {
  v += row_dpp<kRowShr1>(v);
  v += row_dpp<kRowShr2>(v);
  v += row_dpp<kRowShr4>(v);
  v += row_dpp<kRowShr8>(v);
  return v;
}
__device__ __forceinline__ int row_scan_int(int v) {
  v += row_dpp_int<kRowShr1>(v);
  v += row_dpp_int<kRowShr2>(v);
  v += row_dpp_int<kRowShr4>(v);
  v += row_dpp_int<kRowShr8>(v);
  return v;
}
// exclusive prefix sum over the row: the inclusive sum of the lane before
__device__ __forceinline__ float row_exclusive(float v) { return row_dpp<kRowShr1>(row_scan(v)); }

}  // namespace mppi
