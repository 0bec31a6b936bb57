// devutil.hpp -- device helpers shared by the LU panel kernels: the pivot
// search reductions.
#pragma once

#include <climits>

#include "common.hpp"

namespace frob {

// Keys are the bit patterns of FP32 values: for the values used here (>= 0,
// or negative for "no candidate") signed-integer order agrees with numeric
// order wherever it matters (any value >= 0 beats any negative one), and an
// integer max fuses with its DPP operand into one instruction.
template <int CTRL, int RM>
__device__ __forceinline__ int upd_dpp_i32(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, RM, 0xF, false);
}
// maximum over each row of 16 lanes, left in the row's last lane
__device__ __forceinline__ int row_max_key(int v) {
  v = max(v, upd_dpp_i32<0x111, 0xF>(v, v));  // row_shr:1
  v = max(v, upd_dpp_i32<0x112, 0xF>(v, v));  // row_shr:2
  v = max(v, upd_dpp_i32<0x114, 0xF>(v, v));  // row_shr:4
  v = max(v, upd_dpp_i32<0x118, 0xF>(v, v));  // row_shr:8
  return v;
}
// maximum over the wave, the same in every lane
__device__ __forceinline__ int wave_max_key(int v) {
  v = row_max_key(v);
  v = max(v, upd_dpp_i32<0x142, 0xA>(v, v));  // row_bcast:15 into rows 1, 3
  v = max(v, upd_dpp_i32<0x143, 0xC>(v, v));  // row_bcast:31 into rows 2, 3
  return __builtin_amdgcn_readlane(v, 63);
}
// Exact argmax over the lanes in `cand` of (val desc, key asc); returns the
// winning lane.  Rare path (several lanes share the FP32 maximum).
__device__ __forceinline__ int exact_argmax(unsigned long long cand, double val, int key) {
  int wl = -1;
  double bv = -1.0;
  int bk = INT_MAX;
  while (cand) {
    const int l = __ffsll((long long)cand) - 1;
    cand &= cand - 1;
    const double lv = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(val), l),
                                       __builtin_amdgcn_readlane(__double2loint(val), l));
    const int lk = __builtin_amdgcn_readlane(key, l);
    if (lv > bv || (lv == bv && lk < bk)) { bv = lv; bk = lk; wl = l; }
  }
  return wl;
}


}  // namespace frob
