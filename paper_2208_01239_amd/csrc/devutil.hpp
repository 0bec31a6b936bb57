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
// winning lane, the same in every lane.  Keys of candidates are distinct.
// Called with the whole wave active when several lanes share the FP32
// maximum: a butterfly of lane exchanges over (value, key, lane), so its cost
// does not grow with the number of tied lanes (a wave of exactly-zero rows
// ties on every lane).
__device__ __forceinline__ int exact_argmax(unsigned long long cand, double val, int key) {
  const int lane = __lane_id();
  const bool in = (cand >> lane) & 1ull;
  double v = in ? val : -1.0;
  int k = in ? key : INT_MAX;
  int l = in ? lane : 64;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int ok = __shfl_xor(k, off);
    const int ol = __shfl_xor(l, off);
    const bool take = (ov > v) | ((ov == v) & (ok < k));
    v = take ? ov : v;
    k = take ? ok : k;
    l = take ? ol : l;
  }
  return __builtin_amdgcn_readfirstlane(l);
}

}  // namespace frob
