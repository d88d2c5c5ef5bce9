// Cross-lane sums and exchanges within a wavefront of 64 lanes, by DPP row operations,
// lane reads and gfx950's lane-swap instructions (a few cycles each) rather than
// LDS-routed shuffles (an LDS round trip each).  Sums are added in a fixed order, so
// results do not depend on timing.
#pragma once
#include <hip/hip_runtime.h>

namespace lg {

// The DPP forms read lanes of the same row of 16; every lane they read must be active.
template <int Ctrl>
__device__ inline float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), Ctrl, 0xF, 0xF, true));
}
// sum over each half row of 8 lanes, in every lane of it
__device__ inline float sum8(float v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]: pairs
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]: quads
  v += dpp_mov<0x141>(v);  // row_half_mirror: the other quad of each 8
  return v;
}
// sum over each row of 16 lanes, in every lane of the row
__device__ inline float row16_sum(float v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]: pairs
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]: quads
  v += dpp_mov<0x141>(v);  // row_half_mirror: the other quad of each 8
  v += dpp_mov<0x140>(v);  // row_mirror: the other 8 of the row
  return v;
}
__device__ inline float lane_value(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
// sum over the 64 lanes (all active), the same value in every lane
__device__ inline float wave_sum(float v) {
  v = row16_sum(v);
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}
// minimum / maximum over the 64 lanes (all active), the same value in every lane
template <int Ctrl>
__device__ inline int dpp_mov_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, Ctrl, 0xF, 0xF, true);
}
__device__ inline int wave_min_i(int v) {
  v = min(v, dpp_mov_i<0xB1>(v));
  v = min(v, dpp_mov_i<0x4E>(v));
  v = min(v, dpp_mov_i<0x141>(v));
  v = min(v, dpp_mov_i<0x140>(v));
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
__device__ inline int wave_max_i(int v) {
  v = max(v, dpp_mov_i<0xB1>(v));
  v = max(v, dpp_mov_i<0x4E>(v));
  v = max(v, dpp_mov_i<0x141>(v));
  v = max(v, dpp_mov_i<0x140>(v));
  return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
// inclusive prefix sum over the 64 lanes (all active): within each row of 16 by shifts of
// 1, 2, 4 and 8 lanes, then row 0's total into row 1 and row 2's into row 3 (row_bcast:15),
// then row 1's total into rows 2 and 3 (row_bcast:31)
__device__ inline int wave_incl_scan_i(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15, rows 1 and 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31, rows 2 and 3
  return v;
}
// v of the same lane in the other half (rows 0-1 <-> 2-3) and in the other row of the
// half (0 <-> 1, 2 <-> 3), added to u: gfx950's lane-swap instructions
__device__ inline float swap32_add(float keep_lo, float keep_hi) {
  // lanes 0..31 keep keep_lo and receive keep_lo of lane + 32; lanes 32..63 keep keep_hi
  // and receive keep_hi of lane - 32
  const auto p = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(int, keep_lo), __builtin_bit_cast(int, keep_hi),
                                                  false, false);
  return __builtin_bit_cast(float, (int)p[0]) + __builtin_bit_cast(float, (int)p[1]);
}
__device__ inline float swap16_add(float keep_even, float keep_odd) {
  // even rows keep keep_even and receive keep_even of the odd row beside them; odd rows
  // keep keep_odd and receive keep_odd of the even row
  const auto p = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(int, keep_even), __builtin_bit_cast(int, keep_odd),
                                                  false, false);
  return __builtin_bit_cast(float, (int)p[0]) + __builtin_bit_cast(float, (int)p[1]);
}

}  // namespace lg
