// Wavefront-level helpers (64 lanes) for the per-node kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace hm {

// v of lane src, for every lane
__device__ __forceinline__ double readlane_d(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// (v, i) <- the better of (v, i) and (ov, oi): the larger value, ties to the smaller
// index.  A total order on (value, index) pairs without NaN, so any reduction tree
// gives the same winner.
__device__ __forceinline__ void take_better(double& v, int& i, double ov, int oi) {
  const bool t = ov > v || (ov == v && oi < i);
  v = t ? ov : v;
  i = t ? oi : i;
}

// one reduction round with the partner that the DPP control CTRL names (a pattern
// that stays inside a row of 16 lanes, so every lane has a valid source)
template <int CTRL>
__device__ __forceinline__ void argmax_round_dpp(double& v, int& i) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  const int oi = __builtin_amdgcn_update_dpp(0, i, CTRL, 0xF, 0xF, false);
  take_better(v, i, __longlong_as_double(((long long)hi << 32) | (unsigned)lo), oi);
}

// Index of the best (value, index) pair over the 64 lanes, returned to every lane.
// Inside each row of 16: swaps within quads (quad_perm [1,0,3,2], [2,3,0,1]), then
// the half-row mirror (lane 7 - x) joins the two quads of each half, and the row
// mirror (lane 15 - x) the two halves; the four rows' winners are then read from
// lanes 0, 16, 32, 48.  No value may be NaN.
__device__ __forceinline__ int wave_argmax(double v, int i) {
  argmax_round_dpp<0xB1>(v, i);    // quad_perm [1,0,3,2]
  argmax_round_dpp<0x4E>(v, i);    // quad_perm [2,3,0,1]
  argmax_round_dpp<0x141>(v, i);   // row_half_mirror
  argmax_round_dpp<0x140>(v, i);   // row_mirror
  double bv = readlane_d(v, 0);
  int bi = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
  for (int r = 16; r < 64; r += 16) take_better(bv, bi, readlane_d(v, r), __builtin_amdgcn_readlane(i, r));
  return bi;
}

}  // namespace hm
