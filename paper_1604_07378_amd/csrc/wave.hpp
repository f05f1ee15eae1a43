// Cross-lane sums inside a 64-lane wavefront without the LDS crossbar: DPP
// row operations (quad permutes and the 8- and 16-lane mirrors) reduce within
// a row of 16 lanes on the VALU, and v_readlane combines the rows. Every lane
// of a group receives the same value, computed in a fixed order, so the sums
// are bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>

namespace qn {

// v of the lane selected by the DPP control CTRL (full row and bank masks).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// v of lane `lane` (a constant), broadcast to the whole wave.
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7 - i within 8 lanes
constexpr int kDppMirror = 0x140;     // lane i <-> 15 - i within 16 lanes

// Sum over the aligned group of L lanes (L = 1, 2, 4, ..., 64, uniform in the
// wave) that contains this lane. Must be called by all 64 lanes.
__device__ __forceinline__ double group_sum(double v, int L) {
  if (L >= 2) v += dpp_d<kDppXor1>(v);
  if (L >= 4) v += dpp_d<kDppXor2>(v);
  if (L >= 8) v += dpp_d<kDppHalfMirror>(v);
  if (L >= 16) v += dpp_d<kDppMirror>(v);
  if (L == 32) {
    const double lo = readlane_d(v, 0) + readlane_d(v, 16);
    const double hi = readlane_d(v, 32) + readlane_d(v, 48);
    v = (threadIdx.x & 32) ? hi : lo;
  } else if (L == 64) {
    v = (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
  }
  return v;
}

// group_sum of N values together: the same steps in the same order for each
// value (so the same bits as N calls of group_sum), but step by step over all
// N, so that the N independent chains interleave instead of running one after
// another behind the tests of L.
template <int N>
__device__ __forceinline__ void group_sum_n(double (&v)[N], int L) {
  if (L >= 2) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += dpp_d<kDppXor1>(v[i]);
  }
  if (L >= 4) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += dpp_d<kDppXor2>(v[i]);
  }
  if (L >= 8) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += dpp_d<kDppHalfMirror>(v[i]);
  }
  if (L >= 16) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += dpp_d<kDppMirror>(v[i]);
  }
  if (L == 32) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const double lo = readlane_d(v[i], 0) + readlane_d(v[i], 16);
      const double hi = readlane_d(v[i], 32) + readlane_d(v[i], 48);
      v[i] = (threadIdx.x & 32) ? hi : lo;
    }
  } else if (L == 64) {
#pragma unroll
    for (int i = 0; i < N; ++i)
      v[i] = (readlane_d(v[i], 0) + readlane_d(v[i], 16)) +
             (readlane_d(v[i], 32) + readlane_d(v[i], 48));
  }
}

// Sum over the whole wave (every lane receives it).
__device__ __forceinline__ double wave_total(double v) { return group_sum(v, 64); }

}  // namespace qn
