// Helpers shared by the HIP kernel files (device side only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"

namespace cpr {

// The hardware hands workgroup b of a launch to XCD (b mod 8).  Renumbering the
// workgroups so that each XCD receives one contiguous range of the logical
// index space keeps neighbouring rows (and the vector entries they gather) in
// the same XCD's L2 instead of spreading every cache line over eight L2s.
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int q = G >> 3, r = G & 7, x = b & 7, k = b >> 3;
  return x * q + (x < r ? x : r) + k;
}

inline int div_up(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

// DPP controls (GFX9 encoding): shift right by one lane within each row of 16
// lanes (lane 0 of a row has no source), and rotate right by one lane within
// each row (lane 0 reads lane 15).
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowRor1 = 0x121;

// A lane's value moved by a DPP control; a lane without a source keeps its own.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  const int u = __float_as_int(v);
  return __int_as_float(__builtin_amdgcn_update_dpp(u, u, CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = static_cast<int>(u & 0xffffffffll), hi = static_cast<int>(u >> 32);
  const int mlo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
  const int mhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
  return __longlong_as_double((static_cast<long long>(mhi) << 32) | static_cast<unsigned int>(mlo));
}

// Ordered subtraction over one chunk of a 16-lane group (one DPP row).  On
// entry lane 15 holds the running value s; on return lane 15 holds
// (((s - p_0) - p_1) ... - p_15), each step rounded as a sequential loop
// rounds it.  Step 0 hands lane 15's value to lane 0 (rotate), which
// subtracts p_0; step k hands lane k-1's value to lane k.  After step k lanes
// 0..k hold their final prefixes (recomputing an earlier lane reproduces its
// value, lane 0 subtracts +0, which leaves every value unchanged), so lane 15
// is final after step 15.  Other lanes end with unspecified values.
template <typename T>
__device__ __forceinline__ T row_chain_sub(T s, T p, int lane) {
  const T pk = lane == 0 ? (T)0 : p;
  s = dpp_move<kDppRowRor1>(s) - p;
#pragma unroll
  for (int k = 1; k < 16; ++k) s = dpp_move<kDppRowShr1>(s) - pk;
  return s;
}

#define CPR_LAUNCH_CHECK() (void)hipGetLastError()

}  // namespace cpr
