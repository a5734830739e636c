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

#define CPR_LAUNCH_CHECK() (void)hipGetLastError()

}  // namespace cpr
