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
// quad_perm controls: lane i of each quad reads the lane given by bits
// [2i+1:2i].  [3,0,1,2] rotates right by one; [0,0,1,2] shifts right by one
// with lane 0 reading itself.
constexpr int kDppQuadRor1 = 3 | (0 << 2) | (1 << 4) | (2 << 6);
constexpr int kDppQuadShr1 = 0 | (0 << 2) | (1 << 4) | (2 << 6);

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

// The same ordered subtraction over one chunk of a 4-lane group (one quad):
// lane 3 holds the running value on entry and (((s - p_0) - p_1) - p_2) - p_3
// on return.
template <typename T>
__device__ __forceinline__ T quad_chain_sub(T s, T p, int lane) {
  const T pk = lane == 0 ? (T)0 : p;
  s = dpp_move<kDppQuadRor1>(s) - p;
  s = dpp_move<kDppQuadShr1>(s) - pk;
  s = dpp_move<kDppQuadShr1>(s) - pk;
  s = dpp_move<kDppQuadShr1>(s) - pk;
  return s;
}

// Loads through a pointer known to address device memory (global address
// space), for pointers the compiler cannot classify itself (read from a
// descriptor in memory): keeps them off the generic path, whose loads are
// counted with LDS operations and so serialise with them.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> gmem(const T* p) {
  return (gptr<T>)p;
}

// Four consecutive entries starting at a multiple of four (16-byte aligned
// columns, 16- or 32-byte aligned values) as one or two vector loads.
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void load4_cols(const int32_t* col, int32_t e, int32_t c[4]) {
  const i32x4 v = *reinterpret_cast<const i32x4*>(col + e);
  c[0] = v.x; c[1] = v.y; c[2] = v.z; c[3] = v.w;
}
__device__ __forceinline__ void load4_cols(gptr<int32_t> col, int32_t e, int32_t c[4]) {
  const i32x4 v = *(gptr<i32x4>)(col + e);
  c[0] = v.x; c[1] = v.y; c[2] = v.z; c[3] = v.w;
}
__device__ __forceinline__ void load4_vals(const float* val, int32_t e, float a[4]) {
  const f32x4 v = *reinterpret_cast<const f32x4*>(val + e);
  a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
}
__device__ __forceinline__ void load4_vals(gptr<float> val, int32_t e, float a[4]) {
  const f32x4 v = *(gptr<f32x4>)(val + e);
  a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
}
__device__ __forceinline__ void load4_vals(const double* val, int32_t e, double a[4]) {
  const f64x2 v0 = *reinterpret_cast<const f64x2*>(val + e);
  const f64x2 v1 = *reinterpret_cast<const f64x2*>(val + e + 2);
  a[0] = v0.x; a[1] = v0.y; a[2] = v1.x; a[3] = v1.y;
}
__device__ __forceinline__ void load4_vals(gptr<double> val, int32_t e, double a[4]) {
  const f64x2 v0 = *(gptr<f64x2>)(val + e);
  const f64x2 v1 = *(gptr<f64x2>)(val + e + 2);
  a[0] = v0.x; a[1] = v0.y; a[2] = v1.x; a[3] = v1.y;
}

// Row sum of a quad-vector CSR matrix taken by the four lanes of a quad.
// Rows are padded to a multiple of four stored entries (padding: column -1,
// value 0).  Chunk u of a pass covers entries [p + 16u, p + 16u + 16): lane k
// holds the four entries p + 16u + 4k .. + 3 (one vector load each for
// columns and values), so a quad reads whole 64-byte segments.  prod(c, a)
// gives the product of one entry (0 where the entry does not contribute,
// which leaves every running value unchanged).  The products are subtracted
// from s in stored order: lane 0 continues from lane 3's running value
// (rotate) and subtracts its four products; then, three times, each lane
// continues from its left neighbour and subtracts its four (lane 0 subtracts
// zeros, so it keeps its value; a lane recomputing an already final value
// reproduces it), so lane 3 holds the chunk's result, rounded exactly as a
// sequential loop over the row rounds it.  CH chunks are requested at once.
// Entries of a pass beyond the row's end get column `fill` and value 0.
template <typename T, int CH, typename ColP, typename ValP, typename Prod>
__device__ __forceinline__ T quad_row_sub(T s, int32_t p0, int32_t p1, ColP col, ValP val, int lane,
                                          Prod&& prod, int32_t fill = -1) {
  for (int32_t p = p0; p < p1; p += 16 * CH) {
    const int nch = min(CH, (p1 - p + 15) / 16);  // uniform across the quad
    int32_t c[CH][4];
    T a[CH][4];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int32_t e = p + 16 * u + 4 * lane;
      if (e < p1) {
        load4_cols(col, e, c[u]);
        load4_vals(val, e, a[u]);
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          c[u][k] = fill;
          a[u][k] = (T)0;
        }
      }
    }
    T pr[CH][4];
#pragma unroll
    for (int u = 0; u < CH; ++u)
#pragma unroll
      for (int k = 0; k < 4; ++k) pr[u][k] = prod(c[u][k], a[u][k]);
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      if (u < nch) {
        s = dpp_move<kDppQuadRor1>(s);
#pragma unroll
        for (int k = 0; k < 4; ++k) s = s - pr[u][k];
#pragma unroll
        for (int step = 1; step < 4; ++step) {
          s = dpp_move<kDppQuadShr1>(s);
#pragma unroll
          for (int k = 0; k < 4; ++k) s = s - (lane == 0 ? (T)0 : pr[u][k]);
        }
      }
    }
  }
  return s;
}

// One pass of the ordered row sum taken by the 16 lanes of one DPP row over
// the quad-vector CSR layout: chunk u covers entries [p + 64u, p + 64u + 64),
// lane k holds the four entries p + 64u + 4k .. + 3 (one vector load each for
// columns and values).  Lane 0 continues from lane 15's running value
// (rotate) and subtracts its four products; then, fifteen times, each lane
// continues from its left neighbour and subtracts its four (lane 0 subtracts
// zeros), so lane 15 holds the chunk's result, rounded exactly as a
// sequential loop over the row rounds it.  The CH chunks' loads and gathers
// are all requested before the first subtraction; chunks past the row's end
// (u >= nch) read column -1 and value 0 and are not subtracted.
template <typename T, int CH, typename ColP, typename ValP, typename Prod>
__device__ __forceinline__ T row16v4_pass(T s, int32_t p, int32_t p1, ColP col, ValP val, int lane, Prod&& prod) {
  const int nch = min(CH, (p1 - p + 63) / 64);  // uniform across the row group
  int32_t c[CH][4];
  T a[CH][4];
#pragma unroll
  for (int u = 0; u < CH; ++u) {
    const int32_t e = p + 64 * u + 4 * lane;
    if (e < p1) {
      load4_cols(col, e, c[u]);
      load4_vals(val, e, a[u]);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        c[u][k] = -1;
        a[u][k] = (T)0;
      }
    }
  }
  T pr[CH][4];
#pragma unroll
  for (int u = 0; u < CH; ++u)
#pragma unroll
    for (int k = 0; k < 4; ++k) pr[u][k] = prod(c[u][k], a[u][k]);
#pragma unroll
  for (int u = 0; u < CH; ++u) {
    if (u < nch) {
      T m[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) m[k] = lane == 0 ? (T)0 : pr[u][k];
      s = dpp_move<kDppRowRor1>(s);
#pragma unroll
      for (int k = 0; k < 4; ++k) s = s - pr[u][k];
#pragma unroll
      for (int step = 1; step < 16; ++step) {
        s = dpp_move<kDppRowShr1>(s);
#pragma unroll
        for (int k = 0; k < 4; ++k) s = s - m[k];
      }
    }
  }
  return s;
}

// The ordered row sum over passes of up to CH chunks (64 CH entries).  A
// pass requests only as many chunks as the longest row of the wavefront
// still needs (1, 2, 4, 6 or 8, a wavefront-uniform choice): a colour kernel
// lasts as long as its longest row, so CH is sized for the longest rows, and
// the shorter rows of other wavefronts do not pay for those rows' gathers.
template <typename T, int CH, typename ColP, typename ValP, typename Prod>
__device__ __forceinline__ T row16v4_sub(T s, int32_t p0, int32_t p1, ColP col, ValP val, int lane, Prod&& prod) {
  for (int32_t p = p0; p < p1; p += 64 * CH) {
    const int need = min(CH, (p1 - p + 63) / 64);
    int nw = 1;  // chunks the active lanes of the wavefront need
#pragma unroll
    for (int k = 1; k < CH; ++k)
      if (__builtin_amdgcn_ballot_w64(need > k) != 0) nw = k + 1;
    if (CH <= 1 || nw <= 1)
      s = row16v4_pass<T, 1>(s, p, p1, col, val, lane, prod);
    else if (CH <= 2 || nw <= 2)
      s = row16v4_pass<T, (CH < 2 ? CH : 2)>(s, p, p1, col, val, lane, prod);
    else if (CH <= 4 || nw <= 4)
      s = row16v4_pass<T, (CH < 4 ? CH : 4)>(s, p, p1, col, val, lane, prod);
    else if (CH <= 6 || nw <= 6)
      s = row16v4_pass<T, (CH < 6 ? CH : 6)>(s, p, p1, col, val, lane, prod);
    else
      s = row16v4_pass<T, CH>(s, p, p1, col, val, lane, prod);
  }
  return s;
}

// Inverse of a 3x3 block (row-major src, FP64) by LU with partial pivoting,
// then column c of the inverse from (L U) x = P e_c.  Returns false when a
// pivot is not above 1e-300 times the block's largest entry (or the block is
// zero); out is then unspecified.
__device__ inline bool inverse3x3(const double* src, double out[9]) {
  double a[3][3];
  double amax = 0.0;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      a[r][c] = src[3 * r + c];
      amax = fmax(amax, fabs(a[r][c]));
    }
  int perm[3] = {0, 1, 2};
  bool bad = !(amax > 0.0);
  for (int k = 0; k < 3; ++k) {
    int p = k;
    double best = fabs(a[k][k]);
    for (int r = k + 1; r < 3; ++r)
      if (fabs(a[r][k]) > best) {
        best = fabs(a[r][k]);
        p = r;
      }
    if (!(best > 1e-300 * amax)) bad = true;
    if (p != k) {
      for (int c = 0; c < 3; ++c) {
        const double tmp = a[k][c];
        a[k][c] = a[p][c];
        a[p][c] = tmp;
      }
      const int tp = perm[k];
      perm[k] = perm[p];
      perm[p] = tp;
    }
    for (int r = k + 1; r < 3; ++r) {
      a[r][k] = a[r][k] / a[k][k];
      for (int c = k + 1; c < 3; ++c) a[r][c] = a[r][c] - a[r][k] * a[k][c];
    }
  }
  if (bad) return false;
  for (int c = 0; c < 3; ++c) {
    double y[3];
    for (int r = 0; r < 3; ++r) {
      double s = (perm[r] == c) ? 1.0 : 0.0;
      for (int k = 0; k < r; ++k) s = s - a[r][k] * y[k];
      y[r] = s;
    }
    for (int r = 2; r >= 0; --r) {
      double s = y[r];
      for (int k = r + 1; k < 3; ++k) s = s - a[r][k] * y[k];
      y[r] = s / a[r][r];
    }
    for (int r = 0; r < 3; ++r) out[3 * r + c] = y[r];
  }
  return true;
}

#define CPR_LAUNCH_CHECK() (void)hipGetLastError()

}  // namespace cpr
