// Pressure-AMG kernels: the PGS-SCM colour sweep (Algorithm "PGS-SCM"),
// residual, restriction and prolongation.
//
// Storage forms, chosen per matrix at SETUP from its size and row lengths:
//  * SELL-64, one lane per row (many short rows: the finest level, P, R).
//    Slots are fetched U at a time so the gathers of a row overlap.
//  * Quad-vector CSR (Galerkin levels of medium row length): four lanes per
//    row, rows padded to a multiple of four entries, each lane reading four
//    contiguous entries per chunk with one vector load (see quad_row_sub);
//    sixteen rows per wavefront.
//  * 16 lanes per row over the same padded CSR data, four contiguous entries
//    per lane (long rows of the Galerkin levels; see row16v4_sub).
//  * CSR with a group of 16, 32 or 64 lanes per row, one stored entry per
//    lane and chunk (selectable; the group adds the products in stored order,
//    a 16-lane group by DPP moves, wider groups one broadcast at a time).
// Every form accumulates each row exactly as a sequential loop over its
// stored entries would (products rounded, then added in order), so results
// match a sequential implementation bit for bit.  Entries that do not
// contribute are replaced by a zero product, which leaves the sum unchanged.
//
// Rows of a colour are stored in index order and each XCD takes one
// contiguous range of them (xcd_block), so the rows of a workgroup, and of an
// XCD, gather mostly the same vector entries.
#include "kernels_common.hpp"

namespace cpr {

// ------------------------------------------------------------------ helpers
// Row q of a SELL matrix: call f(col, val) for each stored entry in order,
// with the loads of U consecutive slots issued together (U is chosen per
// matrix from its slice widths, so most rows take one batch: every further
// batch costs two dependent memory round trips).
// A matrix whose slices all have the same width (width > 0) needs no slice
// pointer: the slot range is computed, which saves a dependent load.
template <typename T, int U, typename F>
__device__ __forceinline__ void sell_row(int32_t q, int32_t width, const int32_t* __restrict__ slice_ptr,
                                         const int32_t* __restrict__ col, const T* __restrict__ val, F&& f) {
  const int32_t slice = q >> 6, lane = q & 63;
  const int32_t t0 = width > 0 ? slice * width : slice_ptr[slice];
  const int32_t t1 = width > 0 ? t0 + width : slice_ptr[slice + 1];
  for (int32_t t = t0; t < t1; t += U) {
    int32_t c[U];
    T a[U];
    // columns and values are requested together: padded slots hold value 0
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = (int64_t)(t + u) * kWave + lane;
      c[u] = (t + u < t1) ? col[e] : kPadCol;
      a[u] = (t + u < t1) ? val[e] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) f(c[u], a[u]);
  }
}

// Value of lane k (compile-time) of the wavefront, read through the scalar unit.
__device__ __forceinline__ float lane_value(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ __forceinline__ double lane_value(double v, int k) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(u & 0xffffffffll), k);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(u >> 32), k);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Ordered sum over one chunk of a group: s = s (op) p_0 (op) p_1 ... in lane order.
template <typename T, int G, bool SUB>
__device__ __forceinline__ T group_ordered(T s, T p) {
#pragma unroll
  for (int k = 0; k < G; ++k) {
    const T v = (G == kWave) ? lane_value(p, k) : __shfl(p, k, G);
    s = SUB ? (s - v) : (s + v);
  }
  return s;
}

// One chunk of a group's ordered accumulation: s (op) p_0 (op) ... (op) p_{G-1}.
// Addition runs as subtraction of the negated product (a + b and a - (-b) are
// the same IEEE operation).  The result is valid in lane last_lane<G>().
template <int G>
__device__ __forceinline__ constexpr int last_lane() {
  return G == 16 ? 15 : 0;
}
template <typename T, int G, bool SUB>
__device__ __forceinline__ T group_chunk(T s, T p, int lane) {
  if constexpr (G == 16) {
    return row_chain_sub<T>(s, SUB ? p : -p, lane);
  } else {
    return group_ordered<T, G, SUB>(s, p);
  }
}

// ------------------------------------------------------------------ colour sweep
// One colour [lo, hi): x_i = (b_i - sum_{j != i} a_ij xt_j) / a_ii with xt_j =
// s_in[j] for j in [lo, hi) (the colour's values before this colour started)
// and x[j] otherwise; ZERO: x == 0 on entry, so only j < lo contribute.
// The product a_ij xt_j of one stored entry, 0 where it does not contribute
// (padding, the diagonal, and in ZERO mode every column of this colour or a
// later one).  Branch-free: an entry that does not contribute reads row q's
// own value (a valid address) and its product is replaced by 0.
template <typename T, bool ZERO>
__device__ __forceinline__ T gs_prod(int32_t q, int32_t c, T a, int32_t lo, int32_t hi, const T* __restrict__ x,
                                     const T* __restrict__ s_in) {
  const bool use = c >= 0 && c != q && (!ZERO || c < lo);
  const int32_t cc = use ? c : q;
  const T* src = (!ZERO && cc >= lo && cc < hi) ? s_in : x;
  const T xv = src[cc];
  return use ? a * xv : (T)0;
}

template <typename T, int U, bool ZERO>
__global__ __launch_bounds__(kBlock) void k_gs_sell(int32_t lo, int32_t hi, int32_t width,
                                                    const int32_t* __restrict__ slice_ptr,
                                                    const int32_t* __restrict__ col, const T* __restrict__ val,
                                                    const T* __restrict__ diag, const T* __restrict__ b,
                                                    T* __restrict__ x, const T* __restrict__ s_in,
                                                    T* __restrict__ s_out) {
  const int32_t base = lo & ~63;
  const int32_t q = base + xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (q < lo || q >= hi) return;
  T s = b[q];
  const T d = diag[q];  // requested with b, off the row's dependent chain
  sell_row<T, U>(q, width, slice_ptr, col, val,
                 [&](int32_t c, T a) { s = s - gs_prod<T, ZERO>(q, c, a, lo, hi, x, s_in); });
  const T xn = s / d;
  x[q] = xn;
  s_out[q] = xn;
}

// CH chunks of G entries of a row are requested together (chosen per matrix
// from its row lengths so that most rows take one pass).
template <typename T, int G, int CH, bool ZERO>
__global__ __launch_bounds__(kBlock) void k_gs_grp(int32_t lo, int32_t hi, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, const T* __restrict__ val,
                                                   const T* __restrict__ diag, const T* __restrict__ b,
                                                   T* __restrict__ x, const T* __restrict__ s_in,
                                                   T* __restrict__ s_out) {
  // each XCD takes one contiguous range of the colour's rows (as k_gs_q4)
  const int32_t g = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  const int32_t q = lo + g;
  if (q >= hi) return;
  T s = b[q];
  const T d = diag[q];  // requested with b, off the row's dependent chain
  const int32_t p0 = rp[q], p1 = rp[q + 1];
  for (int32_t p = p0; p < p1; p += G * CH) {
    // chunks this row still has (uniform across the group)
    const int nch = min(CH, (p1 - p + G - 1) / G);
    int32_t c[CH];
    T a[CH], prod[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int32_t e = p + u * G + lane;
      c[u] = (e < p1) ? col[e] : kPadCol;
      a[u] = (e < p1) ? val[e] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) prod[u] = gs_prod<T, ZERO>(q, c[u], a[u], lo, hi, x, s_in);
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (u < nch) s = group_chunk<T, G, true>(s, prod[u], lane);
  }
  if (lane == last_lane<G>()) {
    const T xn = s / d;
    x[q] = xn;
    s_out[q] = xn;
  }
}

template <typename T, int G, int CH>
void launch_gs_grp(const MatView<T>& A, const T* diag, int32_t lo, int32_t hi, const T* b, T* x, const T* s_in,
                   T* s_out, bool zero_start, hipStream_t s) {
  const int grid = div_up((int64_t)(hi - lo) * G, kBlock);
  if (zero_start)
    hipLaunchKernelGGL((k_gs_grp<T, G, CH, true>), dim3(grid), dim3(kBlock), 0, s, lo, hi, A.ptr, A.col, A.val, diag,
                       b, x, s_in, s_out);
  else
    hipLaunchKernelGGL((k_gs_grp<T, G, CH, false>), dim3(grid), dim3(kBlock), 0, s, lo, hi, A.ptr, A.col, A.val, diag,
                       b, x, s_in, s_out);
}

// Quad-vector CSR colour sweep: a quad per row.  Each XCD takes one
// contiguous range of the colour's rows (rows in index order, so most of the
// entries its rows gather were written by the same XCD and stay in its L2).
template <typename T, int CH, bool ZERO>
__global__ __launch_bounds__(kBlock) void k_gs_q4(int32_t lo, int32_t hi, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col, const T* __restrict__ val,
                                                  const T* __restrict__ diag, const T* __restrict__ b,
                                                  T* __restrict__ x, const T* __restrict__ s_in,
                                                  T* __restrict__ s_out) {
  const int32_t q = lo + (int32_t)((xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) >> 2);
  const int lane = threadIdx.x & 3;
  if (q >= hi) return;
  const T d = diag[q];  // requested with b, off the row's dependent chain
  const T s = quad_row_sub<T, CH>(b[q], rp[q], rp[q + 1], col, val, lane,
                                  [&](int32_t c, T a) { return gs_prod<T, ZERO>(q, c, a, lo, hi, x, s_in); });
  if (lane == 3) {
    const T xn = s / d;
    x[q] = xn;
    s_out[q] = xn;
  }
}

// 16 lanes per row, four contiguous entries per lane (quad-vector CSR data),
// in workgroups of one wavefront (four rows): a colour's gathers spread over
// four times as many compute units as with 256-thread workgroups.  Each XCD
// takes one contiguous range of the colour's rows, as in k_gs_q4.
constexpr int kV16Block = 64;
template <typename T, int CH, bool ZERO>
__global__ __launch_bounds__(kV16Block) void k_gs_v16(int32_t lo, int32_t hi, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, const T* __restrict__ val,
                                                   const T* __restrict__ diag, const T* __restrict__ b,
                                                   T* __restrict__ x, const T* __restrict__ s_in,
                                                   T* __restrict__ s_out) {
  const int32_t q = lo + (int32_t)((xcd_block(blockIdx.x, gridDim.x) * kV16Block + threadIdx.x) >> 4);
  const int lane = threadIdx.x & 15;
  if (q >= hi) return;
  const T d = diag[q];  // requested with b, off the row's dependent chain
  const T s = row16v4_sub<T, CH>(b[q], rp[q], rp[q + 1], col, val, lane,
                                 [&](int32_t c, T a) { return gs_prod<T, ZERO>(q, c, a, lo, hi, x, s_in); });
  if (lane == 15) {
    const T xn = s / d;
    x[q] = xn;
    s_out[q] = xn;
  }
}

template <typename T, int CH>
void launch_gs_v16(const MatView<T>& A, const T* diag, int32_t lo, int32_t hi, const T* b, T* x, const T* s_in,
                   T* s_out, bool zero_start, hipStream_t s) {
  const int grid = div_up((int64_t)(hi - lo) * 16, kV16Block);
  if (zero_start)
    hipLaunchKernelGGL((k_gs_v16<T, CH, true>), dim3(grid), dim3(kV16Block), 0, s, lo, hi, A.ptr, A.col, A.val, diag,
                       b, x, s_in, s_out);
  else
    hipLaunchKernelGGL((k_gs_v16<T, CH, false>), dim3(grid), dim3(kV16Block), 0, s, lo, hi, A.ptr, A.col, A.val,
                       diag, b, x, s_in, s_out);
}

template <typename T, int CH>
void launch_gs_q4(const MatView<T>& A, const T* diag, int32_t lo, int32_t hi, const T* b, T* x, const T* s_in,
                  T* s_out, bool zero_start, hipStream_t s) {
  const int grid = div_up((int64_t)(hi - lo) * 4, kBlock);
  if (zero_start)
    hipLaunchKernelGGL((k_gs_q4<T, CH, true>), dim3(grid), dim3(kBlock), 0, s, lo, hi, A.ptr, A.col, A.val, diag, b,
                       x, s_in, s_out);
  else
    hipLaunchKernelGGL((k_gs_q4<T, CH, false>), dim3(grid), dim3(kBlock), 0, s, lo, hi, A.ptr, A.col, A.val, diag, b,
                       x, s_in, s_out);
}

template <typename T, int U>
void launch_gs_sell(const MatView<T>& A, const T* diag, int32_t lo, int32_t hi, const T* b, T* x, const T* s_in,
                    T* s_out, bool zero_start, hipStream_t s) {
  const int32_t base = lo & ~63;
  const int grid = div_up(hi - base, kBlock);
  if (zero_start)
    hipLaunchKernelGGL((k_gs_sell<T, U, true>), dim3(grid), dim3(kBlock), 0, s, lo, hi, A.width, A.ptr, A.col, A.val,
                       diag, b, x, s_in, s_out);
  else
    hipLaunchKernelGGL((k_gs_sell<T, U, false>), dim3(grid), dim3(kBlock), 0, s, lo, hi, A.width, A.ptr, A.col,
                       A.val, diag, b, x, s_in, s_out);
}

template <typename T>
void launch_gs_colour(const MatView<T>& A, const T* diag, int32_t lo, int32_t hi, const T* b, T* x, const T* s_in,
                      T* s_out, bool zero_start, hipStream_t s) {
  if (hi <= lo) return;
  if (A.group == 1) {
    if (A.depth <= 8)
      launch_gs_sell<T, 8>(A, diag, lo, hi, b, x, s_in, s_out, zero_start, s);
    else if (A.depth <= 16)
      launch_gs_sell<T, 16>(A, diag, lo, hi, b, x, s_in, s_out, zero_start, s);
    else
      launch_gs_sell<T, 32>(A, diag, lo, hi, b, x, s_in, s_out, zero_start, s);
  } else if (A.group == 2) {
    if (A.depth <= 1)
      launch_gs_v16<T, 1>(A, diag, lo, hi, b, x, s_in, s_out, zero_start, s);
    else if (A.depth <= 2)
      launch_gs_v16<T, 2>(A, diag, lo, hi, b, x, s_in, s_out, zero_start, s);
    else if (A.depth <= 4)
      launch_gs_v16<T, 4>(A, diag, lo, hi, b, x, s_in, s_out, zero_start, s);
    else
      launch_gs_v16<T, 8>(A, diag, lo, hi, b, x, s_in, s_out, zero_start, s);
  } else if (A.group == 4) {
    if (A.depth <= 2)
      launch_gs_q4<T, 2>(A, diag, lo, hi, b, x, s_in, s_out, zero_start, s);
    else if (A.depth <= 4)
      launch_gs_q4<T, 4>(A, diag, lo, hi, b, x, s_in, s_out, zero_start, s);
    else
      launch_gs_q4<T, 8>(A, diag, lo, hi, b, x, s_in, s_out, zero_start, s);
  } else if (A.group == 16) {
    if (A.depth <= 4)
      launch_gs_grp<T, 16, 4>(A, diag, lo, hi, b, x, s_in, s_out, zero_start, s);
    else if (A.depth <= 8)
      launch_gs_grp<T, 16, 8>(A, diag, lo, hi, b, x, s_in, s_out, zero_start, s);
    else
      launch_gs_grp<T, 16, 16>(A, diag, lo, hi, b, x, s_in, s_out, zero_start, s);
  } else if (A.group == 32) {
    launch_gs_grp<T, 32, 4>(A, diag, lo, hi, b, x, s_in, s_out, zero_start, s);
  } else {
    launch_gs_grp<T, 64, 4>(A, diag, lo, hi, b, x, s_in, s_out, zero_start, s);
  }
  CPR_LAUNCH_CHECK();
}
template void launch_gs_colour<double>(const MatView<double>&, const double*, int32_t, int32_t, const double*,
                                       double*, const double*, double*, bool, hipStream_t);
template void launch_gs_colour<float>(const MatView<float>&, const float*, int32_t, int32_t, const float*, float*,
                                      const float*, float*, bool, hipStream_t);

// ------------------------------------------------------------------ PGS-NO
// The natural-order parallel Gauss-Seidel that Section 6 compares PGS-SCM
// with: the rows (natural order, CSR with rows padded by column -1) are split
// into nch contiguous chunks, the first r of q+1 rows and the rest of q rows;
// one lane walks its chunk in row order, reading the newest values of its own
// chunk's rows and, for rows of other chunks, the values of the sweep's start
// (snap, or 0 when snap is null: the sweep starts from x = 0).  Per row:
// s = b_i, s = s - a_ij * xt_j over stored j != i in stored order, x_i = s / a_ii.
template <typename T>
__global__ __launch_bounds__(64) void k_gs_chunks(int32_t nch, int32_t q, int32_t r, const int32_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ col, const T* __restrict__ val,
                                                  const T* __restrict__ diag, const T* __restrict__ b, T* x,
                                                  const T* __restrict__ snap) {
  const int32_t c = blockIdx.x * 64 + threadIdx.x;
  if (c >= nch) return;
  const int32_t lo = c * q + (c < r ? c : r);
  const int32_t hi = lo + q + (c < r ? 1 : 0);
  for (int32_t i = lo; i < hi; ++i) {
    T s = b[i];
    for (int32_t e = ptr[i]; e < ptr[i + 1]; ++e) {
      const int32_t j = col[e];
      if (j < 0 || j == i) continue;
      const T xt = (j >= lo && j < hi) ? x[j] : (snap ? snap[j] : (T)0);
      s = s - val[e] * xt;
    }
    x[i] = s / diag[i];
  }
}

template <typename T>
void launch_gs_chunks(const MatView<T>& A, const T* diag, int32_t n_chunks, const T* b, T* x, const T* snap,
                      hipStream_t s) {
  const int32_t n = A.n_rows;
  if (n == 0) return;
  const int32_t nch = n_chunks < 1 ? 1 : (n_chunks > n ? n : n_chunks);
  const int32_t q = n / nch, r = n % nch;
  hipLaunchKernelGGL((k_gs_chunks<T>), dim3(div_up(nch, 64)), dim3(64), 0, s, nch, q, r, A.ptr, A.col, A.val, diag, b,
                     x, snap);
  CPR_LAUNCH_CHECK();
}
template void launch_gs_chunks<double>(const MatView<double>&, const double*, int32_t, const double*, double*,
                                       const double*, hipStream_t);
template void launch_gs_chunks<float>(const MatView<float>&, const float*, int32_t, const float*, float*, const float*,
                                      hipStream_t);

// ------------------------------------------------------------------ row products
// MODE 0: y = b - A x (residual; products subtracted from b in stored order)
// MODE 1: y = A x (sum from 0 in stored order)
// MODE 2: y = y + (A x), snap = y (prolongation add; the sum from 0 first)
// MODE 3: y = A x (restriction), and rows of the next level's zero-start
//         first colour get x = y / a_ii (see ZeroStart)
// y0: y[q] requested when the row started (MODE 2), off the dependent chain.
template <typename T, int MODE>
__device__ __forceinline__ void finish_row(int32_t q, T acc, T y0, T* __restrict__ y, T* __restrict__ snap,
                                           const ZeroStart<T>& zs) {
  if (MODE == 2) {
    const T yn = y0 + acc;
    y[q] = yn;
    snap[q] = yn;
  } else {
    y[q] = acc;
    if (MODE == 3 && q < zs.n_first) {
      const T xn = acc / zs.diag[q];
      zs.x[q] = xn;
      zs.snap[q] = xn;
    }
  }
}

template <typename T, int U, int MODE>
__global__ __launch_bounds__(kBlock) void k_rows_sell(int32_t n, int32_t width, const int32_t* __restrict__ slice_ptr,
                                                      const int32_t* __restrict__ col, const T* __restrict__ val,
                                                      const T* __restrict__ b, const T* __restrict__ x,
                                                      T* __restrict__ y, T* __restrict__ snap, ZeroStart<T> zs) {
  const int32_t q = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (q >= n) return;
  T acc = (MODE == 0) ? b[q] : (T)0;
  const T y0 = (MODE == 2) ? y[q] : (T)0;
  sell_row<T, U>(q, width, slice_ptr, col, val, [&](int32_t c, T a) {
    const T prod = (c >= 0) ? a * x[c] : (T)0;
    acc = (MODE == 0) ? (acc - prod) : (acc + prod);
  });
  finish_row<T, MODE>(q, acc, y0, y, snap, zs);
}

template <typename T, int G, int CH, int MODE>
__global__ __launch_bounds__(kBlock) void k_rows_grp(int32_t n, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col, const T* __restrict__ val,
                                                     const T* __restrict__ b, const T* __restrict__ x,
                                                     T* __restrict__ y, T* __restrict__ snap, ZeroStart<T> zs) {
  const int32_t q = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  if (q >= n) return;
  T acc = (MODE == 0) ? b[q] : (T)0;
  const T y0 = (MODE == 2) ? y[q] : (T)0;
  const int32_t p0 = rp[q], p1 = rp[q + 1];
  for (int32_t p = p0; p < p1; p += G * CH) {
    const int nch = min(CH, (p1 - p + G - 1) / G);
    int32_t c[CH];
    T a[CH], prod[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int32_t e = p + u * G + lane;
      c[u] = (e < p1) ? col[e] : kPadCol;
      a[u] = (e < p1) ? val[e] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) prod[u] = (c[u] >= 0) ? a[u] * x[c[u]] : (T)0;
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (u < nch) acc = group_chunk<T, G, MODE == 0>(acc, prod[u], lane);
  }
  if (lane == last_lane<G>()) finish_row<T, MODE>(q, acc, y0, y, snap, zs);
}

template <typename T, int CH, int MODE>
__global__ __launch_bounds__(kBlock) void k_rows_q4(int32_t n, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col, const T* __restrict__ val,
                                                    const T* __restrict__ b, const T* __restrict__ x,
                                                    T* __restrict__ y, T* __restrict__ snap, ZeroStart<T> zs) {
  const int32_t q = (int32_t)((xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) >> 2);
  const int lane = threadIdx.x & 3;
  if (q >= n) return;
  const T y0 = (MODE == 2) ? y[q] : (T)0;
  // MODE 1, 2 and 3 add: subtract the negated products (the same IEEE operation)
  const T acc = quad_row_sub<T, CH>((MODE == 0) ? b[q] : (T)0, rp[q], rp[q + 1], col, val, lane,
                                    [&](int32_t c, T a) {
                                      const T pr = (c >= 0) ? a * x[c] : (T)0;
                                      return MODE == 0 ? pr : -pr;
                                    });
  if (lane == 3) finish_row<T, MODE>(q, acc, y0, y, snap, zs);
}

template <typename T, int CH, int MODE>
__global__ __launch_bounds__(kBlock) void k_rows_v16(int32_t n, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col, const T* __restrict__ val,
                                                     const T* __restrict__ b, const T* __restrict__ x,
                                                     T* __restrict__ y, T* __restrict__ snap, ZeroStart<T> zs) {
  const int32_t q = (int32_t)((xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) >> 4);
  const int lane = threadIdx.x & 15;
  if (q >= n) return;
  const T y0 = (MODE == 2) ? y[q] : (T)0;
  // MODE 1, 2 and 3 add: subtract the negated products (the same IEEE operation)
  const T acc = row16v4_sub<T, CH>((MODE == 0) ? b[q] : (T)0, rp[q], rp[q + 1], col, val, lane,
                                   [&](int32_t c, T a) {
                                     const T pr = (c >= 0) ? a * x[c] : (T)0;
                                     return MODE == 0 ? pr : -pr;
                                   });
  if (lane == 15) finish_row<T, MODE>(q, acc, y0, y, snap, zs);
}

template <typename T, int CH, int MODE>
void launch_rows_v16(const MatView<T>& A, const T* b, const T* x, T* y, T* snap, const ZeroStart<T>& zs,
                     hipStream_t s) {
  hipLaunchKernelGGL((k_rows_v16<T, CH, MODE>), dim3(div_up((int64_t)A.n_rows * 16, kBlock)), dim3(kBlock), 0, s,
                     A.n_rows, A.ptr, A.col, A.val, b, x, y, snap, zs);
}

template <typename T, int CH, int MODE>
void launch_rows_q4(const MatView<T>& A, const T* b, const T* x, T* y, T* snap, const ZeroStart<T>& zs,
                    hipStream_t s) {
  hipLaunchKernelGGL((k_rows_q4<T, CH, MODE>), dim3(div_up((int64_t)A.n_rows * 4, kBlock)), dim3(kBlock), 0, s,
                     A.n_rows, A.ptr, A.col, A.val, b, x, y, snap, zs);
}

template <typename T, int G, int CH, int MODE>
void launch_rows_grp(const MatView<T>& A, const T* b, const T* x, T* y, T* snap, const ZeroStart<T>& zs,
                     hipStream_t s) {
  hipLaunchKernelGGL((k_rows_grp<T, G, CH, MODE>), dim3(div_up((int64_t)A.n_rows * G, kBlock)), dim3(kBlock), 0, s,
                     A.n_rows, A.ptr, A.col, A.val, b, x, y, snap, zs);
}

template <typename T, int U, int MODE>
void launch_rows_sell(const MatView<T>& A, const T* b, const T* x, T* y, T* snap, const ZeroStart<T>& zs,
                      hipStream_t s) {
  hipLaunchKernelGGL((k_rows_sell<T, U, MODE>), dim3(div_up(A.n_rows, kBlock)), dim3(kBlock), 0, s, A.n_rows, A.width,
                     A.ptr, A.col, A.val, b, x, y, snap, zs);
}

template <typename T, int MODE>
void launch_rows(const MatView<T>& A, const T* b, const T* x, T* y, T* snap, const ZeroStart<T>& zs,
                 hipStream_t s) {
  if (A.n_rows == 0) return;
  if (A.group == 1 && A.depth <= 8)
    launch_rows_sell<T, 8, MODE>(A, b, x, y, snap, zs, s);
  else if (A.group == 1 && A.depth <= 16)
    launch_rows_sell<T, 16, MODE>(A, b, x, y, snap, zs, s);
  else if (A.group == 1)
    launch_rows_sell<T, 32, MODE>(A, b, x, y, snap, zs, s);
  else if (A.group == 2 && A.depth <= 1)
    launch_rows_v16<T, 1, MODE>(A, b, x, y, snap, zs, s);
  else if (A.group == 2 && A.depth <= 2)
    launch_rows_v16<T, 2, MODE>(A, b, x, y, snap, zs, s);
  else if (A.group == 2 && A.depth <= 4)
    launch_rows_v16<T, 4, MODE>(A, b, x, y, snap, zs, s);
  else if (A.group == 2)
    launch_rows_v16<T, 8, MODE>(A, b, x, y, snap, zs, s);
  else if (A.group == 4 && A.depth <= 2)
    launch_rows_q4<T, 2, MODE>(A, b, x, y, snap, zs, s);
  else if (A.group == 4 && A.depth <= 4)
    launch_rows_q4<T, 4, MODE>(A, b, x, y, snap, zs, s);
  else if (A.group == 4)
    launch_rows_q4<T, 8, MODE>(A, b, x, y, snap, zs, s);
  else if (A.group == 16 && A.depth <= 4)
    launch_rows_grp<T, 16, 4, MODE>(A, b, x, y, snap, zs, s);
  else if (A.group == 16 && A.depth <= 8)
    launch_rows_grp<T, 16, 8, MODE>(A, b, x, y, snap, zs, s);
  else if (A.group == 16)
    launch_rows_grp<T, 16, 16, MODE>(A, b, x, y, snap, zs, s);
  else if (A.group == 32)
    launch_rows_grp<T, 32, 4, MODE>(A, b, x, y, snap, zs, s);
  else
    launch_rows_grp<T, 64, 4, MODE>(A, b, x, y, snap, zs, s);
  CPR_LAUNCH_CHECK();
}

template <typename T>
void launch_csr_residual(const MatView<T>& A, const T* b, const T* x, T* r, hipStream_t s) {
  launch_rows<T, 0>(A, b, x, r, nullptr, ZeroStart<T>{}, s);
}
template <typename T>
void launch_csr_spmv(const MatView<T>& A, const T* x, T* y, hipStream_t s) {
  launch_rows<T, 1>(A, nullptr, x, y, nullptr, ZeroStart<T>{}, s);
}
template <typename T>
void launch_csr_restrict(const MatView<T>& R, const T* r, T* b, const ZeroStart<T>& zs, hipStream_t s) {
  if (zs.n_first > 0)
    launch_rows<T, 3>(R, nullptr, r, b, nullptr, zs, s);
  else
    launch_rows<T, 1>(R, nullptr, r, b, nullptr, zs, s);
}
template <typename T>
void launch_prolong_add(const MatView<T>& P, const T* e, T* x, T* snap, hipStream_t s) {
  launch_rows<T, 2>(P, nullptr, e, x, snap, ZeroStart<T>{}, s);
}
#define CPR_INST_ROWS(T)                                                                               \
  template void launch_csr_residual<T>(const MatView<T>&, const T*, const T*, T*, hipStream_t);     \
  template void launch_csr_spmv<T>(const MatView<T>&, const T*, T*, hipStream_t);                    \
  template void launch_csr_restrict<T>(const MatView<T>&, const T*, T*, const ZeroStart<T>&, hipStream_t); \
  template void launch_prolong_add<T>(const MatView<T>&, const T*, T*, T*, hipStream_t);
CPR_INST_ROWS(double)
CPR_INST_ROWS(float)
#undef CPR_INST_ROWS

}  // namespace cpr
