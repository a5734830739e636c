// Second stage by block ILU(0) (the R of eq. (CPR) that Section 3.1 names),
// applied with level-scheduled triangular solves (Section 6): one launch per
// level, the rows of a level one per lane.  Rows of a level depend only on
// rows of earlier levels, and every row sums its products in stored block
// order, so the result does not depend on the schedule.
//
// The kernels read block SELL-64 images (slice s = rows or positions
// 64s..64s+63; slot t of a slice holds the t-th kept block of each row; plane
// e of slot t, lane l at (t*P + e)*64 + l for P planes; padding has column -1
// at the end of a row): the residual's in natural row order, the triangular
// solves' in their level order.
#include "kernels_common.hpp"

namespace cpr {

// The CPR residual before the forward solve, every row at once (it does
// not depend on the level order): r_i = v_i - sum_j A_ij (pe_j, 0, 0) over
// every stored block j of row i in stored order (image R: column 0 of each
// block, 3 planes, rows in natural order).  This is Algorithm "CPR method"
// with x = 0 up to the second stage: z = Pi_P e, r = v - A z.
constexpr int kBiluUnroll = 4;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_bilu_residual(int32_t n, const int32_t* __restrict__ r_sp,
                                                          const int32_t* __restrict__ r_col,
                                                          const T* __restrict__ r_val, const double* __restrict__ v,
                                                          const T* __restrict__ pe, T* __restrict__ r) {
  const int32_t i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t slice = i >> 6, lane = i & 63;
  T t0 = (T)v[3 * (int64_t)i], t1 = (T)v[3 * (int64_t)i + 1], t2 = (T)v[3 * (int64_t)i + 2];
  const int32_t a0 = r_sp[slice], a1 = r_sp[slice + 1];
  for (int32_t t = a0; t < a1; t += kBiluUnroll) {
    int32_t c[kBiluUnroll];
#pragma unroll
    for (int u = 0; u < kBiluUnroll; ++u) c[u] = (t + u < a1) ? r_col[(int64_t)(t + u) * kWave + lane] : kPadCol;
#pragma unroll
    for (int u = 0; u < kBiluUnroll; ++u) {
      if (c[u] == kPadCol) continue;
      const T* vb = r_val + (int64_t)(t + u) * (3 * kWave) + lane;
      const T p = pe[c[u]];
      t0 = t0 - vb[0] * p;
      t1 = t1 - vb[kWave] * p;
      t2 = t2 - vb[2 * kWave] * p;
    }
  }
  r[3 * (int64_t)i] = t0;
  r[3 * (int64_t)i + 1] = t1;
  r[3 * (int64_t)i + 2] = t2;
}

// Forward solve, positions [lo, hi) of one level (row i = row[q]):
//   y_i = r_i - sum_{k<i} L_ik y_k   (image L: the lower blocks, 9 planes,
// rows in forward-level order).  The columns of a few slots are fetched
// first, then their value planes and the neighbours' y together, so a row
// costs two dependent memory round trips per four blocks.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bilu_forward(int32_t lo, int32_t hi, const int32_t* __restrict__ l_sp,
                                                         const int32_t* __restrict__ l_col,
                                                         const T* __restrict__ l_val, const int32_t* __restrict__ row,
                                                         const T* __restrict__ r, T* __restrict__ y) {
  const int32_t base = lo & ~63;
  const int32_t q = base + xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (q < lo || q >= hi) return;
  const int32_t slice = q >> 6, lane = q & 63;
  const int64_t i = row[q];
  T t0 = r[3 * i], t1 = r[3 * i + 1], t2 = r[3 * i + 2];
  const int32_t b0 = l_sp[slice], b1 = l_sp[slice + 1];
  for (int32_t t = b0; t < b1; t += kBiluUnroll) {
    int32_t c[kBiluUnroll];
#pragma unroll
    for (int u = 0; u < kBiluUnroll; ++u) c[u] = (t + u < b1) ? l_col[(int64_t)(t + u) * kWave + lane] : kPadCol;
#pragma unroll
    for (int u = 0; u < kBiluUnroll; ++u) {
      if (c[u] == kPadCol) continue;
      const T* vb = l_val + (int64_t)(t + u) * (9 * kWave) + lane;
      const int64_t k = c[u];
      const T y0 = y[3 * k], y1 = y[3 * k + 1], y2 = y[3 * k + 2];
      t0 = t0 - vb[0 * kWave] * y0; t0 = t0 - vb[1 * kWave] * y1; t0 = t0 - vb[2 * kWave] * y2;
      t1 = t1 - vb[3 * kWave] * y0; t1 = t1 - vb[4 * kWave] * y1; t1 = t1 - vb[5 * kWave] * y2;
      t2 = t2 - vb[6 * kWave] * y0; t2 = t2 - vb[7 * kWave] * y1; t2 = t2 - vb[8 * kWave] * y2;
    }
  }
  y[3 * i] = t0;
  y[3 * i + 1] = t1;
  y[3 * i + 2] = t2;
}

// Backward solve, positions [lo, hi) of one level (row i = row[q]):
//   d_i = Uinv_i (y_i - sum_{j>i} U_ij d_j)   (image U: the upper blocks;
//         Uinv planes uinv[e*ld + q]; each component of the product summed
//         from 0 over columns 0, 1, 2),
//   z_i = (pe_i + d_i0, d_i1, d_i2)           (z = Pi_P e + d).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bilu_backward(int32_t lo, int32_t hi, const int32_t* __restrict__ u_sp,
                                                          const int32_t* __restrict__ u_col,
                                                          const T* __restrict__ u_val, const T* __restrict__ uinv,
                                                          int32_t ld, const int32_t* __restrict__ row,
                                                          const T* __restrict__ y, const T* __restrict__ pe,
                                                          T* __restrict__ d, T* __restrict__ z) {
  const int32_t base = lo & ~63;
  const int32_t q = base + xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (q < lo || q >= hi) return;
  const int32_t slice = q >> 6, lane = q & 63;
  const int64_t i = row[q];
  T um[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) um[e] = uinv[q + e * (int64_t)ld];
  const T pei = pe[i];
  T t0 = y[3 * i], t1 = y[3 * i + 1], t2 = y[3 * i + 2];
  const int32_t a0 = u_sp[slice], a1 = u_sp[slice + 1];
  for (int32_t t = a0; t < a1; t += kBiluUnroll) {
    int32_t c[kBiluUnroll];
#pragma unroll
    for (int u = 0; u < kBiluUnroll; ++u) c[u] = (t + u < a1) ? u_col[(int64_t)(t + u) * kWave + lane] : kPadCol;
#pragma unroll
    for (int u = 0; u < kBiluUnroll; ++u) {
      if (c[u] == kPadCol) continue;
      const T* vb = u_val + (int64_t)(t + u) * (9 * kWave) + lane;
      const int64_t j = c[u];
      const T d0 = d[3 * j], d1 = d[3 * j + 1], d2 = d[3 * j + 2];
      t0 = t0 - vb[0 * kWave] * d0; t0 = t0 - vb[1 * kWave] * d1; t0 = t0 - vb[2 * kWave] * d2;
      t1 = t1 - vb[3 * kWave] * d0; t1 = t1 - vb[4 * kWave] * d1; t1 = t1 - vb[5 * kWave] * d2;
      t2 = t2 - vb[6 * kWave] * d0; t2 = t2 - vb[7 * kWave] * d1; t2 = t2 - vb[8 * kWave] * d2;
    }
  }
  T o0 = (T)0, o1 = (T)0, o2 = (T)0;
  o0 = o0 + um[0] * t0; o0 = o0 + um[1] * t1; o0 = o0 + um[2] * t2;
  o1 = o1 + um[3] * t0; o1 = o1 + um[4] * t1; o1 = o1 + um[5] * t2;
  o2 = o2 + um[6] * t0; o2 = o2 + um[7] * t1; o2 = o2 + um[8] * t2;
  d[3 * i] = o0;
  d[3 * i + 1] = o1;
  d[3 * i + 2] = o2;
  z[3 * i] = pei + o0;
  z[3 * i + 1] = o1;
  z[3 * i + 2] = o2;
}

template <typename T>
void launch_bilu_residual(const SellView<T>& R, const double* v, const T* pe, T* r, hipStream_t s) {
  if (R.n_rows == 0) return;
  hipLaunchKernelGGL((k_bilu_residual<T>), dim3(div_up(R.n_rows, kBlock)), dim3(kBlock), 0, s, R.n_rows,
                     R.slice_ptr, R.col, R.val, v, pe, r);
  CPR_LAUNCH_CHECK();
}

template <typename T>
void launch_bilu_forward(int32_t lo, int32_t hi, const SellView<T>& L, const int32_t* row, const T* r, T* y,
                         hipStream_t s) {
  if (hi <= lo) return;
  const int32_t base = lo & ~63;
  hipLaunchKernelGGL((k_bilu_forward<T>), dim3(div_up(hi - base, kBlock)), dim3(kBlock), 0, s, lo, hi, L.slice_ptr,
                     L.col, L.val, row, r, y);
  CPR_LAUNCH_CHECK();
}

template <typename T>
void launch_bilu_backward(int32_t lo, int32_t hi, const SellView<T>& U, const T* uinv, int32_t ld, const int32_t* row,
                          const T* y, const T* pe, T* d, T* z, hipStream_t s) {
  if (hi <= lo) return;
  const int32_t base = lo & ~63;
  hipLaunchKernelGGL((k_bilu_backward<T>), dim3(div_up(hi - base, kBlock)), dim3(kBlock), 0, s, lo, hi, U.slice_ptr,
                     U.col, U.val, uinv, ld, row, y, pe, d, z);
  CPR_LAUNCH_CHECK();
}

template void launch_bilu_residual<double>(const SellView<double>&, const double*, const double*, double*,
                                           hipStream_t);
template void launch_bilu_residual<float>(const SellView<float>&, const double*, const float*, float*, hipStream_t);
template void launch_bilu_forward<double>(int32_t, int32_t, const SellView<double>&, const int32_t*, const double*,
                                          double*, hipStream_t);
template void launch_bilu_forward<float>(int32_t, int32_t, const SellView<float>&, const int32_t*, const float*,
                                         float*, hipStream_t);
template void launch_bilu_backward<double>(int32_t, int32_t, const SellView<double>&, const double*, int32_t,
                                           const int32_t*, const double*, const double*, double*, double*,
                                           hipStream_t);
template void launch_bilu_backward<float>(int32_t, int32_t, const SellView<float>&, const float*, int32_t,
                                          const int32_t*, const float*, const float*, float*, float*, hipStream_t);

}  // namespace cpr
