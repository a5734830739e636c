// Fine-level kernels of the CPR apply and the outer FGMRES on 3x3-block
// matrices: block SpMV / residual, pressure restriction (Pi_P^T) and scatter
// (Pi_P), the stage-2 block Gauss-Seidel colour kernel, diagonal-block
// inverses, the strength kernel of SETUP and small vector helpers.
#include <cfloat>
#include <cmath>

#include "kernels_common.hpp"

namespace cpr {

// ----------------------------------------------------------------- BSR SpMV
// One lane per block row; the nine planes of a slot are read lane-contiguous.
// y_r = sum over stored blocks (stored order) of a_r0*x0 + a_r1*x1 + a_r2*x2,
// each product added separately (RESID: subtracted from b_r).  Slots are
// fetched kSpmvUnroll at a time, columns and values together: a padded slot
// has column -1 and zero values, so it reads x at cell 0 and adds zeros.
constexpr int kSpmvUnroll = 2;

// Loads of matrix blocks that no later kernel reads before they leave the
// caches: the outer product streams 534 MB of FP64 blocks and the second
// stage the FP32 copy, more together than the 256 MB last-level cache holds.
// They are non-temporal so that they do not evict the vectors and AMG levels
// the following kernels read (measured: product 121.8 -> 113.1 us, FP32
// solve 11.37 -> 11.18 ms at 3.28M DOF).  The smoothers' matrices are read
// again by the next sweep and keep ordinary loads (non-temporal ones made the
// solve slower).
template <typename P>
__device__ __forceinline__ P stream_load(const P* p) {
  return __builtin_nontemporal_load(p);
}

template <typename TA, typename TX, bool RESID>
__global__ __launch_bounds__(kBlock) void k_bsr_spmv(int32_t n, const int32_t* __restrict__ slice_ptr,
                                                     const int32_t* __restrict__ col,
                                                     const TA* __restrict__ val, const TX* __restrict__ x,
                                                     const double* __restrict__ b, double* __restrict__ y) {
  const int32_t row = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (row >= n) return;
  const int32_t slice = row >> 6, lane = row & 63;
  double y0, y1, y2;
  if (RESID) {
    y0 = b[3 * (int64_t)row];
    y1 = b[3 * (int64_t)row + 1];
    y2 = b[3 * (int64_t)row + 2];
  } else {
    y0 = 0.0;
    y1 = 0.0;
    y2 = 0.0;
  }
  const int32_t t0 = slice_ptr[slice], t1 = slice_ptr[slice + 1];
  for (int32_t t = t0; t < t1; t += kSpmvUnroll) {
    int64_t c[kSpmvUnroll];
    double a[kSpmvUnroll][9];
#pragma unroll
    for (int u = 0; u < kSpmvUnroll; ++u) {
      const bool live = t + u < t1;
      const int32_t cw = live ? stream_load(col + (int64_t)(t + u) * kWave + lane) : kPadCol;
      c[u] = cw < 0 ? 0 : cw;
      const TA* vb = val + (int64_t)(t + u) * (9 * kWave) + lane;
#pragma unroll
      for (int e = 0; e < 9; ++e) a[u][e] = live ? (double)stream_load(vb + e * kWave) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kSpmvUnroll; ++u) {
      const double x0 = (double)x[3 * c[u]], x1 = (double)x[3 * c[u] + 1], x2 = (double)x[3 * c[u] + 2];
      if (RESID) {
        y0 = y0 - a[u][0] * x0; y0 = y0 - a[u][1] * x1; y0 = y0 - a[u][2] * x2;
        y1 = y1 - a[u][3] * x0; y1 = y1 - a[u][4] * x1; y1 = y1 - a[u][5] * x2;
        y2 = y2 - a[u][6] * x0; y2 = y2 - a[u][7] * x1; y2 = y2 - a[u][8] * x2;
      } else {
        y0 = y0 + a[u][0] * x0; y0 = y0 + a[u][1] * x1; y0 = y0 + a[u][2] * x2;
        y1 = y1 + a[u][3] * x0; y1 = y1 + a[u][4] * x1; y1 = y1 + a[u][5] * x2;
        y2 = y2 + a[u][6] * x0; y2 = y2 + a[u][7] * x1; y2 = y2 + a[u][8] * x2;
      }
    }
  }
  y[3 * (int64_t)row] = y0;
  y[3 * (int64_t)row + 1] = y1;
  y[3 * (int64_t)row + 2] = y2;
}

template <typename TA, typename TX>
void launch_bsr_spmv(const SellView<TA>& A, const TX* x, const double* b, double* y, hipStream_t s) {
  if (A.n_rows == 0) return;
  const int grid = div_up(A.n_rows, kBlock);
  if (b)
    hipLaunchKernelGGL((k_bsr_spmv<TA, TX, true>), dim3(grid), dim3(kBlock), 0, s, A.n_rows, A.slice_ptr, A.col,
                       A.val, x, b, y);
  else
    hipLaunchKernelGGL((k_bsr_spmv<TA, TX, false>), dim3(grid), dim3(kBlock), 0, s, A.n_rows, A.slice_ptr, A.col,
                       A.val, x, b, y);
  CPR_LAUNCH_CHECK();
}

template void launch_bsr_spmv<double, double>(const SellView<double>&, const double*, const double*, double*,
                                              hipStream_t);
template void launch_bsr_spmv<double, float>(const SellView<double>&, const float*, const double*, double*,
                                             hipStream_t);

// ----------------------------------------------------------------- Pi_P^T, Pi_P
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict_pressure(int32_t n, const double* __restrict__ v,
                                                              const int32_t* __restrict__ perm,
                                                              T* __restrict__ rp, ZeroStart<T> zs) {
  const int32_t p = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (p >= n) return;
  const T b = (T)v[3 * (int64_t)perm[p]];
  rp[p] = b;
  if (p < zs.n_first) {  // first colour of a zero-start sweep: x = b / a_ii
    const T xn = b / zs.diag[p];
    zs.x[p] = xn;
    zs.snap[p] = xn;
  }
}

template <typename T>
void launch_restrict_pressure(int32_t n, const double* v, const int32_t* perm, T* rp, const ZeroStart<T>& zs,
                              hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_restrict_pressure<T>), dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, n, v, perm, rp, zs);
  CPR_LAUNCH_CHECK();
}
template void launch_restrict_pressure<double>(int32_t, const double*, const int32_t*, double*,
                                               const ZeroStart<double>&, hipStream_t);
template void launch_restrict_pressure<float>(int32_t, const double*, const int32_t*, float*,
                                              const ZeroStart<float>&, hipStream_t);

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter(int32_t n, const T* __restrict__ e,
                                                    const int32_t* __restrict__ perm, T* __restrict__ pe) {
  const int32_t p = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (p >= n) return;
  pe[perm[p]] = e[p];
}

template <typename T>
void launch_scatter(int32_t n, const T* e, const int32_t* perm, T* pe, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_scatter<T>), dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, n, e, perm, pe);
  CPR_LAUNCH_CHECK();
}
template void launch_scatter<double>(int32_t, const double*, const int32_t*, double*, hipStream_t);
template void launch_scatter<float>(int32_t, const float*, const int32_t*, float*, hipStream_t);

// ----------------------------------------------------------------- stage 2
constexpr int kStage2Unroll = 4;

// Rows of A are cells in block-colour order.  For the cells q in [lo, hi) of
// one colour (cell i = cell[q]):
//   t = v_i - sum_j A_ij zt_j,  zt_j = z_j (neighbour of an earlier colour,
//       flagged in the column word; full block) or (pe_j, 0, 0) (column 0 only),
//   d = Dinv_i t,  z_i = (pe_i + d_0, d_1, d_2).
// This is Algorithm "CPR method" with x = 0: z = Pi_P e, r = v - A z, then one
// forward multi-colour block Gauss-Seidel sweep on r from zero, z += d.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_stage2(int32_t lo, int32_t hi, const int32_t* __restrict__ slice_ptr,
                                                   const int32_t* __restrict__ col, const T* __restrict__ val,
                                                   const int32_t* __restrict__ cell, const T* __restrict__ dinv,
                                                   int32_t ld, const double* __restrict__ v,
                                                   const T* __restrict__ pe, T* __restrict__ z) {
  const int32_t base = lo & ~63;
  const int32_t q = base + xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (q < lo || q >= hi) return;
  const int32_t slice = q >> 6, lane = q & 63;
  const int64_t i = cell[q];
  T t0 = (T)v[3 * i], t1 = (T)v[3 * i + 1], t2 = (T)v[3 * i + 2];
  // D^-1 of this cell and its pressure correction, requested with the row's
  // first loads rather than after the neighbour loop
  T dm[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) dm[e] = dinv[q + e * (int64_t)ld];
  const T pei = pe[i];
  const int32_t s0 = slice_ptr[slice], s1 = slice_ptr[slice + 1];
  for (int32_t t = s0; t < s1; t += kStage2Unroll) {
    // column words of a few slots first, then their value planes and vector
    // entries together; padded slots (column -1) contribute nothing
    int32_t cw[kStage2Unroll];
#pragma unroll
    for (int u = 0; u < kStage2Unroll; ++u)
      cw[u] = (t + u < s1) ? stream_load(col + (int64_t)(t + u) * kWave + lane) : kPadCol;
#pragma unroll
    for (int u = 0; u < kStage2Unroll; ++u) {
      const int32_t c = cw[u];
      if (c == kPadCol) continue;
      const int64_t j = c & kColMask;
      const T* vb = val + (int64_t)(t + u) * (9 * kWave) + lane;
      if (c & kEarlierBit) {
        const T z0 = z[3 * j], z1 = z[3 * j + 1], z2 = z[3 * j + 2];
        const T a00 = stream_load(vb), a01 = stream_load(vb + kWave), a02 = stream_load(vb + 2 * kWave);
        const T a10 = stream_load(vb + 3 * kWave), a11 = stream_load(vb + 4 * kWave), a12 = stream_load(vb + 5 * kWave);
        const T a20 = stream_load(vb + 6 * kWave), a21 = stream_load(vb + 7 * kWave), a22 = stream_load(vb + 8 * kWave);
        t0 = t0 - a00 * z0; t0 = t0 - a01 * z1; t0 = t0 - a02 * z2;
        t1 = t1 - a10 * z0; t1 = t1 - a11 * z1; t1 = t1 - a12 * z2;
        t2 = t2 - a20 * z0; t2 = t2 - a21 * z1; t2 = t2 - a22 * z2;
      } else {
        const T p = pe[j];
        const T a00 = stream_load(vb), a10 = stream_load(vb + 3 * kWave), a20 = stream_load(vb + 6 * kWave);
        t0 = t0 - a00 * p;
        t1 = t1 - a10 * p;
        t2 = t2 - a20 * p;
      }
    }
  }
  T d0 = (T)0, d1 = (T)0, d2 = (T)0;
  d0 = d0 + dm[0] * t0; d0 = d0 + dm[1] * t1; d0 = d0 + dm[2] * t2;
  d1 = d1 + dm[3] * t0; d1 = d1 + dm[4] * t1; d1 = d1 + dm[5] * t2;
  d2 = d2 + dm[6] * t0; d2 = d2 + dm[7] * t1; d2 = d2 + dm[8] * t2;
  z[3 * i] = pei + d0;
  z[3 * i + 1] = d1;
  z[3 * i + 2] = d2;
}

template <typename T>
void launch_stage2(const SellView<T>& A, int32_t lo, int32_t hi, const int32_t* cell, const T* dinv,
                   int32_t dinv_ld, const double* v, const T* pe, T* z, hipStream_t s) {
  if (hi <= lo) return;
  const int32_t base = lo & ~63;
  hipLaunchKernelGGL((k_stage2<T>), dim3(div_up(hi - base, kBlock)), dim3(kBlock), 0, s, lo, hi, A.slice_ptr,
                     A.col, A.val, cell, dinv, dinv_ld, v, pe, z);
  CPR_LAUNCH_CHECK();
}
template void launch_stage2<double>(const SellView<double>&, int32_t, int32_t, const int32_t*, const double*,
                                    int32_t, const double*, const double*, double*, hipStream_t);
template void launch_stage2<float>(const SellView<float>&, int32_t, int32_t, const int32_t*, const float*,
                                   int32_t, const double*, const float*, float*, hipStream_t);

// ----------------------------------------------------------------- D^{-1}
// 3x3 LU with partial pivoting (FP64), then the inverse column by column.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_block_inverse(int32_t n, const double* __restrict__ vals,
                                                          const int64_t* __restrict__ diag_pos,
                                                          T* __restrict__ dinv, int32_t ld,
                                                          int32_t* __restrict__ singular) {
  const int32_t q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  double inv[9];
  if (!inverse3x3(vals + 9 * diag_pos[q], inv)) {
    singular[0] = 1;
    for (int e = 0; e < 9; ++e) dinv[(int64_t)e * ld + q] = (T)0;
    return;
  }
  for (int e = 0; e < 9; ++e) dinv[(int64_t)e * ld + q] = (T)inv[e];
}

// SETUP's view of the input values, one thread per block row i (rows and
// columns of the input BSR): the pressure entry (0,0) of every stored block,
// whether the block has any nonzero entry (stage-2 block graph), and the
// first row whose diagonal block fails LU with partial pivoting (a pivot not
// above 1e-300 times the block's largest entry, or an all-zero block).
__global__ __launch_bounds__(kBlock) void k_setup_values(int32_t n, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ vals, double* __restrict__ pval,
                                                         uint8_t* __restrict__ nonzero, int32_t* __restrict__ bad_row) {
  const int32_t i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
    const double* v = vals + (int64_t)k * 9;
    pval[k] = v[0];
    bool nz = false;
    for (int e = 0; e < 9; ++e) nz = nz || v[e] != 0.0;
    nonzero[k] = nz ? 1 : 0;
    if (col[k] != i) continue;
    double a[3][3], amax = 0.0;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        a[r][c] = v[3 * r + c];
        amax = fmax(amax, fabs(a[r][c]));
      }
    bool bad = !(amax > 0.0);
    for (int kk = 0; kk < 3 && !bad; ++kk) {
      int p = kk;
      for (int r = kk + 1; r < 3; ++r)
        if (fabs(a[r][kk]) > fabs(a[p][kk])) p = r;
      if (!(fabs(a[p][kk]) > 1e-300 * amax)) bad = true;
      for (int c = 0; c < 3; ++c) {
        const double t = a[kk][c];
        a[kk][c] = a[p][c];
        a[p][c] = t;
      }
      for (int r = kk + 1; r < 3 && !bad; ++r) {
        const double l = a[r][kk] / a[kk][kk];
        for (int c = kk + 1; c < 3; ++c) a[r][c] = a[r][c] - l * a[kk][c];
      }
    }
    if (bad) atomicMin(bad_row, i);
  }
}

void launch_setup_values(int32_t n, const int32_t* rp, const int32_t* col, const double* vals, double* pval,
                         uint8_t* nonzero, int32_t* bad_row, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_setup_values, dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, n, rp, col, vals, pval, nonzero,
                     bad_row);
  CPR_LAUNCH_CHECK();
}

template <typename T>
void launch_block_inverse(int32_t n, const double* vals, const int64_t* diag_pos, T* dinv, int32_t ld,
                          int32_t* singular, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_block_inverse<T>), dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, n, vals, diag_pos, dinv, ld,
                     singular);
  CPR_LAUNCH_CHECK();
}
template void launch_block_inverse<double>(int32_t, const double*, const int64_t*, double*, int32_t, int32_t*,
                                           hipStream_t);
template void launch_block_inverse<float>(int32_t, const double*, const int64_t*, float*, int32_t, int32_t*,
                                          hipStream_t);

// ----------------------------------------------------------------- value scatter
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bsr_values_to_sell(int64_t nnzb, const double* __restrict__ vals,
                                                               const int64_t* __restrict__ pos,
                                                               T* __restrict__ sv) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= nnzb) return;
  const int64_t e = pos[k];
  const int64_t slot = e >> 6, lane = e & 63;
  T* dst = sv + slot * (9 * kWave) + lane;
  const double* src = vals + 9 * k;
  for (int v = 0; v < 9; ++v) dst[v * kWave] = (T)src[v];
}

template <typename T>
void launch_bsr_values_to_sell(int64_t nnzb, const double* vals, const int64_t* pos, T* sv, hipStream_t s) {
  if (nnzb == 0) return;
  hipLaunchKernelGGL((k_bsr_values_to_sell<T>), dim3(div_up(nnzb, kBlock)), dim3(kBlock), 0, s, nnzb, vals, pos, sv);
  CPR_LAUNCH_CHECK();
}
template void launch_bsr_values_to_sell<double>(int64_t, const double*, const int64_t*, double*, hipStream_t);
template void launch_bsr_values_to_sell<float>(int64_t, const double*, const int64_t*, float*, hipStream_t);

// ----------------------------------------------------------------- strength
// Per row i (original CSR, stored order):
//   RS (bit 1):      j != i and max_{k != i}(-a_ik) > 0 and -a_ij >= theta_rs * max
//   colouring (bit 2, eq. (strong-matrix)):  j != i and |a_ij| > theta_c * sum_k |a_ik|,
//                    the sum over every stored entry, left to right.
__global__ __launch_bounds__(kBlock) void k_strength(int32_t n, const int32_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ val, double theta_rs,
                                                     double theta_c, uint8_t* __restrict__ mask) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t p0 = ptr[i], p1 = ptr[i + 1];
  double mx = -HUGE_VAL, sum = 0.0;
  for (int32_t p = p0; p < p1; ++p) {
    const double a = val[p];
    sum = sum + fabs(a);
    if (col[p] != i && -a > mx) mx = -a;
  }
  const double brs = theta_rs * mx, bc = theta_c * sum;
  for (int32_t p = p0; p < p1; ++p) {
    const double a = val[p];
    uint8_t bits = 0;
    if (col[p] != i) {
      if (mx > 0.0 && -a >= brs) bits |= 1;
      if (fabs(a) > bc) bits |= 2;
    }
    mask[p] = bits;
  }
}

void launch_strength(int32_t n, const int32_t* ptr, const int32_t* col, const double* val, double theta_rs,
                     double theta_color, uint8_t* mask, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_strength, dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, n, ptr, col, val, theta_rs,
                     theta_color, mask);
  CPR_LAUNCH_CHECK();
}

// ----------------------------------------------------------------- vector helpers
template <typename TS, typename TD>
__global__ __launch_bounds__(kBlock) void k_gather(int32_t n, const TS* __restrict__ src,
                                                   const int32_t* __restrict__ perm, TD* __restrict__ dst) {
  const int32_t p = blockIdx.x * kBlock + threadIdx.x;
  if (p < n) dst[p] = (TD)src[perm[p]];
}
template <typename TS, typename TD>
__global__ __launch_bounds__(kBlock) void k_scatter_cast(int32_t n, const TS* __restrict__ src,
                                                         const int32_t* __restrict__ perm, TD* __restrict__ dst) {
  const int32_t p = blockIdx.x * kBlock + threadIdx.x;
  if (p < n) dst[perm[p]] = (TD)src[p];
}
template <typename TS, typename TD>
void launch_gather(int32_t n, const TS* src, const int32_t* perm, TD* dst, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_gather<TS, TD>), dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, n, src, perm, dst);
  CPR_LAUNCH_CHECK();
}
template <typename TS, typename TD>
void launch_scatter_cast(int32_t n, const TS* src, const int32_t* perm, TD* dst, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_scatter_cast<TS, TD>), dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, n, src, perm, dst);
  CPR_LAUNCH_CHECK();
}
#define CPR_INST_GS(TS, TD)                                                                   \
  template void launch_gather<TS, TD>(int32_t, const TS*, const int32_t*, TD*, hipStream_t); \
  template void launch_scatter_cast<TS, TD>(int32_t, const TS*, const int32_t*, TD*, hipStream_t);
CPR_INST_GS(double, double)
CPR_INST_GS(double, float)
CPR_INST_GS(float, double)
CPR_INST_GS(float, float)
#undef CPR_INST_GS

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, T value, T* __restrict__ dst) {
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock)
    dst[k] = value;
}
template <typename T>
void launch_fill(int64_t n, T value, T* dst, hipStream_t s) {
  if (n == 0) return;
  const int grid = (int)std::min<int64_t>(div_up(n, kBlock), 4096);
  hipLaunchKernelGGL((k_fill<T>), dim3(grid), dim3(kBlock), 0, s, n, value, dst);
  CPR_LAUNCH_CHECK();
}
template void launch_fill<double>(int64_t, double, double*, hipStream_t);
template void launch_fill<float>(int64_t, float, float*, hipStream_t);
template void launch_fill<int32_t>(int64_t, int32_t, int32_t*, hipStream_t);

template <typename TS, typename TD>
__global__ __launch_bounds__(kBlock) void k_copy_cast(int64_t n, const TS* __restrict__ src, TD* __restrict__ dst) {
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock)
    dst[k] = (TD)src[k];
}
template <typename TS, typename TD>
void launch_copy_cast(int64_t n, const TS* src, TD* dst, hipStream_t s) {
  if (n == 0) return;
  const int grid = (int)std::min<int64_t>(div_up(n, kBlock), 8192);
  hipLaunchKernelGGL((k_copy_cast<TS, TD>), dim3(grid), dim3(kBlock), 0, s, n, src, dst);
  CPR_LAUNCH_CHECK();
}
template void launch_copy_cast<double, double>(int64_t, const double*, double*, hipStream_t);
template void launch_copy_cast<double, float>(int64_t, const double*, float*, hipStream_t);
template void launch_copy_cast<float, double>(int64_t, const float*, double*, hipStream_t);
template void launch_copy_cast<float, float>(int64_t, const float*, float*, hipStream_t);

// flag = 1 if a[i] != b[i] for some i < n (every writer stores the same value).
__global__ __launch_bounds__(kBlock) void k_int_diff(int64_t n, const int32_t* __restrict__ a,
                                                     const int32_t* __restrict__ b, int32_t* __restrict__ flag) {
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock)
    if (a[k] != b[k]) *flag = 1;
}
void launch_int_diff(int64_t n, const int32_t* a, const int32_t* b, int32_t* flag, hipStream_t s) {
  if (n <= 0) return;
  const int grid = (int)std::min<int64_t>(div_up(n, kBlock), 4096);
  hipLaunchKernelGGL(k_int_diff, dim3(grid), dim3(kBlock), 0, s, n, a, b, flag);
  CPR_LAUNCH_CHECK();
}

// Plain streaming copy in 16-byte words (tail in bytes); used to calibrate
// hardware traffic counters against a kernel of known size.
__global__ __launch_bounds__(kBlock) void k_copy_bytes(int64_t n16, const uint4* __restrict__ src,
                                                       uint4* __restrict__ dst) {
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n16; k += (int64_t)gridDim.x * kBlock)
    dst[k] = src[k];
}
__global__ void k_copy_tail(int64_t n, const uint8_t* __restrict__ src, uint8_t* __restrict__ dst) {
  const int64_t k = threadIdx.x;
  if (k < n) dst[k] = src[k];
}
void launch_copy_bytes(int64_t n_bytes, const void* src, void* dst, hipStream_t s) {
  const int64_t n16 = n_bytes / 16;
  if (n16 > 0) {
    const int grid = (int)std::min<int64_t>(div_up(n16, kBlock), 8192);
    hipLaunchKernelGGL(k_copy_bytes, dim3(grid), dim3(kBlock), 0, s, n16, (const uint4*)src, (uint4*)dst);
  }
  const int64_t tail = n_bytes - 16 * n16;
  if (tail > 0)
    hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(16), 0, s, tail, (const uint8_t*)src + 16 * n16,
                       (uint8_t*)dst + 16 * n16);
  CPR_LAUNCH_CHECK();
}

}  // namespace cpr
