// Pressure-AMG kernels: the PGS-SCM colour sweep (Algorithm "PGS-SCM"),
// residual, restriction, prolongation and the dense coarsest solve.  Level
// matrices are SELL-64 with rows in colour order; each lane sums its own row
// in stored order, so results match a sequential row loop bit for bit.
#include "kernels_common.hpp"

namespace cpr {

// One colour [lo, hi).  Same-colour neighbours are read from the snapshot s_in
// (their values before this colour started), all others from x (earlier
// colours already updated in this sweep).  ZERO: x == 0 on entry, so only the
// earlier colours (j < lo) contribute.
template <typename T, bool ZERO>
__global__ __launch_bounds__(kBlock) void k_gs_colour(int32_t lo, int32_t hi, const int32_t* __restrict__ slice_ptr,
                                                      const int32_t* __restrict__ col, const T* __restrict__ val,
                                                      const T* __restrict__ diag, const T* __restrict__ b,
                                                      T* __restrict__ x, const T* __restrict__ s_in,
                                                      T* __restrict__ s_out) {
  const int32_t base = lo & ~63;
  const int32_t q = base + xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (q < lo || q >= hi) return;
  const int32_t slice = q >> 6, lane = q & 63;
  T s = b[q];
  const int32_t t0 = slice_ptr[slice], t1 = slice_ptr[slice + 1];
  for (int32_t t = t0; t < t1; ++t) {
    const int64_t e = (int64_t)t * kWave + lane;
    const int32_t c = col[e];
    if (c < 0) break;
    if (c == q) continue;
    T xv;
    if (ZERO) {
      if (c >= lo) continue;
      xv = x[c];
    } else {
      xv = (c >= lo && c < hi) ? s_in[c] : x[c];
    }
    s = s - val[e] * xv;
  }
  const T xn = s / diag[q];
  x[q] = xn;
  s_out[q] = xn;
}

template <typename T>
void launch_gs_colour(const SellView<T>& A, const T* diag, int32_t lo, int32_t hi, const T* b, T* x, const T* s_in,
                      T* s_out, bool zero_start, hipStream_t s) {
  if (hi <= lo) return;
  const int32_t base = lo & ~63;
  const int grid = div_up(hi - base, kBlock);
  if (zero_start)
    hipLaunchKernelGGL((k_gs_colour<T, true>), dim3(grid), dim3(kBlock), 0, s, lo, hi, A.slice_ptr, A.col, A.val,
                       diag, b, x, s_in, s_out);
  else
    hipLaunchKernelGGL((k_gs_colour<T, false>), dim3(grid), dim3(kBlock), 0, s, lo, hi, A.slice_ptr, A.col, A.val,
                       diag, b, x, s_in, s_out);
  CPR_LAUNCH_CHECK();
}
template void launch_gs_colour<double>(const SellView<double>&, const double*, int32_t, int32_t, const double*,
                                       double*, const double*, double*, bool, hipStream_t);
template void launch_gs_colour<float>(const SellView<float>&, const float*, int32_t, int32_t, const float*, float*,
                                      const float*, float*, bool, hipStream_t);

// r_i = b_i - a_i1 x_1 - a_i2 x_2 - ... (stored order, diagonal included)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_csr_residual(int32_t n, const int32_t* __restrict__ slice_ptr,
                                                         const int32_t* __restrict__ col, const T* __restrict__ val,
                                                         const T* __restrict__ b, const T* __restrict__ x,
                                                         T* __restrict__ r) {
  const int32_t q = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (q >= n) return;
  const int32_t slice = q >> 6, lane = q & 63;
  T s = b[q];
  const int32_t t0 = slice_ptr[slice], t1 = slice_ptr[slice + 1];
  for (int32_t t = t0; t < t1; ++t) {
    const int64_t e = (int64_t)t * kWave + lane;
    const int32_t c = col[e];
    if (c < 0) break;
    s = s - val[e] * x[c];
  }
  r[q] = s;
}

template <typename T>
void launch_csr_residual(const SellView<T>& A, const T* b, const T* x, T* r, hipStream_t s) {
  if (A.n_rows == 0) return;
  hipLaunchKernelGGL((k_csr_residual<T>), dim3(div_up(A.n_rows, kBlock)), dim3(kBlock), 0, s, A.n_rows, A.slice_ptr,
                     A.col, A.val, b, x, r);
  CPR_LAUNCH_CHECK();
}
template void launch_csr_residual<double>(const SellView<double>&, const double*, const double*, double*,
                                          hipStream_t);
template void launch_csr_residual<float>(const SellView<float>&, const float*, const float*, float*, hipStream_t);

// y_i = 0 + a_i1 x_1 + a_i2 x_2 + ... (stored order)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_csr_spmv(int32_t n, const int32_t* __restrict__ slice_ptr,
                                                     const int32_t* __restrict__ col, const T* __restrict__ val,
                                                     const T* __restrict__ x, T* __restrict__ y) {
  const int32_t q = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (q >= n) return;
  const int32_t slice = q >> 6, lane = q & 63;
  T s = (T)0;
  const int32_t t0 = slice_ptr[slice], t1 = slice_ptr[slice + 1];
  for (int32_t t = t0; t < t1; ++t) {
    const int64_t e = (int64_t)t * kWave + lane;
    const int32_t c = col[e];
    if (c < 0) break;
    s = s + val[e] * x[c];
  }
  y[q] = s;
}

template <typename T>
void launch_csr_spmv(const SellView<T>& A, const T* x, T* y, hipStream_t s) {
  if (A.n_rows == 0) return;
  hipLaunchKernelGGL((k_csr_spmv<T>), dim3(div_up(A.n_rows, kBlock)), dim3(kBlock), 0, s, A.n_rows, A.slice_ptr,
                     A.col, A.val, x, y);
  CPR_LAUNCH_CHECK();
}
template void launch_csr_spmv<double>(const SellView<double>&, const double*, double*, hipStream_t);
template void launch_csr_spmv<float>(const SellView<float>&, const float*, float*, hipStream_t);

// x_i = x_i + (0 + p_i1 e_1 + ...); snap_i = x_i
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_add(int32_t n, const int32_t* __restrict__ slice_ptr,
                                                        const int32_t* __restrict__ col, const T* __restrict__ val,
                                                        const T* __restrict__ e, T* __restrict__ x,
                                                        T* __restrict__ snap) {
  const int32_t q = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (q >= n) return;
  const int32_t slice = q >> 6, lane = q & 63;
  T s = (T)0;
  const int32_t t0 = slice_ptr[slice], t1 = slice_ptr[slice + 1];
  for (int32_t t = t0; t < t1; ++t) {
    const int64_t k = (int64_t)t * kWave + lane;
    const int32_t c = col[k];
    if (c < 0) break;
    s = s + val[k] * e[c];
  }
  const T xn = x[q] + s;
  x[q] = xn;
  snap[q] = xn;
}

template <typename T>
void launch_prolong_add(const SellView<T>& P, const T* e, T* x, T* snap, hipStream_t s) {
  if (P.n_rows == 0) return;
  hipLaunchKernelGGL((k_prolong_add<T>), dim3(div_up(P.n_rows, kBlock)), dim3(kBlock), 0, s, P.n_rows, P.slice_ptr,
                     P.col, P.val, e, x, snap);
  CPR_LAUNCH_CHECK();
}
template void launch_prolong_add<double>(const SellView<double>&, const double*, double*, double*, hipStream_t);
template void launch_prolong_add<float>(const SellView<float>&, const float*, float*, float*, hipStream_t);

// Dense LU solve in one workgroup (FP64): P A = L U with the row swaps applied
// to b in factorisation order, unit-lower forward and upper back substitution.
template <typename T>
__global__ __launch_bounds__(1024) void k_coarse_solve(int32_t n, const double* __restrict__ lu,
                                                       const int32_t* __restrict__ piv, const T* __restrict__ b,
                                                       T* __restrict__ x) {
  extern __shared__ double xs[];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < n; i += nt) xs[i] = (double)b[i];
  __syncthreads();
  if (tid == 0)
    for (int k = 0; k < n; ++k) {
      const int p = piv[k];
      if (p != k) {
        const double t = xs[k];
        xs[k] = xs[p];
        xs[p] = t;
      }
    }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double xk = xs[k];
    for (int r = k + 1 + tid; r < n; r += nt) xs[r] = xs[r] - lu[(int64_t)r * n + k] * xk;
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    if (tid == 0) xs[k] = xs[k] / lu[(int64_t)k * n + k];
    __syncthreads();
    const double xk = xs[k];
    for (int r = tid; r < k; r += nt) xs[r] = xs[r] - lu[(int64_t)r * n + k] * xk;
    __syncthreads();
  }
  for (int i = tid; i < n; i += nt) x[i] = (T)xs[i];
}

template <typename T>
void launch_coarse_solve(int32_t n, const double* lu, const int32_t* piv, const T* b, T* x, hipStream_t s) {
  if (n == 0) return;
  const int threads = n >= 256 ? 1024 : 256;
  hipLaunchKernelGGL((k_coarse_solve<T>), dim3(1), dim3(threads), n * sizeof(double), s, n, lu, piv, b, x);
  CPR_LAUNCH_CHECK();
}
template void launch_coarse_solve<double>(int32_t, const double*, const int32_t*, const double*, double*,
                                          hipStream_t);
template void launch_coarse_solve<float>(int32_t, const double*, const int32_t*, const float*, float*, hipStream_t);

}  // namespace cpr
