// The coarse end of the pressure V-cycle in one workgroup.
//
// On the small coarse levels every kernel of the V-cycle is bound by launch
// and memory latency, not bandwidth: a colour of a level with a few thousand
// rows moves well under a megabyte.  This kernel runs the whole V-cycle of
// the levels [first, last] — PGS-SCM pre-sweeps, residual, restriction,
// the dense coarsest LU solve, prolongation and post-sweeps — inside one
// workgroup of 1024 threads, with a workgroup barrier between dependent
// phases instead of a kernel boundary.  The arithmetic is exactly that of the
// per-colour kernels: each row is summed by a 16-lane group in stored order
// (the running value carried lane to lane by DPP moves), so the results are
// bit-identical to theirs.
#include "kernels_common.hpp"

namespace cpr {

constexpr int kTailThreads = 1024;
constexpr int kTailGroup = 16;
constexpr int kTailRows = kTailThreads / kTailGroup;
constexpr int kTailChunks = 4;  // chunks of a row whose loads are issued together

static_assert(kTailGroup == 16, "the ordered row sums use one DPP row per group");
constexpr int kTailLast = kTailGroup - 1;  // lane that ends with a row's sum

// One colour of a sweep over rows [lo, hi) (see k_gs_grp for the semantics).
template <typename T>
__device__ void tail_colour(const TailLevel<T>& L, int32_t lo, int32_t hi, const T* s_in, T* s_out, bool zero) {
  const int lane = threadIdx.x % kTailGroup;
  for (int32_t q = lo + (int32_t)threadIdx.x / kTailGroup; q < hi; q += kTailRows) {
    T s = L.b[q];
    const int32_t p0 = L.a_rp[q], p1 = L.a_rp[q + 1];
    for (int32_t p = p0; p < p1; p += kTailGroup * kTailChunks) {
      int32_t c[kTailChunks];
      T a[kTailChunks], prod[kTailChunks];
#pragma unroll
      for (int u = 0; u < kTailChunks; ++u) {
        const int32_t e = p + u * kTailGroup + lane;
        c[u] = (e < p1) ? L.a_col[e] : -1;
        a[u] = (e < p1) ? L.a_val[e] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < kTailChunks; ++u) {
        const bool use = c[u] >= 0 && c[u] != q && (!zero || c[u] < lo);
        T xv = (T)0;
        if (use) xv = zero ? L.x[c[u]] : ((c[u] >= lo && c[u] < hi) ? s_in[c[u]] : L.x[c[u]]);
        prod[u] = use ? a[u] * xv : (T)0;
      }
      const int nch = min(kTailChunks, (p1 - p + kTailGroup - 1) / kTailGroup);
#pragma unroll
      for (int u = 0; u < kTailChunks; ++u)
        if (u < nch) s = row_chain_sub<T>(s, prod[u], lane);
    }
    if (lane == kTailLast) {
      const T xn = s / L.diag[q];
      L.x[q] = xn;
      s_out[q] = xn;
    }
  }
}

// MODE 0: y = b - A x;  MODE 1: y = A x;  MODE 2: y += A x and snap = y.
template <typename T, int MODE>
__device__ void tail_rows(int32_t n, const int32_t* rp, const int32_t* col, const T* val, const T* b, const T* x,
                          T* y, T* snap) {
  const int lane = threadIdx.x % kTailGroup;
  for (int32_t q = (int32_t)threadIdx.x / kTailGroup; q < n; q += kTailRows) {
    T acc = (MODE == 0) ? b[q] : (T)0;
    const int32_t p0 = rp[q], p1 = rp[q + 1];
    for (int32_t p = p0; p < p1; p += kTailGroup * kTailChunks) {
      int32_t c[kTailChunks];
      T a[kTailChunks], prod[kTailChunks];
#pragma unroll
      for (int u = 0; u < kTailChunks; ++u) {
        const int32_t e = p + u * kTailGroup + lane;
        c[u] = (e < p1) ? col[e] : -1;
        a[u] = (e < p1) ? val[e] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < kTailChunks; ++u) prod[u] = (c[u] >= 0) ? a[u] * x[c[u]] : (T)0;
      const int nch = min(kTailChunks, (p1 - p + kTailGroup - 1) / kTailGroup);
#pragma unroll
      for (int u = 0; u < kTailChunks; ++u)
        if (u < nch) acc = row_chain_sub<T>(acc, MODE == 0 ? prod[u] : -prod[u], lane);
    }
    if (lane == kTailLast) {
      if (MODE == 2) {
        const T yn = y[q] + acc;
        y[q] = yn;
        snap[q] = yn;
      } else {
        y[q] = acc;
      }
    }
  }
}

template <typename T>
__device__ void tail_sweep(const TailLevel<T>& L, int& cur, bool zero) {
  T* S[2] = {L.s0, L.s1};
  for (int c = 0; c < L.ncol; ++c) {
    tail_colour<T>(L, L.coff[c], L.coff[c + 1], S[cur], S[cur ^ 1], zero);
    __syncthreads();
  }
  cur ^= 1;
}

template <typename T>
__global__ __launch_bounds__(kTailThreads) void k_tail_vcycle(const TailLevel<T>* __restrict__ levels, int nlev,
                                                               int pre, int post, int32_t n_coarse,
                                                               const double* __restrict__ lu,
                                                               const int32_t* __restrict__ rperm) {
  extern __shared__ double xs[];
  // Snapshot bookkeeping: every sweep reads S[cur] and writes S[cur ^ 1], so
  // after the pre-sweeps S[pre & 1] equals x on every level.
  // down: smoothing from zero, residual, restriction
  for (int l = 0; l + 1 < nlev; ++l) {
    const TailLevel<T>& L = levels[l];
    int cur = 0;
    if (pre == 0) {
      for (int32_t q = threadIdx.x; q < L.n; q += kTailThreads) L.x[q] = (T)0;
      __syncthreads();
    }
    for (int w = 0; w < pre; ++w) tail_sweep<T>(L, cur, w == 0);
    tail_rows<T, 0>(L.n, L.a_rp, L.a_col, L.a_val, L.b, L.x, L.r, nullptr);
    __syncthreads();
    const TailLevel<T>& C = levels[l + 1];
    tail_rows<T, 1>(C.n, L.r_rp, L.r_col, L.r_val, nullptr, L.r, C.b, nullptr);
    __syncthreads();
  }
  // coarsest: P A = L U in FP64.  rperm composes the row swaps of the
  // factorisation, so (P b)_i = b[rperm[i]].
  {
    const TailLevel<T>& L = levels[nlev - 1];
    const int n = n_coarse;
    if (n <= kWave) {
      // one wavefront, one row per lane, factors staged in LDS; the lanes stay
      // in lockstep, so no barrier is needed between substitution steps
      double* luS = xs + kWave;
      for (int i = threadIdx.x; i < n * n; i += kTailThreads) luS[i] = lu[i];
      __syncthreads();
      if (threadIdx.x < kWave) {
        const int r = threadIdx.x;
        double xr = r < n ? (double)L.b[rperm[r]] : 0.0;
        for (int k = 0; k < n; ++k) {
          const double xk = __shfl(xr, k, kWave);
          if (r > k && r < n) xr = xr - luS[r * n + k] * xk;
        }
        for (int k = n - 1; k >= 0; --k) {
          if (r == k) xr = xr / luS[k * n + k];
          const double xk = __shfl(xr, k, kWave);
          if (r < k) xr = xr - luS[r * n + k] * xk;
        }
        if (r < n) L.x[r] = (T)xr;
      }
      __syncthreads();
    } else {
      for (int i = threadIdx.x; i < n; i += kTailThreads) xs[i] = (double)L.b[rperm[i]];
      __syncthreads();
      for (int k = 0; k < n; ++k) {
        const double xk = xs[k];
        for (int r = k + 1 + threadIdx.x; r < n; r += kTailThreads) xs[r] = xs[r] - lu[(int64_t)r * n + k] * xk;
        __syncthreads();
      }
      for (int k = n - 1; k >= 0; --k) {
        if (threadIdx.x == 0) xs[k] = xs[k] / lu[(int64_t)k * n + k];
        __syncthreads();
        const double xk = xs[k];
        for (int r = threadIdx.x; r < k; r += kTailThreads) xs[r] = xs[r] - lu[(int64_t)r * n + k] * xk;
        __syncthreads();
      }
      for (int i = threadIdx.x; i < n; i += kTailThreads) L.x[i] = (T)xs[i];
      __syncthreads();
    }
  }
  // up: prolongation and post-smoothing
  for (int l = nlev - 2; l >= 0; --l) {
    const TailLevel<T>& L = levels[l];
    const TailLevel<T>& C = levels[l + 1];
    T* S[2] = {L.s0, L.s1};
    int cur = pre & 1;
    tail_rows<T, 2>(L.n, L.p_rp, L.p_col, L.p_val, nullptr, C.x, L.x, S[cur]);
    __syncthreads();
    for (int w = 0; w < post; ++w) tail_sweep<T>(L, cur, false);
  }
}

template <typename T>
void launch_tail_vcycle(const TailLevel<T>* levels, int nlev, int pre, int post, int32_t n_coarse, const double* lu,
                        const int32_t* rperm, hipStream_t s) {
  const size_t lds = n_coarse <= kWave ? (kWave + (size_t)n_coarse * n_coarse) * sizeof(double)
                                       : (size_t)n_coarse * sizeof(double);
  hipLaunchKernelGGL((k_tail_vcycle<T>), dim3(1), dim3(kTailThreads), lds, s, levels, nlev, pre, post, n_coarse, lu,
                     rperm);
  CPR_LAUNCH_CHECK();
}
template void launch_tail_vcycle<double>(const TailLevel<double>*, int, int, int, int32_t, const double*,
                                         const int32_t*, hipStream_t);
template void launch_tail_vcycle<float>(const TailLevel<float>*, int, int, int, int32_t, const double*,
                                        const int32_t*, hipStream_t);

}  // namespace cpr
