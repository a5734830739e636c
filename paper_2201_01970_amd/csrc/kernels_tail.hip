// The coarse end of the pressure V-cycle in one workgroup.
//
// On the small coarse levels every per-colour kernel is bound by launch and
// memory latency, not bandwidth: a colour of a level with a few hundred rows
// moves a few hundred kilobytes.  This kernel runs the whole V-cycle of the
// levels [first, last] — PGS-SCM pre-sweeps, residual, restriction, the dense
// coarsest LU solve, prolongation and post-sweeps — inside one workgroup of
// 1024 threads, with a workgroup barrier between dependent phases instead of a
// kernel boundary.  Every vector of these levels stays in LDS for the whole
// kernel, so a phase's gathers and writes never leave the compute unit; the
// matrices are read from device memory (they stay in L2 across the sweeps).
//
// Rows are taken by quads in the quad-vector CSR layout (256 rows per pass;
// see quad_row_sub): every row sum is accumulated in stored order and rounded
// exactly as a sequential loop rounds it, so the results are bit-identical to
// those of the per-colour kernels.  Matrix pointers come from a descriptor in
// memory and are read through gmem (global loads); the level vectors are LDS.
#include "kernels_common.hpp"

namespace cpr {

constexpr int kTailThreads = 1024;
constexpr int kTailRows = kTailThreads / 4;  // rows per pass
// chunks of 16 entries a quad requests at once (fewer in FP64: a 1024-thread
// workgroup leaves 128 registers per lane)
template <typename T>
constexpr int tail_chunks() {
  return sizeof(T) == 4 ? 8 : 4;
}

// One colour [lo, hi) of a sweep (semantics of k_gs_grp).
template <typename T>
__device__ __forceinline__ void tail_colour(const TailLevel<T>& L, T* V, int32_t lo, int32_t hi, const T* s_in,
                                            T* s_out, bool zero) {
  const int lane = threadIdx.x & 3;
  T* x = V + L.off_x;
  const T* b = V + L.off_b;
  const auto rp = gmem(L.a_rp);
  const auto col = gmem(L.a_col);
  const auto val = gmem(L.a_val);
  for (int32_t q = lo + (int32_t)(threadIdx.x >> 2); q < hi; q += kTailRows) {
    const T d = gmem(L.diag)[q];  // requested with the row pointers, off the dependent chain
    // branch-free gather: an entry that does not contribute reads row q's own
    // value and its product is replaced by 0
    const T s = quad_row_sub<T, tail_chunks<T>()>(b[q], rp[q], rp[q + 1], col, val, lane, [&](int32_t c, T a) {
      const bool use = c >= 0 && c != q && (!zero || c < lo);
      const int32_t cc = use ? c : q;
      const T* src = (!zero && cc >= lo && cc < hi) ? s_in : x;
      const T xv = src[cc];
      return use ? a * xv : (T)0;
    });
    if (lane == 3) {
      const T xn = s / d;
      x[q] = xn;
      s_out[q] = xn;
    }
  }
}

// MODE 0: y = b - A x;  MODE 1: y = A x;  MODE 2: y += A x and snap = y.
// b, x, y, snap are LDS arrays; the matrix is in device memory.
template <typename T, int MODE>
__device__ __forceinline__ void tail_rows(int32_t n, const int32_t* rp_, const int32_t* col_, const T* val_,
                                          const T* b, const T* x, T* y, T* snap) {
  const int lane = threadIdx.x & 3;
  const auto rp = gmem(rp_);
  const auto col = gmem(col_);
  const auto val = gmem(val_);
  for (int32_t q = (int32_t)(threadIdx.x >> 2); q < n; q += kTailRows) {
    const T y0 = (MODE == 2) ? y[q] : (T)0;
    // addition runs as subtraction of the negated products (the same IEEE operation)
    const T acc = quad_row_sub<T, tail_chunks<T>()>((MODE == 0) ? b[q] : (T)0, rp[q], rp[q + 1], col, val, lane,
                                               [&](int32_t c, T a) {
                                                 const T xv = x[c < 0 ? 0 : c];
                                                 const T pr = (c >= 0) ? a * xv : (T)0;
                                                 return MODE == 0 ? pr : -pr;
                                               });
    if (lane == 3) {
      if (MODE == 2) {
        const T yn = y0 + acc;
        y[q] = yn;
        snap[q] = yn;
      } else {
        y[q] = acc;
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void tail_sweep(const TailLevel<T>& L, T* V, int& cur, bool zero) {
  // snapshots selected by value (an indexed pointer array would live in scratch)
  T* s_in = cur ? V + L.off_s1 : V + L.off_s0;
  T* s_out = cur ? V + L.off_s0 : V + L.off_s1;
  const auto coff = gmem(L.coff);
  for (int c = 0; c < L.ncol; ++c) {
    tail_colour<T>(L, V, coff[c], coff[c + 1], s_in, s_out, zero);
    __syncthreads();
  }
  cur ^= 1;
}

template <typename T>
__global__ __launch_bounds__(kTailThreads) void k_tail_vcycle(const TailLevel<T>* __restrict__ levels, int nlev,
                                                               int pre, int post, int32_t n_coarse,
                                                               const double* __restrict__ lu,
                                                               const int32_t* __restrict__ rperm) {
  extern __shared__ double lds[];
  double* xs = lds;                                          // coarsest-solve staging
  T* V = reinterpret_cast<T*>(lds + tail_lds_doubles(n_coarse));  // level vectors
  {
    const TailLevel<T>& F = levels[0];
    for (int32_t i = threadIdx.x; i < F.n; i += kTailThreads) V[F.off_b + i] = gmem(F.gb)[i];
    __syncthreads();
  }
  // Snapshot bookkeeping: every sweep reads S[cur] and writes S[cur ^ 1], so
  // after the pre-sweeps S[pre & 1] equals x on every level.
  // down: smoothing from zero, residual, restriction
  for (int l = 0; l + 1 < nlev; ++l) {
    const TailLevel<T>& L = levels[l];
    int cur = 0;
    if (pre == 0) {
      for (int32_t q = threadIdx.x; q < L.n; q += kTailThreads) V[L.off_x + q] = (T)0;
      __syncthreads();
    }
    for (int w = 0; w < pre; ++w) tail_sweep<T>(L, V, cur, w == 0);
    tail_rows<T, 0>(L.n, L.a_rp, L.a_col, L.a_val, V + L.off_b, V + L.off_x, V + L.off_r, nullptr);
    __syncthreads();
    const TailLevel<T>& C = levels[l + 1];
    tail_rows<T, 1>(C.n, L.r_rp, L.r_col, L.r_val, nullptr, V + L.off_r, V + C.off_b, nullptr);
    __syncthreads();
  }
  // coarsest: P A = L U in FP64.  rperm composes the row swaps of the
  // factorisation, so (P b)_i = b[rperm[i]].
  {
    const TailLevel<T>& L = levels[nlev - 1];
    const T* b = V + L.off_b;
    T* x = V + L.off_x;
    const int n = n_coarse;
    if (n <= kWave) {
      // one wavefront, one row per lane, factors staged in LDS; the lanes stay
      // in lockstep, so no barrier is needed between substitution steps
      double* luS = xs + kWave;
      for (int i = threadIdx.x; i < n * n; i += kTailThreads) luS[i] = gmem(lu)[i];
      __syncthreads();
      if (threadIdx.x < kWave) {
        const int r = threadIdx.x;
        double xr = r < n ? (double)b[gmem(rperm)[r]] : 0.0;
        for (int k = 0; k < n; ++k) {
          const double xk = __shfl(xr, k, kWave);
          if (r > k && r < n) xr = xr - luS[r * n + k] * xk;
        }
        for (int k = n - 1; k >= 0; --k) {
          if (r == k) xr = xr / luS[k * n + k];
          const double xk = __shfl(xr, k, kWave);
          if (r < k) xr = xr - luS[r * n + k] * xk;
        }
        if (r < n) x[r] = (T)xr;
      }
      __syncthreads();
    } else {
      for (int i = threadIdx.x; i < n; i += kTailThreads) xs[i] = (double)b[gmem(rperm)[i]];
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
      for (int i = threadIdx.x; i < n; i += kTailThreads) x[i] = (T)xs[i];
      __syncthreads();
    }
  }
  // up: prolongation and post-smoothing
  for (int l = nlev - 2; l >= 0; --l) {
    const TailLevel<T>& L = levels[l];
    const TailLevel<T>& C = levels[l + 1];
    int cur = pre & 1;
    tail_rows<T, 2>(L.n, L.p_rp, L.p_col, L.p_val, nullptr, V + C.off_x, V + L.off_x,
                    cur ? V + L.off_s1 : V + L.off_s0);
    __syncthreads();
    for (int w = 0; w < post; ++w) tail_sweep<T>(L, V, cur, false);
  }
  {
    const TailLevel<T>& F = levels[0];
    for (int32_t i = threadIdx.x; i < F.n; i += kTailThreads) F.gx[i] = V[F.off_x + i];
  }
}

size_t tail_lds_limit() {
  int dev = 0, bytes = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
  return static_cast<size_t>(bytes);
}

template <typename T>
void launch_tail_vcycle(const TailLevel<T>* levels, int nlev, int pre, int post, int32_t n_coarse, const double* lu,
                        const int32_t* rperm, size_t lds_bytes, hipStream_t s) {
  hipLaunchKernelGGL((k_tail_vcycle<T>), dim3(1), dim3(kTailThreads), lds_bytes, s, levels, nlev, pre, post, n_coarse,
                     lu, rperm);
  CPR_LAUNCH_CHECK();
}
template void launch_tail_vcycle<double>(const TailLevel<double>*, int, int, int, int32_t, const double*,
                                         const int32_t*, size_t, hipStream_t);
template void launch_tail_vcycle<float>(const TailLevel<float>*, int, int, int, int32_t, const double*,
                                        const int32_t*, size_t, hipStream_t);

}  // namespace cpr
