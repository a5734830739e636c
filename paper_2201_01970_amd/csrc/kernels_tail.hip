// The coarse end of the pressure V-cycle in one workgroup.
//
// On the small coarse levels every per-colour kernel is bound by launch and
// memory latency, not bandwidth: a colour of a level with a few hundred rows
// moves a few hundred kilobytes.  This kernel runs the whole V-cycle of the
// levels [first, last] — PGS-SCM pre-sweeps, residual, restriction, the dense
// coarsest LU solve, prolongation and post-sweeps — inside one workgroup of
// 1024 threads, with a workgroup barrier between dependent phases instead of a
// kernel boundary.  Every vector of these levels stays in LDS for the whole
// kernel, so a phase's gathers and writes never leave the compute unit.  So do
// the colour offsets, diagonals and row pointers, and the sweep matrices of as
// many levels (coarsest first) as the LDS holds, copied in with one
// vectorised pass when the kernel starts: a sweep phase of a staged level
// never waits on device memory, the other phases wait only for the columns
// and values of their rows (which stay in L2 across the sweeps).
//
// Rows are taken by quads in the quad-vector CSR layout (256 rows per pass;
// see quad_row_sub): every row sum is accumulated in stored order and rounded
// exactly as a sequential loop rounds it, so the results are bit-identical to
// those of the per-colour kernels.  Matrix pointers come from a descriptor in
// memory and are read through gmem (global loads).
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

// One colour [lo, hi) of a sweep (semantics of k_gs_grp).  Neighbour j
// contributes xt_j = x_j for j < lo (updated earlier in this sweep) and
// s_in[j] otherwise: s_in holds x as it was when the sweep started, which is
// what x still holds for the rows of this and later colours.  The sweep
// matrix points the diagonal and padding at the zero entry n with value 0, so
// every product is a * xt (+0 for those entries).  A sweep from x = 0 takes
// only j < lo.
// The sweep matrix is read through col/val: LDS pointers when it is staged,
// device memory otherwise.
template <typename T, typename ColP, typename ValP>
__device__ __forceinline__ void tail_colour(const TailLevel<T>& L, T* V, const uint32_t* S, int32_t lo, int32_t hi,
                                            const T* s_in, T* s_out, bool zero, ColP col, ValP val) {
  const int lane = threadIdx.x & 3;
  T* x = V + L.off_x;
  const T* b = V + L.off_b;
  const T* dg = reinterpret_cast<const T*>(S + L.w_diag);
  const int32_t* rp = reinterpret_cast<const int32_t*>(S + L.w_arp);
  const int32_t zs = L.n;
  for (int32_t q = lo + (int32_t)(threadIdx.x >> 2); q < hi; q += kTailRows) {
    const T d = dg[q];
    T s;
    if (zero)
      s = quad_row_sub<T, tail_chunks<T>()>(
          b[q], rp[q], rp[q + 1], col, val, lane, [&](int32_t c, T a) { return c < lo ? a * x[c] : (T)0; }, zs);
    else
      s = quad_row_sub<T, tail_chunks<T>()>(
          b[q], rp[q], rp[q + 1], col, val, lane, [&](int32_t c, T a) { return a * (c < lo ? x : s_in)[c]; }, zs);
    if (lane == 3) {
      const T xn = s / d;
      x[q] = xn;
      s_out[q] = xn;
    }
  }
}

// MODE 0: y = b - A x;  MODE 1: y = A x;  MODE 2: y += A x and snap = y.
// b, x, y, snap and the row pointers are in LDS; columns and values in device
// memory (padding: column -1).
template <typename T, int MODE>
__device__ __forceinline__ void tail_rows(int32_t n, const int32_t* rp, const int32_t* col_, const T* val_,
                                          const T* b, const T* x, T* y, T* snap) {
  const int lane = threadIdx.x & 3;
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
__device__ __forceinline__ void tail_sweep(const TailLevel<T>& L, T* V, const uint32_t* S, int& cur, bool zero) {
  // snapshots selected by value (an indexed pointer array would live in scratch)
  T* s_in = cur ? V + L.off_s1 : V + L.off_s0;
  T* s_out = cur ? V + L.off_s0 : V + L.off_s1;
  const int32_t* coff = reinterpret_cast<const int32_t*>(S + L.w_coff);
  if (L.w_wcol >= 0) {
    const int32_t* col = reinterpret_cast<const int32_t*>(S + L.w_wcol);
    const T* val = reinterpret_cast<const T*>(S + L.w_wval);
    for (int c = 0; c < L.ncol; ++c) {
      tail_colour<T>(L, V, S, coff[c], coff[c + 1], s_in, s_out, zero, col, val);
      __syncthreads();
    }
  } else {
    for (int c = 0; c < L.ncol; ++c) {
      tail_colour<T>(L, V, S, coff[c], coff[c + 1], s_in, s_out, zero, gmem(L.w_col), gmem(L.w_val));
      __syncthreads();
    }
  }
  cur ^= 1;
}

// Lane k's value broadcast to the wavefront (k wavefront-uniform): two
// v_readlane into scalar registers, no LDS round trip.
__device__ __forceinline__ double lane_value(double v, int k) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(u & 0xffffffffll), k);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(u >> 32), k);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

template <typename T>
__global__ __launch_bounds__(kTailThreads) void k_tail_vcycle(const TailLevel<T>* __restrict__ levels, int nlev,
                                                               int pre, int post, int32_t n_coarse,
                                                               const double* __restrict__ lu,
                                                               const uint32_t* __restrict__ img, TailLayout lay) {
  extern __shared__ double lds[];
  uint32_t* S = reinterpret_cast<uint32_t*>(lds);
  T* V = reinterpret_cast<T*>(S + lay.v_off);  // level vectors
  {
    // the image and the first level's b, every load of a thread requested
    // before its stores
    const TailLevel<T>& F = levels[0];
    const auto src = gmem(reinterpret_cast<const i32x4*>(img));
    const auto gb = gmem(F.gb);
    i32x4* dst = reinterpret_cast<i32x4*>(S);
    T* fb = V + F.off_b;
    const int32_t n4 = lay.img_words >> 2;  // >= 1: the image holds rperm
    const int32_t nmax = n4 > F.n ? n4 : F.n;
    constexpr int U = 8;  // 16-byte loads in flight per thread: 128 KiB per round
    for (int32_t i0 = 0; i0 < nmax; i0 += U * kTailThreads) {
      i32x4 w[U];
      T bv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // branch-free: an index past the end reads the last element again
        const int32_t i = i0 + u * kTailThreads + (int32_t)threadIdx.x;
        w[u] = src[i < n4 ? i : n4 - 1];
        bv[u] = gb[i < F.n ? i : F.n - 1];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t i = i0 + u * kTailThreads + (int32_t)threadIdx.x;
        if (i < n4) dst[i] = w[u];
        if (i < F.n) fb[i] = bv[u];
      }
    }
    // the zero entry n of x and of both snapshots of every smoothed level
    for (int l = (int)threadIdx.x; l + 1 < nlev; l += kTailThreads) {
      const TailLevel<T>& L = levels[l];
      V[L.off_x + L.n] = (T)0;
      V[L.off_s0 + L.n] = (T)0;
      V[L.off_s1 + L.n] = (T)0;
    }
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
    for (int w = 0; w < pre; ++w) tail_sweep<T>(L, V, S, cur, w == 0);
    tail_rows<T, 0>(L.n, reinterpret_cast<const int32_t*>(S + L.w_arp), L.a_col, L.a_val, V + L.off_b,
                    V + L.off_x, V + L.off_r, nullptr);
    __syncthreads();
    const TailLevel<T>& C = levels[l + 1];
    tail_rows<T, 1>(C.n, reinterpret_cast<const int32_t*>(S + L.w_rrp), L.r_col, L.r_val, nullptr, V + L.off_r,
                    V + C.off_b, nullptr);
    __syncthreads();
  }
  // coarsest: P A = L U in FP64.  rperm composes the row swaps of the
  // factorisation, so (P b)_i = b[rperm[i]].
  {
    const TailLevel<T>& L = levels[nlev - 1];
    const T* b = V + L.off_b;
    T* x = V + L.off_x;
    const int32_t* rperm = reinterpret_cast<const int32_t*>(S + lay.w_rperm);
    const int n = n_coarse;
    if (n <= kWave) {
      // one wavefront, one row per lane, factors in the LDS image; the lanes
      // stay in lockstep, so no barrier is needed between substitution steps
      const double* luS = reinterpret_cast<const double*>(S);
      if (threadIdx.x < kWave) {
        const int r = threadIdx.x;
        double xr = r < n ? (double)b[rperm[r]] : 0.0;
        for (int k = 0; k < n; ++k) {
          const double xk = lane_value(xr, k);
          if (r > k && r < n) xr = xr - luS[r * n + k] * xk;
        }
        for (int k = n - 1; k >= 0; --k) {
          if (r == k) xr = xr / luS[k * n + k];
          const double xk = lane_value(xr, k);
          if (r < k) xr = xr - luS[r * n + k] * xk;
        }
        if (r < n) x[r] = (T)xr;
      }
      __syncthreads();
    } else {
      double* xs = reinterpret_cast<double*>(S + lay.xs_off);
      for (int i = threadIdx.x; i < n; i += kTailThreads) xs[i] = (double)b[rperm[i]];
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
    tail_rows<T, 2>(L.n, reinterpret_cast<const int32_t*>(S + L.w_prp), L.p_col, L.p_val, nullptr, V + C.off_x,
                    V + L.off_x, cur ? V + L.off_s1 : V + L.off_s0);
    __syncthreads();
    for (int w = 0; w < post; ++w) tail_sweep<T>(L, V, S, cur, false);
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
                        const uint32_t* img, const TailLayout& lay, hipStream_t s) {
  hipLaunchKernelGGL((k_tail_vcycle<T>), dim3(1), dim3(kTailThreads), lay.lds_bytes, s, levels, nlev, pre, post,
                     n_coarse, lu, img, lay);
  CPR_LAUNCH_CHECK();
}
template void launch_tail_vcycle<double>(const TailLevel<double>*, int, int, int, int32_t, const double*,
                                         const uint32_t*, const TailLayout&, hipStream_t);
template void launch_tail_vcycle<float>(const TailLevel<float>*, int, int, int, int32_t, const double*,
                                        const uint32_t*, const TailLayout&, hipStream_t);

}  // namespace cpr
