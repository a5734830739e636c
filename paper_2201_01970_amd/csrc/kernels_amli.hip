// Kernels of the paper's pressure solver B_P (Section 6): unsmoothed
// aggregation AMG with the nonlinear AMLI-cycle.  The coarse correction of a
// level is two steps of flexible GCR on the next level's matrix,
// preconditioned by that level's cycle:
//   z1 = B(f), w1 = A z1, alpha1 = (f, w1)/(w1, w1), r1 = f - alpha1 w1;
//   z2 = B(r1), w2 = A z2, beta = (w2, w1)/(w1, w1), z2 -= beta z1,
//   w2 -= beta w1, alpha2 = (r1, w2)/(w2, w2), e = alpha1 z1 + alpha2 z2.
// Dot products are two-stage: every workgroup of a fixed-size grid writes a
// partial sum (FP64) and the consuming kernel re-adds the partials in a fixed
// order, so results do not depend on scheduling and every workgroup derives
// the same scalar.  The coarsest level is solved with its explicit inverse,
// formed at SETUP by Gauss-Jordan elimination with partial pivoting on the
// GPU and applied as a dense FP64 matrix-vector product.
#include "kernels_common.hpp"

namespace cpr {

namespace {

constexpr int kDotGridMax = 256;

int dot_grid(int64_t n) {
  const int64_t g = (n + 4 * kBlock - 1) / (4 * kBlock);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, kDotGridMax));
}

// Sum over the workgroup in a fixed order (wave shuffles down, then the wave
// sums in order), returned to every thread.
__device__ double block_sum_bcast(double v, double* lds) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s = s + lds[w];
    lds[16] = s;
  }
  __syncthreads();
  return lds[16];
}

// Sum of part[0..G) (G <= kBlock), identical in every workgroup.
__device__ double sum_parts(const double* part, int G, double* lds) {
  const double v = (int)threadIdx.x < G ? part[threadIdx.x] : 0.0;
  return block_sum_bcast(v, lds);
}

}  // namespace

int amli_dot_grid(int64_t n) { return dot_grid(n); }

// part[b] = partial (x1, y1), part[G + b] = partial (x2, y2) of workgroup b.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dot2(int64_t n, const T* __restrict__ x1, const T* __restrict__ y1,
                                                 const T* __restrict__ x2, const T* __restrict__ y2,
                                                 double* __restrict__ part) {
  __shared__ double lds[17];
  double a = 0.0, c = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    a = a + (double)x1[i] * (double)y1[i];
    if (x2) c = c + (double)x2[i] * (double)y2[i];
  }
  const double sa = block_sum_bcast(a, lds);
  const double sc = block_sum_bcast(c, lds);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sa;
    part[gridDim.x + blockIdx.x] = sc;
  }
}

// First GCR step: d1 = (w1, w1), alpha1 = (f, w1) / d1 (0 when d1 = 0);
// z1 = x (the cycle's output), f = f - alpha1 w1 (now r1); scal = {alpha1, d1}.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gcr_step1(int64_t n, const double* __restrict__ part, int G,
                                                      const T* __restrict__ x, T* __restrict__ z1, T* __restrict__ f,
                                                      const T* __restrict__ w1, double* __restrict__ scal) {
  __shared__ double lds[17];
  const double d1 = sum_parts(part, G, lds);
  const double p = sum_parts(part + G, G, lds);
  const double alpha = d1 != 0.0 ? p / d1 : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[0] = alpha;
    scal[1] = d1;
  }
  const T a = (T)alpha;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    z1[i] = x[i];
    f[i] = f[i] - a * w1[i];
  }
}

// One GCR step only: x = alpha1 x with alpha1 = (f, w1) / (w1, w1).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gcr_single(int64_t n, const double* __restrict__ part, int G,
                                                       T* __restrict__ x) {
  __shared__ double lds[17];
  const double d1 = sum_parts(part, G, lds);
  const double p = sum_parts(part + G, G, lds);
  const T a = (T)(d1 != 0.0 ? p / d1 : 0.0);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) x[i] = a * x[i];
}

// Second step, orthogonalisation: beta = (w2, w1) / d1 (0 when d1 = 0);
// w2 -= beta w1, x (= z2) -= beta z1; then partials of (w2, w2) and (r1, w2)
// into part2.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gcr_orth(int64_t n, const double* __restrict__ part, int G,
                                                     const double* __restrict__ scal, T* __restrict__ w2,
                                                     const T* __restrict__ w1, T* __restrict__ x,
                                                     const T* __restrict__ z1, const T* __restrict__ r1,
                                                     double* __restrict__ part2) {
  __shared__ double lds[17];
  const double s21 = sum_parts(part, G, lds);
  const double d1 = scal[1];
  const T beta = (T)(d1 != 0.0 ? s21 / d1 : 0.0);
  double ww = 0.0, rw = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const T w = w2[i] - beta * w1[i];
    w2[i] = w;
    x[i] = x[i] - beta * z1[i];
    ww = ww + (double)w * (double)w;
    rw = rw + (double)r1[i] * (double)w;
  }
  const double sww = block_sum_bcast(ww, lds);
  const double srw = block_sum_bcast(rw, lds);
  if (threadIdx.x == 0) {
    part2[blockIdx.x] = sww;
    part2[gridDim.x + blockIdx.x] = srw;
  }
}

// e = alpha1 z1 + alpha2 z2 with alpha2 = (r1, w2) / (w2, w2) (0 when that
// norm or d1 is 0); written over x (= z2).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gcr_finish(int64_t n, const double* __restrict__ part2, int G,
                                                       const double* __restrict__ scal, T* __restrict__ x,
                                                       const T* __restrict__ z1) {
  __shared__ double lds[17];
  const double d2 = sum_parts(part2, G, lds);
  const double p = sum_parts(part2 + G, G, lds);
  const T a1 = (T)scal[0];
  const T a2 = (T)((d2 != 0.0 && scal[1] != 0.0) ? p / d2 : 0.0);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    T e = a1 * z1[i];
    e = e + a2 * x[i];
    x[i] = e;
  }
}

template <typename T>
void launch_gcr_dots(int64_t n, const T* x1, const T* y1, const T* x2, const T* y2, double* part, hipStream_t s) {
  hipLaunchKernelGGL((k_dot2<T>), dim3(dot_grid(n)), dim3(kBlock), 0, s, n, x1, y1, x2, y2, part);
  CPR_LAUNCH_CHECK();
}

template <typename T>
void launch_gcr_step1(int64_t n, const double* part, const T* x, T* z1, T* f, const T* w1, double* scal,
                      hipStream_t s) {
  const int G = dot_grid(n);
  hipLaunchKernelGGL((k_gcr_step1<T>), dim3(G), dim3(kBlock), 0, s, n, part, G, x, z1, f, w1, scal);
  CPR_LAUNCH_CHECK();
}

template <typename T>
void launch_gcr_single(int64_t n, const double* part, T* x, hipStream_t s) {
  const int G = dot_grid(n);
  hipLaunchKernelGGL((k_gcr_single<T>), dim3(G), dim3(kBlock), 0, s, n, part, G, x);
  CPR_LAUNCH_CHECK();
}

template <typename T>
void launch_gcr_orth(int64_t n, const double* part, const double* scal, T* w2, const T* w1, T* x, const T* z1,
                     const T* r1, double* part2, hipStream_t s) {
  const int G = dot_grid(n);
  hipLaunchKernelGGL((k_gcr_orth<T>), dim3(G), dim3(kBlock), 0, s, n, part, G, scal, w2, w1, x, z1, r1, part2);
  CPR_LAUNCH_CHECK();
}

template <typename T>
void launch_gcr_finish(int64_t n, const double* part2, const double* scal, T* x, const T* z1, hipStream_t s) {
  const int G = dot_grid(n);
  hipLaunchKernelGGL((k_gcr_finish<T>), dim3(G), dim3(kBlock), 0, s, n, part2, G, scal, x, z1);
  CPR_LAUNCH_CHECK();
}

#define CPR_GCR_INST(T)                                                                                         \
  template void launch_gcr_dots<T>(int64_t, const T*, const T*, const T*, const T*, double*, hipStream_t);     \
  template void launch_gcr_step1<T>(int64_t, const double*, const T*, T*, T*, const T*, double*, hipStream_t); \
  template void launch_gcr_single<T>(int64_t, const double*, T*, hipStream_t);                                 \
  template void launch_gcr_orth<T>(int64_t, const double*, const double*, T*, const T*, T*, const T*, const T*, \
                                   double*, hipStream_t);                                                      \
  template void launch_gcr_finish<T>(int64_t, const double*, const double*, T*, const T*, hipStream_t);
CPR_GCR_INST(double)
CPR_GCR_INST(float)
#undef CPR_GCR_INST

// ------------------------------------------------ coarsest level: dense inverse
// In-place Gauss-Jordan elimination with partial pivoting on the row-major
// n x n matrix a, step k.  Column k of the matrix before step k is kept
// contiguous in cur[0..n) (written by the previous step, so the pivot search
// reads it without striding through a).  Pivot search, row swap and the
// scaling of the pivot row run in one workgroup; the elimination of the other
// rows in a second kernel, which also leaves column k+1 in nxt.  After step k,
// row k holds (row k)/pivot with entry k = 1/pivot, and every other row i has
// had m_i (its old entry k) times the new row k subtracted, entry k becoming
// -m_i/pivot.
constexpr int kGjBlock = 1024;

__global__ __launch_bounds__(kBlock) void k_gj_column(int n, const double* __restrict__ a, double* __restrict__ col) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) col[i] = a[(int64_t)i * n];
}

__global__ __launch_bounds__(kGjBlock) void k_gj_pivot(int n, int k, double* __restrict__ a, int32_t* __restrict__ piv,
                                                       double* __restrict__ cur, double* __restrict__ nxt,
                                                       int32_t* __restrict__ bad) {
  __shared__ double sv[kGjBlock];
  __shared__ int si[kGjBlock];
  double best = -1.0;
  int bi = n;
  for (int i = k + (int)threadIdx.x; i < n; i += kGjBlock) {
    const double v = fabs(cur[i]);
    if (v > best) {  // rows visited in ascending order: ties keep the smallest index
      best = v;
      bi = i;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int w = kGjBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double ov = sv[threadIdx.x + w];
      const int oi = si[threadIdx.x + w];
      if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
        sv[threadIdx.x] = ov;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const int p = si[0];
  const bool ok = p < n && sv[0] > 0.0;
  if (p < n && p != k) {
    for (int j = threadIdx.x; j < n; j += kGjBlock) {
      const double t = a[(int64_t)k * n + j];
      a[(int64_t)k * n + j] = a[(int64_t)p * n + j];
      a[(int64_t)p * n + j] = t;
    }
    if (threadIdx.x == 0) {
      const double t = cur[k];
      cur[k] = cur[p];
      cur[p] = t;
    }
  }
  __syncthreads();
  const double pv = ok ? a[(int64_t)k * n + k] : 1.0;
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += kGjBlock) {
    const double v = j == k ? 1.0 : a[(int64_t)k * n + j];
    const double r = v / pv;
    a[(int64_t)k * n + j] = r;
    if (j == k + 1) nxt[k] = r;
  }
  if (threadIdx.x == 0) {
    piv[k] = ok ? p : k;
    if (!ok) bad[0] = 1;
  }
}

__global__ __launch_bounds__(kBlock) void k_gj_eliminate(int n, int k, double* __restrict__ a,
                                                         const double* __restrict__ cur, double* __restrict__ nxt) {
  const int i = blockIdx.x;
  if (i == k) return;
  const double f = cur[i];
  double* row = a + (int64_t)i * n;
  // a zero multiplier leaves the row as it is (the coarsest Galerkin matrix
  // is sparse, so most rows of the early steps have nothing to eliminate)
  if (f == 0.0) {
    if (threadIdx.x == 0 && k + 1 < n) nxt[i] = row[k + 1];
    return;
  }
  const double* rk = a + (int64_t)k * n;
  for (int j = threadIdx.x; j < n; j += kBlock) {
    const double v = j == k ? 0.0 : row[j];
    const double prod = f * rk[j];
    const double r = v - prod;
    row[j] = r;
    if (j == k + 1) nxt[i] = r;
  }
}

// dst[i][j] = src[i][cols[j]]
__global__ __launch_bounds__(kBlock) void k_permute_cols(int n, const double* __restrict__ src,
                                                         const int32_t* __restrict__ cols, double* __restrict__ dst) {
  const int i = blockIdx.x;
  for (int j = threadIdx.x; j < n; j += kBlock) dst[(int64_t)i * n + j] = src[(int64_t)i * n + cols[j]];
}

void launch_gj_step(int n, int k, double* a, int32_t* piv, double* col2, int32_t* bad, hipStream_t s) {
  double* cur = col2 + (int64_t)(k & 1) * n;
  double* nxt = col2 + (int64_t)((k + 1) & 1) * n;
  if (k == 0) {
    hipLaunchKernelGGL(k_gj_column, dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, n, a, cur);
    CPR_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(kGjBlock), 0, s, n, k, a, piv, cur, nxt, bad);
  CPR_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gj_eliminate, dim3(n), dim3(kBlock), 0, s, n, k, a, cur, nxt);
  CPR_LAUNCH_CHECK();
}

void launch_permute_cols(int n, const double* src, const int32_t* cols, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_permute_cols, dim3(n), dim3(kBlock), 0, s, n, src, cols, dst);
  CPR_LAUNCH_CHECK();
}

// x = Ainv b: one wavefront per row.  Lane l sums the FP64 products of
// columns l + 64 k into four accumulators by k mod 4 (four independent loads
// in flight per lane), which are added in a fixed order and then across the
// lanes in a fixed order, so the result does not depend on the launch.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_gemv(int n, const double* __restrict__ ainv,
                                                       const T* __restrict__ b, T* __restrict__ x) {
  const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const double* r = ainv + (int64_t)row * n;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int j = lane;
  for (; j + 192 < n; j += 256) {
    a0 = a0 + r[j] * (double)b[j];
    a1 = a1 + r[j + 64] * (double)b[j + 64];
    a2 = a2 + r[j + 128] * (double)b[j + 128];
    a3 = a3 + r[j + 192] * (double)b[j + 192];
  }
  if (j < n) a0 = a0 + r[j] * (double)b[j];
  if (j + 64 < n) a1 = a1 + r[j + 64] * (double)b[j + 64];
  if (j + 128 < n) a2 = a2 + r[j + 128] * (double)b[j + 128];
  double acc = (a0 + a1) + (a2 + a3);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) x[row] = (T)acc;
}

template <typename T>
void launch_dense_gemv(int n, const double* ainv, const T* b, T* x, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_dense_gemv<T>), dim3(div_up(n, kBlock / 64)), dim3(kBlock), 0, s, n, ainv, b, x);
  CPR_LAUNCH_CHECK();
}
template void launch_dense_gemv<double>(int, const double*, const double*, double*, hipStream_t);
template void launch_dense_gemv<float>(int, const double*, const float*, float*, hipStream_t);

}  // namespace cpr
