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
// n x n matrix a.  Step k: p = the row >= k of largest |a[p][k]| (ties to the
// smaller row), rows k and p interchanged, row k divided by the pivot with
// entry k becoming 1/pivot, and every other row i losing m_i (its entry k)
// times the new row k, its entry k becoming -m_i/pivot.  A step changes
// column j using only columns j and k, so the steps of a panel of kb columns
// [k0, k0 + kb) run on a copy of those columns alone (every row), and their
// effect on every other column j is, with the panel's row interchanges
// applied first,
//   a[i][j] = (k0 <= i < k0 + kb ? 0 : a[i][j]) + sum_t X[i][t] Y[t][j],
// X the eliminated panel and Y rows k0..k0+kb-1 before the update: one
// rank-kb update of the matrix per panel instead of a full pass per column.
constexpr int kGjPanel = 64;                 // columns per panel, one per lane
constexpr int kGjRows = 64;                  // rows per workgroup of a column step
constexpr int kGjThreads = 1024;             // 16 wavefronts of four rows each
constexpr int kGjWaves = kGjThreads / 64;
constexpr int kGjSwapThreads = 64;
constexpr int kGjTile = 64;                  // update tile: 64 x 64 entries, 256 threads

// (v, i) ranks above (bv, bi): larger magnitude, ties to the smaller row
__device__ __forceinline__ bool gj_better(double v, int i, double bv, int bi) {
  return v > bv || (v == bv && i < bi);
}

// The workgroup's pivot candidate from the one held by lane `owner` of every
// wavefront, stored at cv[blockIdx.x], ci[blockIdx.x].
__device__ void gj_block_candidate(double v, int i, int owner, double* cv, int32_t* ci) {
  __shared__ double sv[kGjWaves];
  __shared__ int si[kGjWaves];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == owner) {
    sv[wave] = v;
    si[wave] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bv = sv[0];
    int bi = si[0];
    for (int w = 1; w < kGjWaves; ++w)
      if (gj_better(sv[w], si[w], bv, bi)) {
        bv = sv[w];
        bi = si[w];
      }
    cv[blockIdx.x] = bv;
    ci[blockIdx.x] = bi;
  }
}

// pan (n x kGjPanel, row-major) = columns k0..k0+kb-1 of a, zero beyond kb;
// the candidates for the pivot of column k0.
__global__ __launch_bounds__(kGjThreads) void k_gj_panel_load(int n, int k0, int kb, const double* __restrict__ a,
                                                              double* __restrict__ pan, double* __restrict__ cv,
                                                              int32_t* __restrict__ ci) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double bv = -1.0;
  int bi = n;
  for (int m = 0; m < kGjRows / kGjWaves; ++m) {
    const int i = blockIdx.x * kGjRows + wave + kGjWaves * m;
    if (i >= n) break;
    const double v = lane < kb ? a[(int64_t)i * n + k0 + lane] : 0.0;
    pan[(int64_t)i * kGjPanel + lane] = v;
    if (lane == 0 && i >= k0 && fabs(v) > bv) {
      bv = fabs(v);
      bi = i;
    }
  }
  gj_block_candidate(bv, bi, 0, cv, ci);
}

// Step k = k0 + t on the panel: src -> dst.  Every workgroup reduces the
// candidates of the previous launch to the same pivot row, and leaves its
// candidate for column t + 1 (rows > k).  Lane j holds panel column j; the
// wavefront of a row is uniform, so the shuffles see every lane.
__global__ __launch_bounds__(kGjThreads) void k_gj_panel_step(int n, int k0, int kb, int t, int nwg,
                                                              const double* __restrict__ src, double* __restrict__ dst,
                                                              const double* __restrict__ cv_in,
                                                              const int32_t* __restrict__ ci_in,
                                                              double* __restrict__ cv_out, int32_t* __restrict__ ci_out,
                                                              int32_t* __restrict__ piv, int32_t* __restrict__ bad) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int k = k0 + t;
  constexpr int kM = kGjRows / kGjWaves;
  double rv[kM];  // this workgroup's rows, requested before the pivot is known
#pragma unroll
  for (int m = 0; m < kM; ++m) {
    const int i = blockIdx.x * kGjRows + wave + kGjWaves * m;
    rv[m] = i < n ? src[(int64_t)i * kGjPanel + lane] : 0.0;
  }
  double bv = -1.0;
  int bi = n;
  for (int w = lane; w < nwg; w += 64)
    if (gj_better(cv_in[w], ci_in[w], bv, bi)) {
      bv = cv_in[w];
      bi = ci_in[w];
    }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(bv, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (gj_better(ov, oi, bv, bi)) {
      bv = ov;
      bi = oi;
    }
  }
  const bool ok = bi < n && bv > 0.0;
  const int p = ok ? bi : k;
  const double rk = src[(int64_t)k * kGjPanel + lane];
  const double rp = p == k ? rk : src[(int64_t)p * kGjPanel + lane];
  const double pv = ok ? __shfl(rp, t, 64) : 1.0;
  const double sp = (lane == t ? 1.0 : rp) / pv;  // the new row k
  double cbv = -1.0;
  int cbi = n;
#pragma unroll
  for (int m = 0; m < kM; ++m) {
    const int i = blockIdx.x * kGjRows + wave + kGjWaves * m;
    if (i < n) {
      double out;
      if (i == k) {
        out = sp;
      } else {
        const double v = i == p ? rk : rv[m];
        const double f = __shfl(v, t, 64);
        const double prod = f * sp;
        out = (lane == t ? 0.0 : v) - prod;
      }
      dst[(int64_t)i * kGjPanel + lane] = out;
      if (lane == t + 1 && i > k && fabs(out) > cbv) {
        cbv = fabs(out);
        cbi = i;
      }
    }
  }
  if (t + 1 < kb) gj_block_candidate(cbv, cbi, t + 1, cv_out, ci_out);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    piv[k] = p;
    if (!ok) bad[0] = 1;
  }
}

// The panel's row interchanges, in step order, on every column outside the
// panel (one thread per column): rows k0..k0+kb-1 leave their values in y
// (row t of y is row k0 + t) and hold zero.  The interchanges move at most
// 2 kb rows; the first thread lists them (pos: row, org: the row its value
// comes from).
__global__ __launch_bounds__(kGjSwapThreads) void k_gj_panel_swap(int n, int k0, int kb, double* __restrict__ a,
                                                                  const int32_t* __restrict__ piv,
                                                                  double* __restrict__ y) {
  __shared__ int pos[2 * kGjPanel], org[2 * kGjPanel];
  __shared__ int cnt;
  __shared__ double vals[2 * kGjPanel][kGjSwapThreads];
  if (threadIdx.x == 0) {
    int c = kb;
    for (int t = 0; t < kb; ++t) {
      pos[t] = k0 + t;
      org[t] = k0 + t;
    }
    for (int t = 0; t < kb; ++t) {
      const int p = piv[k0 + t];
      if (p == k0 + t) continue;
      int m = -1;
      for (int q = t + 1; q < c; ++q)
        if (pos[q] == p) {
          m = q;
          break;
        }
      if (m < 0) {
        m = c++;
        pos[m] = p;
        org[m] = p;
      }
      const int o = org[t];
      org[t] = org[m];
      org[m] = o;
    }
    cnt = c;
  }
  __syncthreads();
  const int j = blockIdx.x * kGjSwapThreads + threadIdx.x;
  if (j >= n || (j >= k0 && j < k0 + kb)) return;
  const int c = cnt;
  for (int m = 0; m < c; ++m) vals[m][threadIdx.x] = a[(int64_t)org[m] * n + j];
  for (int m = 0; m < c; ++m) {
    const double v = vals[m][threadIdx.x];
    if (m < kb) {
      y[(int64_t)m * n + j] = v;
      a[(int64_t)pos[m] * n + j] = 0.0;
    } else {
      a[(int64_t)pos[m] * n + j] = v;
    }
  }
}

// a[i][j] += sum_t x[i][t] y[t][j] outside the panel's columns, which take x.
// 64 x 64 tiles; thread (ty, tx) owns rows 4 ty + r and columns tx + 16 c.
__global__ __launch_bounds__(256) void k_gj_panel_update(int n, int k0, int kb, double* __restrict__ a,
                                                         const double* __restrict__ x, const double* __restrict__ y) {
  __shared__ double xs[kGjTile][kGjPanel + 1];
  __shared__ double ys[kGjPanel][kGjTile];
  const int i0 = blockIdx.y * kGjTile, j0 = blockIdx.x * kGjTile;
  if (j0 == k0) {  // panels start on tile boundaries
    for (int e = threadIdx.x; e < kGjTile * kGjPanel; e += 256) {
      const int r = e / kGjPanel, t = e % kGjPanel;
      if (i0 + r < n && t < kb) a[(int64_t)(i0 + r) * n + k0 + t] = x[(int64_t)(i0 + r) * kGjPanel + t];
    }
    return;
  }
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = i0 + 4 * ty + r, j = j0 + tx + 16 * c;
      acc[r][c] = (i < n && j < n) ? a[(int64_t)i * n + j] : 0.0;
    }
  for (int e = threadIdx.x; e < kGjTile * kGjPanel; e += 256) {
    const int r = e / kGjPanel, t = e % kGjPanel;
    xs[r][t] = i0 + r < n ? x[(int64_t)(i0 + r) * kGjPanel + t] : 0.0;
  }
  for (int e = threadIdx.x; e < kGjPanel * kGjTile; e += 256) {
    const int t = e / kGjTile, c = e % kGjTile;
    ys[t][c] = (t < kb && j0 + c < n) ? y[(int64_t)t * n + j0 + c] : 0.0;
  }
  __syncthreads();
  for (int t = 0; t < kb; ++t) {
    double xr[4], yc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) xr[r] = xs[4 * ty + r][t];
#pragma unroll
    for (int c = 0; c < 4; ++c) yc[c] = ys[t][tx + 16 * c];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] = fma(xr[r], yc[c], acc[r][c]);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = i0 + 4 * ty + r, j = j0 + tx + 16 * c;
      if (i < n && j < n) a[(int64_t)i * n + j] = acc[r][c];
    }
}

int64_t gj_workspace_doubles(int n) {
  const int64_t nwg = div_up(n, kGjRows);
  return 2 * (int64_t)n * kGjPanel + (int64_t)kGjPanel * n + 2 * nwg;
}

int64_t gj_workspace_ints(int n) { return 2 * (int64_t)div_up(n, kGjRows); }

void launch_gj_inverse(int n, double* a, double* work, int32_t* iwork, int32_t* piv, int32_t* bad, hipStream_t s) {
  const int nwg = div_up(n, kGjRows);
  double* pan[2] = {work, work + (int64_t)n * kGjPanel};
  double* y = work + 2 * (int64_t)n * kGjPanel;
  double* cv[2] = {y + (int64_t)kGjPanel * n, y + (int64_t)kGjPanel * n + nwg};
  int32_t* ci[2] = {iwork, iwork + nwg};
  const int tiles = div_up(n, kGjTile);
  for (int k0 = 0; k0 < n; k0 += kGjPanel) {
    const int kb = std::min(kGjPanel, n - k0);
    hipLaunchKernelGGL(k_gj_panel_load, dim3(nwg), dim3(kGjThreads), 0, s, n, k0, kb, a, pan[0], cv[0], ci[0]);
    CPR_LAUNCH_CHECK();
    for (int t = 0; t < kb; ++t) {
      hipLaunchKernelGGL(k_gj_panel_step, dim3(nwg), dim3(kGjThreads), 0, s, n, k0, kb, t, nwg, pan[t & 1],
                         pan[(t + 1) & 1], cv[t & 1], ci[t & 1], cv[(t + 1) & 1], ci[(t + 1) & 1], piv, bad);
      CPR_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_gj_panel_swap, dim3(div_up(n, kGjSwapThreads)), dim3(kGjSwapThreads), 0, s, n, k0, kb, a,
                       piv, y);
    CPR_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gj_panel_update, dim3(tiles, tiles), dim3(256), 0, s, n, k0, kb, a, pan[kb & 1], y);
    CPR_LAUNCH_CHECK();
  }
}

// dst[i][j] = src[i][cols[j]]
__global__ __launch_bounds__(kBlock) void k_permute_cols(int n, const double* __restrict__ src,
                                                         const int32_t* __restrict__ cols, double* __restrict__ dst) {
  const int i = blockIdx.x;
  for (int j = threadIdx.x; j < n; j += kBlock) dst[(int64_t)i * n + j] = src[(int64_t)i * n + cols[j]];
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
  // the inverse is streamed once per cycle: non-temporal loads keep it from
  // evicting the level data the next kernels read (22.9 -> 21.8 us at 3702
  // rows)
  for (; j + 192 < n; j += 256) {
    a0 = a0 + __builtin_nontemporal_load(r + j) * (double)b[j];
    a1 = a1 + __builtin_nontemporal_load(r + j + 64) * (double)b[j + 64];
    a2 = a2 + __builtin_nontemporal_load(r + j + 128) * (double)b[j + 128];
    a3 = a3 + __builtin_nontemporal_load(r + j + 192) * (double)b[j + 192];
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
