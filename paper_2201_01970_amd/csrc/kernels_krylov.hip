// FP64 kernels of the flexible GMRES (Algorithm "ASCPR-GMRES"): fused
// classical Gram-Schmidt dots and updates, norms, the Givens update of the
// Hessenberg least-squares problem, back substitution and the solution
// update.  Reductions are two-stage with a fixed grid and a fixed combining
// order, so results do not depend on scheduling.
#include "kernels_common.hpp"

namespace cpr {

int krylov_grid(int64_t n) {
  const int64_t g = (n + kBlock * 4 - 1) / (kBlock * 4);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, kKrylovGridMax));
}

// Sum of v over the workgroup: wave shuffles then the four wave sums in order.
// Valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* lds) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s = s + lds[w];
  return s;
}

template <int NB>
__global__ __launch_bounds__(kBlock) void k_multidot(int64_t n, const double* __restrict__ w,
                                                     const double* __restrict__ V, int64_t ld, int j0,
                                                     double* __restrict__ partial) {
  __shared__ double lds[kBlock / 64];
  double acc[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) acc[i] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += stride) {
    const double wk = w[k];
#pragma unroll
    for (int i = 0; i < NB; ++i) acc[i] = acc[i] + wk * V[(int64_t)(j0 + i) * ld + k];
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const double s = block_sum(acc[i], lds);
    if (threadIdx.x == 0) partial[(int64_t)i * gridDim.x + blockIdx.x] = s;
  }
}

template <int NB, bool NORM>
__global__ __launch_bounds__(kBlock) void k_axpy_norm(int64_t n, double* __restrict__ w,
                                                      const double* __restrict__ V, int64_t ld, int j0,
                                                      const double* __restrict__ h,
                                                      double* __restrict__ norm_partial) {
  __shared__ double lds[kBlock / 64];
  double hh[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) hh[i] = h[i];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += stride) {
    double wk = w[k];
#pragma unroll
    for (int i = 0; i < NB; ++i) wk = wk - hh[i] * V[(int64_t)(j0 + i) * ld + k];
    w[k] = wk;
    if (NORM) acc = acc + wk * wk;
  }
  if (NORM) {
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) norm_partial[blockIdx.x] = s;
  }
}

template <int NB, typename TZ>
__global__ __launch_bounds__(kBlock) void k_update_x(int64_t n, double* __restrict__ x, const TZ* __restrict__ Z,
                                                     int64_t ld, int j0, const double* __restrict__ y) {
  double yy[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) yy[i] = y[j0 + i];
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += stride) {
    double xk = x[k];
#pragma unroll
    for (int i = 0; i < NB; ++i) xk = xk + yy[i] * (double)Z[(int64_t)(j0 + i) * ld + k];
    x[k] = xk;
  }
}

#define CPR_NB_SWITCH(NBV, CALL) \
  switch (NBV) {                 \
    case 1: CALL(1); break;      \
    case 2: CALL(2); break;      \
    case 3: CALL(3); break;      \
    case 4: CALL(4); break;      \
    case 5: CALL(5); break;      \
    case 6: CALL(6); break;      \
    case 7: CALL(7); break;      \
    case 8: CALL(8); break;      \
    case 9: CALL(9); break;      \
    case 10: CALL(10); break;    \
    case 11: CALL(11); break;    \
    case 12: CALL(12); break;    \
    case 13: CALL(13); break;    \
    case 14: CALL(14); break;    \
    case 15: CALL(15); break;    \
    case 16: CALL(16); break;    \
    default: break;              \
  }
constexpr int kNbMax = 16;

void launch_multidot(int64_t n, const double* w, const double* V, int64_t ld, int j0, int nb, double* partial,
                     hipStream_t s) {
  const int grid = krylov_grid(n);
  for (int c = 0; c < nb; c += kNbMax) {
    const int cnt = std::min(kNbMax, nb - c);
#define CALL(K)                                                                                      \
  hipLaunchKernelGGL((k_multidot<K>), dim3(grid), dim3(kBlock), 0, s, n, w, V, ld, j0 + c, \
                     partial + (int64_t)c * grid)
    CPR_NB_SWITCH(cnt, CALL)
#undef CALL
  }
  CPR_LAUNCH_CHECK();
}

void launch_axpy_norm(int64_t n, double* w, const double* V, int64_t ld, int j0, int nb, const double* h,
                      double* norm_partial, hipStream_t s) {
  const int grid = krylov_grid(n);
  for (int c = 0; c < nb; c += kNbMax) {
    const int cnt = std::min(kNbMax, nb - c);
    const bool last = c + cnt >= nb;
    if (last && norm_partial) {
#define CALL(K)                                                                                            \
  hipLaunchKernelGGL((k_axpy_norm<K, true>), dim3(grid), dim3(kBlock), 0, s, n, w, V, ld, j0 + c, h + c, \
                     norm_partial)
      CPR_NB_SWITCH(cnt, CALL)
#undef CALL
    } else {
#define CALL(K)                                                                                             \
  hipLaunchKernelGGL((k_axpy_norm<K, false>), dim3(grid), dim3(kBlock), 0, s, n, w, V, ld, j0 + c, h + c, \
                     norm_partial)
      CPR_NB_SWITCH(cnt, CALL)
#undef CALL
    }
  }
  CPR_LAUNCH_CHECK();
}

template <typename TZ>
void launch_update_x(int64_t n, double* x, const TZ* Z, int64_t ld, int k, const double* y, hipStream_t s) {
  const int grid = krylov_grid(n);
  for (int c = 0; c < k; c += kNbMax) {
    const int cnt = std::min(kNbMax, k - c);
#define CALL(K) hipLaunchKernelGGL((k_update_x<K, TZ>), dim3(grid), dim3(kBlock), 0, s, n, x, Z, ld, c, y)
    CPR_NB_SWITCH(cnt, CALL)
#undef CALL
  }
  CPR_LAUNCH_CHECK();
}
template void launch_update_x<double>(int64_t, double*, const double*, int64_t, int, const double*, hipStream_t);
template void launch_update_x<float>(int64_t, double*, const float*, int64_t, int, const double*, hipStream_t);

__global__ __launch_bounds__(kBlock) void k_norm_partial(int64_t n, const double* __restrict__ v,
                                                         double* __restrict__ partial) {
  __shared__ double lds[kBlock / 64];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += stride) acc = acc + v[k] * v[k];
  const double s = block_sum(acc, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

void launch_norm_partial(int64_t n, const double* v, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_partial, dim3(krylov_grid(n)), dim3(kBlock), 0, s, n, v, partial);
  CPR_LAUNCH_CHECK();
}

// out[i] = sum_b partial[i*grid + b], one workgroup per i, fixed order.
__global__ __launch_bounds__(kBlock) void k_reduce_partials(const double* __restrict__ partial, int grid,
                                                            double* __restrict__ out) {
  __shared__ double lds[kBlock / 64];
  const double* p = partial + (int64_t)blockIdx.x * grid;
  double acc = 0.0;
  for (int b = threadIdx.x; b < grid; b += kBlock) acc = acc + p[b];
  const double s = block_sum(acc, lds);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

void launch_reduce_partials(const double* partial, int grid, int count, double* out, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_reduce_partials, dim3(count), dim3(kBlock), 0, s, partial, grid, out);
  CPR_LAUNCH_CHECK();
}

__global__ __launch_bounds__(kBlock) void k_scale_div(int64_t n, const double* __restrict__ w,
                                                      const double* __restrict__ h, double* __restrict__ v) {
  const double d = h[0];
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += stride) v[k] = w[k] / d;
}

void launch_scale_div(int64_t n, const double* w, const double* h, double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_div, dim3(krylov_grid(n)), dim3(kBlock), 0, s, n, w, h, v);
  CPR_LAUNCH_CHECK();
}

// Column j of the Hessenberg matrix H (column-major, leading dimension m+1):
// h_{j+1,j} = ||w|| from the norm partials, the previous rotations applied to
// the column, the new rotation rho = sqrt(h_jj^2 + h_{j+1,j}^2),
// c = h_jj/rho, s = h_{j+1,j}/rho, then g_{j+1} = -s g_j, g_j = c g_j.
// report[0] = |g_{j+1}|, report[1] = h_{j+1,j}; hnorm[0] = h_{j+1,j}.
__global__ __launch_bounds__(kBlock) void k_givens(int m, int j, const double* __restrict__ norm_partial, int grid,
                                                   double* __restrict__ H, double* __restrict__ cs,
                                                   double* __restrict__ sn, double* __restrict__ g,
                                                   double* __restrict__ hnorm, double* __restrict__ report) {
  __shared__ double lds[kBlock / 64];
  double acc = 0.0;
  for (int b = threadIdx.x; b < grid; b += kBlock) acc = acc + norm_partial[b];
  const double ss = block_sum(acc, lds);
  if (threadIdx.x != 0) return;
  const double hn = sqrt(ss);
  double* Hj = H + (int64_t)j * (m + 1);
  Hj[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * Hj[i] + sn[i] * Hj[i + 1];
    Hj[i + 1] = -sn[i] * Hj[i] + cs[i] * Hj[i + 1];
    Hj[i] = t;
  }
  const double rho = sqrt(Hj[j] * Hj[j] + Hj[j + 1] * Hj[j + 1]);
  cs[j] = Hj[j] / rho;
  sn[j] = Hj[j + 1] / rho;
  Hj[j] = rho;
  Hj[j + 1] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  hnorm[0] = hn;
  report[0] = fabs(g[j + 1]);
  report[1] = hn;
}

void launch_givens(int m, int j, const double* norm_partial, int grid, double* H, double* cs, double* sn, double* g,
                   double* hnorm, double* report, hipStream_t s) {
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(kBlock), 0, s, m, j, norm_partial, grid, H, cs, sn, g, hnorm, report);
  CPR_LAUNCH_CHECK();
}

__global__ __launch_bounds__(kBlock) void k_start_cycle(int m, const double* __restrict__ norm_partial, int grid,
                                                        double* __restrict__ g, double* __restrict__ hnorm,
                                                        double* __restrict__ report) {
  __shared__ double lds[kBlock / 64];
  double acc = 0.0;
  for (int b = threadIdx.x; b < grid; b += kBlock) acc = acc + norm_partial[b];
  const double ss = block_sum(acc, lds);
  if (threadIdx.x != 0) return;
  const double rn = sqrt(ss);
  for (int i = 0; i <= m; ++i) g[i] = 0.0;
  g[0] = rn;
  hnorm[0] = rn;
  report[0] = rn;
  report[1] = rn;
}

void launch_start_cycle(int m, const double* norm_partial, int grid, double* g, double* hnorm, double* report,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_start_cycle, dim3(1), dim3(kBlock), 0, s, m, norm_partial, grid, g, hnorm, report);
  CPR_LAUNCH_CHECK();
}

// y_i = (g_i - sum_{l>i} h_il y_l) / h_ii for i = k-1 .. 0
__global__ void k_backsolve(int m, int k, const double* __restrict__ H, const double* __restrict__ g,
                            double* __restrict__ y) {
  if (threadIdx.x != 0) return;
  const int ld = m + 1;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int l = i + 1; l < k; ++l) s = s - H[(int64_t)l * ld + i] * y[l];
    y[i] = s / H[(int64_t)i * ld + i];
  }
}

void launch_backsolve(int m, int k, const double* H, const double* g, double* y, hipStream_t s) {
  if (k == 0) return;
  hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(64), 0, s, m, k, H, g, y);
  CPR_LAUNCH_CHECK();
}

}  // namespace cpr
