// Decoupling of the block rows before the CPR preconditioner is built: the
// rows of A are multiplied by a block-diagonal W (one 3x3 block per cell), B
// is built on W A and applied to W v, while the outer FGMRES keeps A.  Two
// classical choices for the pressure equation of a black-oil Jacobian:
//   quasi-IMPES: W_i = I with (0,1) = -D_01/D_11 and (0,2) = -D_02/D_22, D_i
//     the diagonal block of cell i (the pressure row loses the saturation
//     derivatives of its own diagonal block, using diagonal entries only);
//   alternate block factorisation (ABF): W_i = D_i^{-1}, so every diagonal
//     block of W A is the identity.
// The paper leaves the decoupling out with the well terms (Section 2.2);
// these kernels extend the hot path to the full system of eq.
// (Jacobian-system), where wells are extra block rows of A.
#include "kernels_common.hpp"

namespace cpr {

// One thread per block row i: W_i from the diagonal block (searched in the
// row's stored columns).  *bad_row = min over rows whose W cannot be formed
// (ABF: singular D_i; quasi-IMPES: D_11 or D_22 zero).
__global__ __launch_bounds__(kBlock) void k_decouple_weights(int32_t n, const int32_t* __restrict__ rp,
                                                             const int32_t* __restrict__ col,
                                                             const double* __restrict__ vals, int32_t kind,
                                                             double* __restrict__ w, int32_t* __restrict__ bad_row) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  int64_t dk = -1;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
    if (col[k] == i) dk = k;
  double out[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
  bool ok = dk >= 0;
  if (ok) {
    const double* d = vals + 9 * dk;
    if (kind == 2) {
      ok = inverse3x3(d, out);
    } else {
      ok = d[4] != 0.0 && d[8] != 0.0;
      out[1] = -d[1] / d[4];
      out[2] = -d[2] / d[8];
    }
  }
  if (!ok) {
    atomicMin(bad_row, i);
    for (int e = 0; e < 9; ++e) out[e] = 0.0;
  }
  for (int e = 0; e < 9; ++e) w[9 * (int64_t)i + e] = out[e];
}

// One thread per block row i: every stored block of row i multiplied on the
// left by W_i, each entry sum_m W[r][m] A[m][c] accumulated from 0 over m.
__global__ __launch_bounds__(kBlock) void k_left_blocks(int32_t n, const int32_t* __restrict__ rp,
                                                        const double* __restrict__ w,
                                                        const double* __restrict__ vals, double* __restrict__ out) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double wi[9];
  for (int e = 0; e < 9; ++e) wi[e] = w[9 * (int64_t)i + e];
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
    const double* a = vals + 9 * (int64_t)k;
    double* o = out + 9 * (int64_t)k;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double t = 0.0;
        t = t + wi[3 * r + 0] * a[0 + c];
        t = t + wi[3 * r + 1] * a[3 + c];
        t = t + wi[3 * r + 2] * a[6 + c];
        o[3 * r + c] = t;
      }
  }
}

// (W v)_i = W_i v_i in the preconditioner's precision T (v cast to T first),
// each component accumulated from 0 over columns 0, 1, 2; stored as FP64
// (exact for T = float).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_block_gemv(int32_t n, const T* __restrict__ w,
                                                       const double* __restrict__ v, double* __restrict__ out) {
  const int32_t i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const T v0 = (T)v[3 * (int64_t)i], v1 = (T)v[3 * (int64_t)i + 1], v2 = (T)v[3 * (int64_t)i + 2];
  const T* wi = w + 9 * (int64_t)i;
  for (int r = 0; r < 3; ++r) {
    T o = (T)0;
    o = o + wi[3 * r + 0] * v0;
    o = o + wi[3 * r + 1] * v1;
    o = o + wi[3 * r + 2] * v2;
    out[3 * (int64_t)i + r] = (double)o;
  }
}

void launch_decouple(int32_t n, const int32_t* rp, const int32_t* col, const double* vals, int32_t kind, double* w,
                     double* wa, int32_t* bad_row, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_decouple_weights, dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, n, rp, col, vals, kind, w,
                     bad_row);
  CPR_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_left_blocks, dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, n, rp, w, vals, wa);
  CPR_LAUNCH_CHECK();
}

template <typename T>
void launch_block_gemv(int32_t n, const T* w, const double* v, double* out, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_block_gemv<T>), dim3(div_up(n, kBlock)), dim3(kBlock), 0, s, n, w, v, out);
  CPR_LAUNCH_CHECK();
}
template void launch_block_gemv<double>(int32_t, const double*, const double*, double*, hipStream_t);
template void launch_block_gemv<float>(int32_t, const float*, const double*, double*, hipStream_t);

}  // namespace cpr
