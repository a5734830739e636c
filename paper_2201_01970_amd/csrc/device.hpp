// Device data layouts and kernel launchers of the CPR solve phase (gfx950).
//
// Layouts.  The fine 3x3 block matrix is stored as SELL-64 ("sliced
// ELLPACK"): rows are grouped in slices of 64 consecutive rows, one row per
// lane of a 64-wide wavefront; slice s occupies slots [slice_ptr[s],
// slice_ptr[s+1]), slot t of a slice holds the t-th stored entry of each of its
// 64 rows, lane-contiguous, so a wavefront streams each slot with fully
// coalesced loads while every lane still sums its own row sequentially in
// stored order.  Rows shorter than the slice width are padded with column -1.
// The nine values of a slot are stored as nine lane-contiguous planes (value e
// of lane l of slot t at (t*9 + e)*64 + l).  Scalar AMG matrices (levels, P, R)
// use SELL-64 too when their rows are short and many, otherwise CSR read by a
// group of lanes per row (MatView::group); every layout sums each row in its
// stored order, so all of them give bit-identical results.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cpr {

constexpr int kWave = 64;
constexpr int kBlock = 256;  // threads per workgroup for row kernels (4 slices)
constexpr int32_t kPadCol = -1;
constexpr int32_t kEarlierBit = 1 << 30;  // stage-2 column flag: neighbour of an earlier colour
constexpr int32_t kColMask = kEarlierBit - 1;

template <typename T>
struct SellView {
  int32_t n_rows = 0;
  const int32_t* slice_ptr = nullptr;
  const int32_t* col = nullptr;
  const T* val = nullptr;
};

// An AMG level matrix (or P, R): group == 1 -> SELL-64 (ptr = slice_ptr);
// otherwise CSR (ptr = row_ptr): group 2 -> 16 lanes per row with four
// contiguous entries per lane, 4 -> quad-vector (four lanes per row, four
// contiguous entries per lane), 16/32/64 -> that many lanes per row, one entry
// each.  Groups 2 and 4 need rows padded to a multiple of four entries.
template <typename T>
struct MatView {
  int32_t n_rows = 0;
  int32_t group = 1;   // 1: SELL-64, one lane per row; 4: quad-vector CSR; 16/32/64: CSR, lanes per row
  int32_t depth = 8;   // requests in flight per row: SELL slots (8, 16, 32) or CSR chunks of `group` (4, 8, 16)
  int32_t width = 0;   // SELL: width of every slice when all are equal (ptr unused), else 0
  const int32_t* ptr = nullptr;
  const int32_t* col = nullptr;
  const T* val = nullptr;
};

// Kernel classes whose launches can be timed with HIP events.
struct LaunchTimer {
  virtual ~LaunchTimer() = default;
  virtual void begin(int kind, hipStream_t s) = 0;
  virtual void end(int kind, hipStream_t s, double bytes) = 0;
};

// ---- fine-level (3x3 BSR) kernels ----
// y = A x  (resid == nullptr)  or  y = b - A x (b != nullptr).  A: FP64 or FP32
// values; x: FP64 or FP32; y and b: FP64.
template <typename TA, typename TX>
void launch_bsr_spmv(const SellView<TA>& A, const TX* x, const double* b, double* y, hipStream_t s);

// The first colour of a sweep that starts from x = 0 reads no neighbour: its
// rows get x_i = b_i / a_ii (the sum over earlier colours is empty).  A kernel
// that produces b can write these directly: for device rows p < n_first,
// x[p] = b[p] / diag[p] and snap[p] = x[p] (the sweep's output snapshot), and
// the sweep then starts at its second colour.  n_first = 0: nothing fused.
template <typename T>
struct ZeroStart {
  int32_t n_first = 0;
  const T* diag = nullptr;
  T* x = nullptr;
  T* snap = nullptr;
};

// rp[p] = v[3 perm[p]] (pressure entries of the level-0 device rows), with
// the zero-start first colour of level 0 fused (see ZeroStart)
template <typename T>
void launch_restrict_pressure(int32_t n, const double* v, const int32_t* perm, T* rp, const ZeroStart<T>& zs,
                              hipStream_t s);

// pe[perm[p]] = e[p]
template <typename T>
void launch_scatter(int32_t n, const T* e, const int32_t* perm, T* pe, hipStream_t s);

// One block colour [lo, hi) of the stage-2 block Gauss-Seidel fused with the
// CPR prolongation and residual (rows in block-colour order, cell[q] = cell).
template <typename T>
void launch_stage2(const SellView<T>& A, int32_t lo, int32_t hi, const int32_t* cell, const T* dinv,
                   int32_t dinv_ld, const double* v, const T* pe, T* z, hipStream_t s);

// Block ILU(0) second stage.  Residual (all rows, natural order; R = column 0
// of every stored block, 3 planes): r_i = v_i - sum_j A_ij (pe_j, 0, 0).
// One level of each triangular solve (positions [lo, hi) of that solve's
// level order, row[q] = cell): forward, L = the lower factor blocks (9
// planes), y_i = r_i - sum_{k<i} L_ik y_k; backward, U = the upper blocks,
// uinv[e*ld + q] the inverted pivot blocks, d_i = Uinv_i (y_i - sum_{j>i}
// U_ij d_j), z_i = (pe_i + d_i0, d_i1, d_i2).
template <typename T>
void launch_bilu_residual(const SellView<T>& R, const double* v, const T* pe, T* r, hipStream_t s);
template <typename T>
void launch_bilu_forward(int32_t lo, int32_t hi, const SellView<T>& L, const int32_t* row, const T* r, T* y,
                         hipStream_t s);
template <typename T>
void launch_bilu_backward(int32_t lo, int32_t hi, const SellView<T>& U, const T* uinv, int32_t ld, const int32_t* row,
                          const T* y, const T* pe, T* d, T* z, hipStream_t s);

// One PGS-NO sweep (in place on x) of a CSR level matrix in natural row order
// (A.group 2 or 4: rows padded with column -1): n_chunks contiguous chunks,
// Gauss-Seidel inside a chunk, other chunks' values from snap (null: 0).
template <typename T>
void launch_gs_chunks(const MatView<T>& A, const T* diag, int32_t n_chunks, const T* b, T* x, const T* snap,
                      hipStream_t s);

// ---- nonlinear AMLI-cycle (aggregation AMG) ----
// Dot-product grid of a level of n rows (partials: 2 * grid doubles).
int amli_dot_grid(int64_t n);
// part = partial sums of (x1, y1) and, if x2, of (x2, y2)
template <typename T>
void launch_gcr_dots(int64_t n, const T* x1, const T* y1, const T* x2, const T* y2, double* part, hipStream_t s);
// alpha1 = (f,w1)/(w1,w1) from part; z1 = x; f -= alpha1 w1; scal = {alpha1, (w1,w1)}
template <typename T>
void launch_gcr_step1(int64_t n, const double* part, const T* x, T* z1, T* f, const T* w1, double* scal,
                      hipStream_t s);
// x = alpha1 x, alpha1 = (f,w1)/(w1,w1) from part (a single GCR step)
template <typename T>
void launch_gcr_single(int64_t n, const double* part, T* x, hipStream_t s);
// beta = (w2,w1)/scal[1] from part; w2 -= beta w1; x -= beta z1; part2 = partials of (w2,w2), (r1,w2)
template <typename T>
void launch_gcr_orth(int64_t n, const double* part, const double* scal, T* w2, const T* w1, T* x, const T* z1,
                     const T* r1, double* part2, hipStream_t s);
// x = alpha1 z1 + alpha2 x, alpha2 = (r1,w2)/(w2,w2) from part2
template <typename T>
void launch_gcr_finish(int64_t n, const double* part2, const double* scal, T* x, const T* z1, hipStream_t s);
// Gauss-Jordan elimination with partial pivoting of the row-major n x n
// matrix a in place, by panels of 64 columns (work: gj_workspace_doubles(n)
// doubles, iwork: gj_workspace_ints(n) ints).  Afterwards a holds the inverse
// of the row-interchanged matrix; piv[k] = the row interchanged with row k at
// step k; *bad is set to 1 when a column has no nonzero pivot (*bad is not
// cleared here).
int64_t gj_workspace_doubles(int n);
int64_t gj_workspace_ints(int n);
void launch_gj_inverse(int n, double* a, double* work, int32_t* iwork, int32_t* piv, int32_t* bad, hipStream_t s);
// dst[i][j] = src[i][cols[j]] (n x n, row-major)
void launch_permute_cols(int n, const double* src, const int32_t* cols, double* dst, hipStream_t s);
// x = Ainv b (Ainv n x n FP64 row-major; b, x in T)
template <typename T>
void launch_dense_gemv(int n, const double* ainv, const T* b, T* x, hipStream_t s);

// Decoupling (kind 1 quasi-IMPES, 2 ABF): w[9i..] = W_i from the diagonal
// block of row i, wa[9k..] = W_i A_k for every stored block k of row i (FP64,
// input order); *bad_row = min(*bad_row, i) for rows whose W_i cannot be formed.
void launch_decouple(int32_t n, const int32_t* rp, const int32_t* col, const double* vals, int32_t kind, double* w,
                     double* wa, int32_t* bad_row, hipStream_t s);
// out[3i+r] = (W_i v_i)_r computed in T from (T)v, stored as FP64; w: n x 9 in T.
template <typename T>
void launch_block_gemv(int32_t n, const T* w, const double* v, double* out, hipStream_t s);

// Inverse of the diagonal blocks (LU with partial pivoting), planes dinv[e*ld + q];
// diag_pos[q] = index of the diagonal block of cell cell[q] in the input BSR.
// singular[0] is set to 1 when a pivot is below 1e-300 * max|block|.
template <typename T>
void launch_block_inverse(int32_t n, const double* vals, const int64_t* diag_pos, T* dinv, int32_t ld,
                          int32_t* singular, hipStream_t s);

// For SETUP, from the input BSR (row pointers, columns, values on the device):
// pval[k] = entry (0,0) of block k; nonzero[k] = 1 if block k has a nonzero
// entry; *bad_row = min(*bad_row, i) for every row i whose diagonal block fails
// LU with partial pivoting (pivot <= 1e-300 * max |block entry|).
void launch_setup_values(int32_t n, const int32_t* rp, const int32_t* col, const double* vals, double* pval,
                         uint8_t* nonzero, int32_t* bad_row, hipStream_t s);

// Scatter BSR values (row-major blocks in input order) into a block SELL layout
// given slot positions pos[k] (slot index of input block k, lane included).
template <typename T>
void launch_bsr_values_to_sell(int64_t nnzb, const double* vals, const int64_t* pos, T* sell_val,
                               hipStream_t s);

// ---- AMG level kernels (rows in colour order) ----
// One colour [lo, hi): x_i = (b_i - sum_{j != i} a_ij xt_j) / a_ii, where xt_j is
// s_in[j] for j in [lo, hi) and x[j] otherwise; zero_start: x = 0 on entry, so
// only j < lo contribute.  Writes x[i] and s_out[i].
template <typename T>
void launch_gs_colour(const MatView<T>& A, const T* diag, int32_t lo, int32_t hi, const T* b, T* x,
                      const T* s_in, T* s_out, bool zero_start, hipStream_t s);

// r = b - A x (stored order, diagonal included)
template <typename T>
void launch_csr_residual(const MatView<T>& A, const T* b, const T* x, T* r, hipStream_t s);

// y = A x (sum from 0 in stored order)
template <typename T>
void launch_csr_spmv(const MatView<T>& A, const T* x, T* y, hipStream_t s);

// b = R r (sum from 0 in stored order), with the zero-start first colour of
// the next level fused as above
template <typename T>
void launch_csr_restrict(const MatView<T>& R, const T* r, T* b, const ZeroStart<T>& zs, hipStream_t s);

// x_i = x_i + (sum_J p_iJ e_J); snap[i] = x_i
template <typename T>
void launch_prolong_add(const MatView<T>& P, const T* e, T* x, T* snap, hipStream_t s);

// One level of the one-workgroup tail of the V-cycle.  Matrices stay in
// device memory (quad-vector CSR, rows in colour order); the level's vectors
// x, b, r and the two sweep snapshots live in the LDS vector area for the
// whole kernel, at element offsets off_*.  x, s0 and s1 hold n + 1 entries:
// entry n is a zero that the sweep matrix (w_col, w_val) points at in place of
// the diagonal and of padding, with value 0, so a sweep's products need no
// test for either.  a_col/a_val keep the diagonal (residual).  Colour offsets,
// the diagonal and the row pointers of A, P and R are part of the LDS image
// copied in when the kernel starts, at the 32-bit word offsets w_*.  The first
// tail level reads b from gb when the kernel starts and writes x to gx when it
// ends (its parent level restricts into gb and prolongates from gx).  P
// interpolates from the next level to this one, R restricts this level to the
// next.  When w_wcol >= 0 the sweep matrix is part of the image as well
// (columns at w_wcol, values at w_wval, both at multiples of four words) and
// the sweeps read it from LDS.
template <typename T>
struct TailLevel {
  int32_t n = 0, ncol = 0;
  int32_t off_x = 0, off_b = 0, off_r = 0, off_s0 = 0, off_s1 = 0;
  int32_t w_coff = 0, w_diag = 0, w_arp = 0, w_prp = 0, w_rrp = 0;
  int32_t w_wcol = -1, w_wval = -1;
  const int32_t *a_col = nullptr, *w_col = nullptr, *p_col = nullptr, *r_col = nullptr;
  const T *a_val = nullptr, *w_val = nullptr, *p_val = nullptr, *r_val = nullptr;
  T* gx = nullptr;
  const T* gb = nullptr;
};

// Where the tail kernel keeps things in LDS (offsets in 32-bit words from the
// start of its dynamic LDS): the image [0, img_words) copied from device memory
// when the kernel starts (the coarsest level's FP64 LU factors first when the
// coarsest level has at most 64 rows, then the per-level diagonals, colour
// offsets, row pointers and staged sweep matrices, and rperm at w_rperm); the
// FP64 right-hand side of
// a coarsest level of more than 64 rows at xs_off; the level vectors at v_off.
// img_words is a multiple of 4, xs_off and v_off are even.
struct TailLayout {
  int32_t img_words = 0, w_rperm = 0, xs_off = 0, v_off = 0;
  size_t lds_bytes = 0;
};

// V-cycle of the levels levels[0..nlev-1] (the last one the coarsest, solved
// with the FP64 LU factors of P A = L U, rperm[i] = source row of row i of
// P b; lu is read from the image when n_coarse <= 64, else from device memory)
// in one workgroup.
template <typename T>
void launch_tail_vcycle(const TailLevel<T>* levels, int nlev, int pre, int post, int32_t n_coarse, const double* lu,
                        const uint32_t* img, const TailLayout& lay, hipStream_t s);

// Largest dynamic LDS a workgroup of the tail kernel may use on the current device.
size_t tail_lds_limit();

// ---- setup kernel: strength masks (bit 1: RS strength, bit 2: eq. (strong-matrix))
void launch_strength(int32_t n, const int32_t* ptr, const int32_t* col, const double* val, double theta_rs,
                     double theta_color, uint8_t* mask, hipStream_t s);

// ---- vector helpers ----
template <typename TS, typename TD>
void launch_gather(int32_t n, const TS* src, const int32_t* perm, TD* dst, hipStream_t s);  // dst[p]=src[perm[p]]
template <typename TS, typename TD>
void launch_scatter_cast(int32_t n, const TS* src, const int32_t* perm, TD* dst, hipStream_t s);  // dst[perm[p]]=src[p]
template <typename T>
void launch_fill(int64_t n, T value, T* dst, hipStream_t s);
template <typename TS, typename TD>
void launch_copy_cast(int64_t n, const TS* src, TD* dst, hipStream_t s);
void launch_copy_bytes(int64_t n_bytes, const void* src, void* dst, hipStream_t s);
// *flag = 1 if the int arrays a and b (device, n entries) differ anywhere; *flag is not cleared
void launch_int_diff(int64_t n, const int32_t* a, const int32_t* b, int32_t* flag, hipStream_t s);

// ---- Krylov kernels (FP64) ----
// Reductions run on at most this many workgroups (two-stage, fixed order).
constexpr int kKrylovGridMax = 2048;
int krylov_grid(int64_t n);

// The device scalars and partial sums of one FGMRES solve with restart m:
// Hessenberg H ((m+1) x m, column-major), Givens cosines and sines (m), the
// least-squares right-hand side g (m+1), y (m), the current column norm
// (hnorm), the per-workgroup partial dots of up to m+1 basis vectors
// (partial, (m+1) x kKrylovGridMax) and of one norm (norm_partial), and four
// report words the host reads back after every step.
struct KrylovWork {
  double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr, *hnorm = nullptr;
  double *partial = nullptr, *norm_partial = nullptr, *report = nullptr;
};
// Doubles a KrylovWork of restart m occupies when carved out of one array
// (every part starts on a 256-byte boundary: 32 doubles).
constexpr int64_t krylov_round_up(int64_t n) { return (n + 31) / 32 * 32; }
constexpr int64_t krylov_work_doubles(int m) {
  return krylov_round_up(int64_t(m + 1) * m) + 3 * krylov_round_up(m) + krylov_round_up(m + 1) + krylov_round_up(1) +
         krylov_round_up(int64_t(m + 1) * kKrylovGridMax) + krylov_round_up(kKrylovGridMax) + krylov_round_up(4);
}
// The parts of a KrylovWork of restart m laid out from base (256-byte aligned).
KrylovWork krylov_work_carve(double* base, int m);

// Largest restart the allocation-free solve accepts, and the device address
// of that solve's static scratch array on `device` (looked up once per device).
constexpr int kNoAllocMaxRestart = 64;
double* noalloc_scratch(int device);
// partial[i*grid + blk] = partial dot of w with V[j0+i] (i < nb); V row stride ld
void launch_multidot(int64_t n, const double* w, const double* V, int64_t ld, int j0, int nb, double* partial,
                     hipStream_t s);
// out[i] = sum over blocks of partial[i*grid + blk] (fixed order), for i < count
void launch_reduce_partials(const double* partial, int grid, int count, double* out, hipStream_t s);
// w -= sum_i h[i] * V[j0+i] for i < nb; if norm_partial: partial sums of w^2
void launch_axpy_norm(int64_t n, double* w, const double* V, int64_t ld, int j0, int nb, const double* h,
                      double* norm_partial, hipStream_t s);
// partial sums of v^2
void launch_norm_partial(int64_t n, const double* v, double* partial, hipStream_t s);
// v = w / h[0]  (h on device)
void launch_scale_div(int64_t n, const double* w, const double* h, double* v, hipStream_t s);
// Givens step j of the Hessenberg column; see krylov.hip
void launch_givens(int m, int j, const double* norm_partial, int grid, double* H, double* cs, double* sn,
                   double* g, double* hnorm, double* report, hipStream_t s);
// set g = 0 except g[0] = norm (from the partials); report[0..1]; v-scale factor
void launch_start_cycle(int m, const double* norm_partial, int grid, double* g, double* hnorm, double* report,
                        hipStream_t s);
// y = H(0:k,0:k)^{-1} g(0:k) (upper triangular), H column-major with ld m+1
void launch_backsolve(int m, int k, const double* H, const double* g, double* y, hipStream_t s);
// x += sum_{i<k} y[i] * Z[i]
template <typename TZ>
void launch_update_x(int64_t n, double* x, const TZ* Z, int64_t ld, int k, const double* y, hipStream_t s);

}  // namespace cpr
