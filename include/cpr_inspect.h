/*
 * cpr_inspect.h - entry points that expose single steps of the CPR solve
 * phase and the products of SETUP, so that each can be checked on its own
 * against an independent implementation and timed in isolation.
 *
 * Same conventions as cpr.h: C functions, status codes, device pointers on
 * the handle's GPU, work on the handle's stream, calls return after the
 * stream has finished the work.  Levels are numbered from 0 (the pressure
 * matrix A_PP) to n_levels-1 (the coarsest, solved by dense LU).  Vectors
 * on level l are indexed in the level's own row numbering (the numbering the
 * Galerkin product produces: coarse points in ascending fine index), never
 * in the device's internal colour-permuted order.
 */
#ifndef CPR_MI355X_INSPECT_H
#define CPR_MI355X_INSPECT_H

#include <stdint.h>

#include "cpr.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---- single steps of the solve phase (device arrays) ------------------- */

/* y = A x with the outer FP64 matrix (the product of Algorithm
 * "ASCPR-GMRES" and the residuals of Algorithm "CPR method").
 * x, y: 3*n_block_rows doubles. */
cpr_status cpr_spmv(cpr_handle* h, const double* x, double* y);

/* z = B v: one application of the CPR preconditioner (Algorithm "CPR
 * method" with x = 0).  v, z: 3*n_block_rows doubles. */
cpr_status cpr_precond_apply(cpr_handle* h, const double* v, double* z);

/* e = B_P r: one V-cycle of the pressure AMG from a zero initial guess
 * (stage 1 of eq. (CPR)).  r, e: n_block_rows doubles, level-0 numbering. */
cpr_status cpr_vcycle(cpr_handle* h, const double* r, double* e);

/* n_sweeps PGS-SCM sweeps (Algorithm "PGS-SCM") on level `level`, in place
 * on x (n_l doubles), right-hand side b.  zero_start = 1 declares x = 0 on
 * entry (the V-cycle's first pre-sweep), which the device exploits. */
cpr_status cpr_smooth(cpr_handle* h, int32_t level, double* x, const double* b, int32_t n_sweeps,
                      int32_t zero_start);

/* z = Pi_P pe + R (v - A Pi_P pe): the second stage of Algorithm "CPR
 * method" given a stage-1 pressure correction pe, with the handle's R (block
 * Gauss-Seidel or block ILU(0), cpr_params.second_stage) and the copy of A
 * the preconditioner was built on, in the preconditioner's precision.
 * v, z: 3*n_block_rows doubles; pe: n_block_rows doubles (cell order). */
cpr_status cpr_second_stage(cpr_handle* h, const double* v, const double* pe, double* z);

/* ---- products of SETUP (host arrays, filled from the handle) ---------- */

/* out[0..7] = n_rows, nnz, n_colours, n_coarse (rows of level+1, 0 on the
 * coarsest), is_coarsest, n_levels, nnz_P, n_block_colours. */
cpr_status cpr_level_info(const cpr_handle* h, int32_t level, int64_t out[8]);

/* The level matrix in its own numbering (row_ptr[n+1], col[nnz], val[nnz]),
 * the strength masks over its stored entries computed on the GPU
 * (rs_strong: classical RS strength; color_strong: eq. (strong-matrix);
 * uint8 0/1, may be NULL), the colour of every row (int32, may be NULL;
 * numbered in creation order of Algorithm "VerticesGrouping") and the C/F
 * split (int8, 1 = C, 2 = F, may be NULL; not defined on the coarsest). */
cpr_status cpr_level_arrays(const cpr_handle* h, int32_t level, int32_t* row_ptr, int32_t* col,
                            double* val, uint8_t* rs_strong, uint8_t* color_strong,
                            int32_t* colour, int8_t* cf);

/* Interpolation P of level -> level+1 in the levels' own numbering
 * (row_ptr[n+1], col[nnz_P], val[nnz_P]). */
cpr_status cpr_level_interp(const cpr_handle* h, int32_t level, int32_t* row_ptr, int32_t* col,
                            double* val);

/* Aggregate of every row of level `level` (int32[n_l], numbered in formation
 * order) when the pressure solver is the aggregation AMG (amg_kind 1).
 * CPR_ERR_INVALID_ARG for the coarsest level or a Ruge-Stueben hierarchy. */
cpr_status cpr_level_aggregates(const cpr_handle* h, int32_t level, int32_t* agg);

/* Colour of every cell in the stage-2 block colouring (int32[n_block_rows]). */
cpr_status cpr_block_colours(const cpr_handle* h, int32_t* colour);

/* The block ILU(0) factors of a handle whose second stage is block ILU(0)
 * (Sections 3.1 and 6), FP64, in the input block order: lu[nnz_blocks*9]
 * holds L_ik (k < i) and U_ij (j >= i, U_ii before inversion), uinv[n*9] the
 * inverted pivot blocks, flev/blev[n] the level of every row in the forward
 * and backward solve; n_levels[2] receives the two level counts.  Any array
 * may be NULL.  CPR_ERR_INVALID_ARG when the second stage is block GS. */
cpr_status cpr_bilu_factors(const cpr_handle* h, double* lu, double* uinv, int32_t* flev, int32_t* blev,
                            int32_t* n_levels);

/* ---- host-only SETUP routines (no GPU work; for CPU tests) ------------- */

/* Algorithm "VerticesGrouping" on a strength pattern S given as CSR rows
 * (s_ptr[n+1], s_col; s_col lists the strong neighbours of each row).
 * colour[n] receives the colour of each vertex; returns the colour count
 * in *n_colours. */
cpr_status cpr_host_grouping(int32_t n, const int32_t* s_ptr, const int32_t* s_col,
                             int32_t* colour, int32_t* n_colours);

/* Classical RS C/F split (first pass with lambda = |S^T_i| and ties to the
 * smallest index, second pass enforcing shared C points); cf[n] receives
 * 1 = C, 2 = F. */
cpr_status cpr_host_rs_split(int32_t n, const int32_t* s_ptr, const int32_t* s_col, int8_t* cf);

/* Classical RS interpolation of the CSR matrix A (rows sorted) given the RS
 * strength mask over its stored entries and a C/F split.  Writes P with
 * n rows; p_ptr must hold n+1 entries, p_col/p_val at least nnz(A) entries;
 * returns the coarse size in *n_coarse. */
cpr_status cpr_host_interpolation(int32_t n, const int32_t* a_ptr, const int32_t* a_col,
                                  const double* a_val, const uint8_t* strong, const int8_t* cf,
                                  int32_t* p_ptr, int32_t* p_col, double* p_val, int32_t* n_coarse);

/* Galerkin product A_c = P^T A P in the library's fixed summation order.
 * First call with c_ptr != NULL and c_col == NULL to get the row pointer
 * (c_ptr[n_coarse+1]), then with all arrays to get columns and values. */
cpr_status cpr_host_galerkin(int32_t n, int32_t n_coarse, const int32_t* a_ptr, const int32_t* a_col,
                             const double* a_val, const int32_t* p_ptr, const int32_t* p_col,
                             const double* p_val, int32_t* c_ptr, int32_t* c_col, double* c_val);

/* Aggregates of unsmoothed-aggregation AMG (the paper's NPAIR aggregation,
 * Section 6): npair passes of non-symmetric pairwise matching with
 * threshold beta on the CSR matrix A (rows sorted).  agg[n] receives the
 * aggregate of every row (numbered in formation order), *n_agg their count. */
cpr_status cpr_host_aggregates(int32_t n, const int32_t* a_ptr, const int32_t* a_col, const double* a_val,
                               double beta, int32_t npair, int32_t* agg, int32_t* n_agg);

/* Block ILU(0) (the second stage R of eq. (CPR) named in Section 3.1, with
 * the level scheduling of Section 6) of a 3x3-block matrix with sorted
 * columns and stored diagonal blocks: vals[nnz*9] in, lu[nnz*9] (L_ik for
 * k < i, U_ij for j >= i), uinv[n*9] (inverted pivot blocks), flev/blev[n]
 * (forward / backward level of every row) out.  CPR_ERR_SINGULAR_BLOCK when
 * a pivot block is singular. */
cpr_status cpr_host_bilu0(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* vals, double* lu,
                          double* uinv, int32_t* flev, int32_t* blev);

/* ---- measurement ------------------------------------------------------ */

/* Kernel classes timed with HIP events on the handle's stream while
 * profiling is enabled. */
enum {
  CPR_KSTAT_SPMV = 0,           /* outer FP64 BSR product */
  CPR_KSTAT_SMOOTH_L0 = 1,      /* PGS-SCM colour sweeps of level 0 */
  CPR_KSTAT_TRANSFER_L0 = 2,    /* level-0 residual + restriction + prolongation */
  CPR_KSTAT_STAGE2 = 3,         /* stage-2 block Gauss-Seidel colour kernels */
  CPR_KSTAT_SMOOTH_COARSE = 4,  /* PGS-SCM colour sweeps of levels 1.. (outside the tail) */
  CPR_KSTAT_TRANSFER_COARSE = 5,/* residual + restriction + prolongation of levels 1.. */
  CPR_KSTAT_TAIL = 6,           /* the one-workgroup V-cycle of the smallest levels */
  CPR_KSTAT_COUNT = 7
};

/* enable != 0: record a HIP event pair around every launch of the kernel
 * classes above during cpr_solve; enable == 0 stops and keeps the totals. */
cpr_status cpr_profile_enable(cpr_handle* h, int32_t enable);

/* Launch count, summed duration (ms) and algorithmic bytes for a kernel
 * class since profiling was last enabled. */
cpr_status cpr_profile_read(cpr_handle* h, int32_t kind, int64_t* launches, double* total_ms,
                            double* bytes);

/* Copy n_bytes from src to dst (device) with a plain streaming kernel on
 * hip_stream; used to calibrate hardware traffic counters. */
cpr_status cpr_copy_kernel(void* dst, const void* src, int64_t n_bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* CPR_MI355X_INSPECT_H */
