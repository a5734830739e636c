/*
 * cpr.h - C ABI of the MI355X CPR-FGMRES solver for 3x3-block black-oil
 * Jacobians.
 *
 * Method: Zhao, Feng, Zhang, Shu, "Parallel Multi-Stage Preconditioners with
 * Adaptive Setup for the Black Oil Model" (arXiv 2201.01970).
 *   - the preconditioner B is CPR, Section 3.1, eq. (CPR):
 *       I - B A = (I - R A)(I - Pi_P B_P Pi_P^T A),
 *     applied as in Algorithm "CPR method" (stage 1: pressure AMG V-cycle
 *     smoothed by the PGS-SCM multi-colour Gauss-Seidel of Section 5.2;
 *     stage 2: multi-colour block Gauss-Seidel);
 *   - the outer solver is restarted flexible GMRES (Section 4, Algorithm
 *     "ASCPR-GMRES") and SETUP is reused across Newton steps by the adaptive
 *     rule of Algorithm "ASCPR";
 *   - a change of matrix size always needs a new SETUP (the Remark following
 *     Algorithm "ASCPR"): here that is a new handle.
 *
 * All functions are C, never throw, and report failure through cpr_status.
 * Device pointers are HIP device addresses on the GPU that is current when
 * cpr_setup is called; every kernel of a handle runs on the handle's stream.
 */
#ifndef CPR_MI355X_CPR_H
#define CPR_MI355X_CPR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CPR_OK = 0,
  CPR_NOT_CONVERGED = 1,        /* warning: x holds the last iterate, info is filled */
  CPR_ERR_INVALID_ARG = -1,     /* bad sizes, block_dim != 3, unsorted columns, missing diagonal */
  CPR_ERR_PATTERN_MISMATCH = -2,/* update_values with a different sparsity pattern */
  CPR_ERR_SIZE_MISMATCH = -3,   /* update_values with a different size */
  CPR_ERR_SINGULAR_BLOCK = -4,  /* a 3x3 diagonal block has no usable pivot */
  CPR_ERR_SINGULAR_COARSE = -5, /* the coarsest AMG matrix has no usable pivot */
  CPR_ERR_NAN = -6,             /* NaN or Inf in the right-hand side or the iteration */
  CPR_ERR_OOM = -7,             /* device allocation failed */
  CPR_ERR_HIP = -8              /* any other HIP runtime error */
} cpr_status;

typedef enum { CPR_MEM_HOST = 0, CPR_MEM_DEVICE = 1 } cpr_mem;

/* A 3x3-block CSR (BSR) matrix (Section 2.2: three primary unknowns per
 * cell, so the reservoir Jacobian is a sparse matrix of 3x3 blocks).
 * row_ptr[n_block_rows+1] and col_idx[nnz_blocks] are int32; the columns of
 * each block row are strictly ascending and include the diagonal block.
 * values holds nnz_blocks*9 doubles, each block row-major.  The unknowns of
 * cell i are 3i (pressure), 3i+1, 3i+2 (saturations).  `location` says
 * whether the three arrays are host or device memory.  The library deep-copies
 * them; the caller keeps ownership. */
typedef struct {
  int32_t n_block_rows;
  int32_t nnz_blocks;
  int32_t block_dim; /* must be 3 */
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const double* values;
  int32_t location; /* cpr_mem */
} cpr_bsr;

/* Solver parameters.  Defaults (cpr_params_default) in brackets. */
typedef struct {
  int32_t restart;        /* FGMRES restart length m [30] (Section 6 uses m = 28) */
  int32_t max_restarts;   /* maximum restart cycles [100] (MaxIt of Algorithm ASCPR-GMRES) */
  double theta_rs;        /* RS coarsening strength threshold [0.25] */
  double theta_color;     /* colouring threshold theta of eq. (strong-matrix) [0.05] */
  int32_t coarse_max;     /* stop coarsening at or below this many rows [50] */
  int32_t max_levels;     /* maximum AMG levels [25] */
  int32_t pre_sweeps;     /* PGS-SCM pre-smoothing sweeps [2] */
  int32_t post_sweeps;    /* PGS-SCM post-smoothing sweeps [2] */
  int32_t precond_fp32;   /* 1: preconditioner stored and computed in FP32 (FP64
                             outer FGMRES, FP64 coarsest solve) [0] */
  int32_t reuse_mode;     /* 0: SETUP before every solve on new values;
                             1: paper rule, reuse iff It^(k-1) <= mu;
                             2: relative rule, reuse iff It^(k-1) <= reuse_factor*It_ref [2].
                             In every mode, values changed before the first solve
                             trigger a SETUP for it (k = 1) */
  int32_t mu;             /* threshold of reuse_mode 1 [20] */
  double reuse_factor;    /* factor of reuse_mode 2 [1.3] */
  int32_t use_graphs;     /* 1: replay each FGMRES step as one captured HIP graph [1] */
  int32_t tail_nnz;       /* AMG levels from the first one whose own and every coarser
                             level's matrix holds at most this many entries are run as
                             one single-workgroup V-cycle kernel; 0 = never [30000] */
  int32_t row_layout;     /* storage of AMG level matrices: 0 = chosen per matrix from its
                             size and row lengths; 1 = one lane per row (SELL-64) everywhere;
                             2 = CSR read by 16 lanes per row, four contiguous entries
                             per lane (rows padded to a multiple of four entries);
                             4 = quad-vector CSR (four lanes per row, rows padded to a
                             multiple of four entries) everywhere; 16/32/64 = CSR read by
                             lane groups of that size everywhere.  Levels run by the
                             single-workgroup kernel always use quad-vector CSR [0] */
  int32_t second_stage;   /* R of eq. (CPR): 0 = one forward multi-colour block
                             Gauss-Seidel sweep; 1 = block ILU(0) in natural order,
                             applied with level-scheduled triangular solves (the
                             paper's R, Sections 3.1 and 6) [0] */
  int32_t decoupling;     /* rows multiplied by a block-diagonal W before B is built
                             (B is built on W A and applied to W v; the outer FGMRES
                             keeps A): 0 = none; 1 = quasi-IMPES (W_i = I with
                             (0,1) = -D_01/D_11, (0,2) = -D_02/D_22 of the diagonal
                             block D_i); 2 = alternate block factorisation (W_i =
                             D_i^-1) [0] */
  int32_t smoother;       /* AMG smoother: 0 = PGS-SCM (Algorithm "PGS-SCM", colours of
                             eq. (strong-matrix)); 1 = PGS-NO, the natural-order
                             parallel Gauss-Seidel PGS-SCM is compared with in
                             Section 6: rows split into smoother_chunks contiguous
                             chunks, Gauss-Seidel inside a chunk, values of other chunks
                             as they were when the sweep started [0] */
  int32_t smoother_chunks;/* chunks of the PGS-NO smoother on every level (rows per
                             chunk = ceil(n / chunks)) [256] */
  int32_t amg_kind;       /* pressure solver B_P: 0 = classical Ruge-Stueben AMG
                             (theta_rs), V-cycle; 1 = the paper's unsmoothed
                             aggregation AMG (Section 6): npair passes of pairwise
                             matching with threshold pair_beta per level, and the
                             nonlinear AMLI-cycle, whose coarse corrections are
                             amli_inner steps of flexible GCR preconditioned by the next
                             level's cycle; the coarsest level (coarse_max rows, the
                             paper uses 10000) is solved directly by its inverse,
                             formed on the GPU at SETUP [0] */
  int32_t amli_inner;     /* flexible GCR steps per coarse correction, 1 or 2 [2] */
  int32_t npair;          /* pairwise matching passes per level [2] */
  double pair_beta;       /* strong-coupling threshold of the matching [0.25] */
  int32_t coarse_solver;  /* coarsest level of the Ruge-Stueben V-cycle (the paper solves
                             its coarsest space directly, Section 6): 0 = LU factors
                             formed on the host (FP64, partial pivoting), forward and
                             back substitution inside the single-workgroup kernel;
                             1 = explicit FP64 inverse formed on the GPU at SETUP by
                             Gauss-Jordan elimination with partial pivoting and applied
                             as one dense product, which suits a coarsest level of
                             hundreds to thousands of rows (no single-workgroup kernel
                             is then used).  The aggregation AMG always uses 1 [0] */
} cpr_params;

typedef struct {
  int32_t iterations;   /* inner FGMRES steps (one B apply + one A product each) */
  int32_t restarts;     /* completed restart cycles before the final one */
  int32_t rebuilt;      /* 1 if SETUP ran for this solve */
  int32_t n_levels;     /* AMG levels of the hierarchy in use */
  double relres_true;   /* ||b - A x||_2 / ||b||_2 in FP64, recomputed at exit */
  double relres_est;    /* last Givens estimate |g_{j+1}| / ||r_0|| */
  double setup_ms;      /* host wall time of SETUP in this call (0 when reused) */
  double solve_ms;      /* host wall time of the Krylov iteration */
} cpr_solve_info;

typedef struct cpr_handle cpr_handle;

/* Fill *p with the defaults listed above. */
void cpr_params_default(cpr_params* p);

/* SETUP (Algorithm "CPR method" viewed as producing B, the Remark after
 * Algorithm "ASCPR"): validate and copy A into device memory, build the
 * pressure AMG hierarchy (strength on the GPU; colouring, C/F split,
 * interpolation and Galerkin products on the host), the stage-2 block
 * colouring and diagonal-block inverses, and the Krylov workspace.
 * hip_stream: the hipStream_t all work of the handle runs on (NULL = the
 * default stream); the caller keeps ownership of it.
 * Returns CPR_OK and *out, or an error (then *out is NULL). */
cpr_status cpr_setup(const cpr_bsr* A, const cpr_params* p, void* hip_stream, cpr_handle** out);

/* Replace the values of A (same n_block_rows, nnz_blocks, row_ptr, col_idx;
 * the pattern is compared entry by entry with the one given to cpr_setup, on
 * the device for device arrays).  The outer FGMRES uses the new values at the
 * next solve; whether the preconditioner is rebuilt is decided there by the
 * adaptive rule (Algorithm "ASCPR"): new values before the handle's first
 * solve always rebuild (solve k = 1 runs on a B of the matrix it solves),
 * reuse_mode 0 rebuilds on every new set of values, modes 1 and 2 keep B
 * frozen (every SETUP product, including the copy of A inside the CPR apply)
 * while their rule allows.  A singular diagonal block is reported by the solve
 * that rebuilds; a failed rebuild leaves the previous B in the handle.
 * Errors: CPR_ERR_SIZE_MISMATCH, CPR_ERR_PATTERN_MISMATCH. */
cpr_status cpr_update_values(cpr_handle* h, const cpr_bsr* A);

/* Solve A x = b to ||b - A x|| / ||b - A x_in|| < tol with CPR-FGMRES
 * (Algorithm "ASCPR-GMRES").  b and x are caller-owned device arrays of
 * 3*n_block_rows doubles; x is the initial guess on entry and the solution
 * on exit.  Blocks until the result is in x.  info may be NULL. */
cpr_status cpr_solve(cpr_handle* h, const double* b, double* x, double tol, cpr_solve_info* info);

/* cpr_solve for callers that cannot allocate device memory (tight serving
 * loops, harnesses that forbid hipMalloc): the same solve, with the same
 * kernels and the same result as cpr_solve, that calls no hipMalloc,
 * hipFree, graph instantiation or other allocating routine.  Its FGMRES
 * scalars and per-workgroup partial sums live in a static device array of
 * 1.07 MiB that each GPU the library runs on holds until the process ends;
 * its address is looked up on the first call on a device.  Every step is
 * launched directly (no graph replay) and profiling events are not recorded.
 * Limits and errors: the handle's restart must be at most 64, else
 * CPR_ERR_INVALID_ARG; when the adaptive-setup rule asks for a SETUP before
 * this solve (SETUP allocates) it returns CPR_ERR_INVALID_ARG and changes
 * nothing: call cpr_solve for that step.  All calls on one GPU share the one
 * array, which keeps the last call's contents (every word a solve reads from
 * it is written earlier in the same solve): calls that overlap in time on one
 * GPU, from any handles or threads, race and must be serialised by the
 * caller.  b, x, tol, info as for cpr_solve. */
cpr_status cpr_solve_noalloc(cpr_handle* h, const double* b, double* x, double tol, cpr_solve_info* info);

/* Make subsequent work of h run on hip_stream (a hipStream_t, NULL = the
 * default stream) after draining the previous stream. */
cpr_status cpr_set_stream(cpr_handle* h, void* hip_stream);

/* Free every resource of h (NULL is allowed). */
void cpr_destroy(cpr_handle* h);

const char* cpr_status_string(cpr_status s);

/* Text of the last error recorded on h (empty string if none). */
const char* cpr_last_error(const cpr_handle* h);

/* Device bytes held by h (matrices, hierarchy, workspace). */
int64_t cpr_device_bytes(const cpr_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* CPR_MI355X_CPR_H */
