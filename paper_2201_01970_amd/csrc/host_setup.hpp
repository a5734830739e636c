// Host-side SETUP algorithms of the CPR preconditioner.
//
// The greedy steps of SETUP are sequential by nature (the paper's Section 3.2
// lists this as shortcoming (ii) of CPR), so they run on the host:
//   * VerticesSplitting / VerticesGrouping (Section 5.2) on a strength pattern;
//   * classical Ruge-Stueben C/F splitting, interpolation and the Galerkin
//     product for the pressure AMG;
//   * a dense LU with partial pivoting for the coarsest level.
// Every result that the solve phase consumes must be reproducible bit for bit,
// so tie-breaks and summation orders are fixed and documented per function;
// this file is compiled with -ffp-contract=off.
#pragma once

#include <cstdint>
#include <functional>
#include <memory>
#include <new>
#include <type_traits>
#include <utility>
#include <vector>

namespace cpr {

// Allocator whose resize() leaves new elements uninitialised: the SETUP
// arrays (hundreds of MB at 3.28M DOF) are written in full by parallel passes
// right after they are sized, and zero-filling them first cost a serial pass
// plus every page fault on one thread.
template <typename T>
struct NoInitAlloc : std::allocator<T> {
  template <typename U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <typename U>
  NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <typename U>
  void construct(U* p) noexcept(std::is_nothrow_default_constructible<U>::value) {
    ::new (static_cast<void*>(p)) U;
  }
  template <typename U, typename... Args>
  void construct(U* p, Args&&... args) {
    ::new (static_cast<void*>(p)) U(std::forward<Args>(args)...);
  }
};
template <typename T>
using HostVec = std::vector<T, NoInitAlloc<T>>;

struct HostCsr {
  int32_t n_rows = 0, n_cols = 0;
  HostVec<int32_t> ptr, col;  // resize() leaves entries uninitialised
  HostVec<double> val;
  int64_t nnz() const { return static_cast<int64_t>(col.size()); }
};

// Pattern rows (strong neighbours) extracted from a mask over stored entries.
struct Pattern {
  int32_t n = 0;
  HostVec<int32_t> ptr, col;  // resize() leaves entries uninitialised
};

Pattern pattern_from_mask(const HostCsr& A, const std::vector<uint8_t>& mask, uint8_t bit);
Pattern transpose_pattern(const Pattern& S);

// Algorithm VerticesGrouping.  Selection: largest |S_i| (static row count of
// S), ties to the smallest index; the frontier (second circle of each vertex
// put in W) is searched first while it holds an undecided vertex; a vertex
// joins W iff none of its S-row neighbours is in W, in which case its
// undecided S-row neighbours join W-bar and the undecided vertices of its
// second circle join the frontier; otherwise it joins W-bar.  Colours are
// numbered in creation order.  Returns the number of colours.
int32_t vertices_grouping(const Pattern& S, std::vector<int32_t>& colour);

// Classical RS split.  cf: 1 = C, 2 = F.
//  first pass: isolated points (S_i and S^T_i empty) are F; the rest start
//  undecided with lambda_i = |S^T_i|; while the largest undecided lambda is
//  positive, take that point (ties: smallest index) as C, make its undecided
//  dependents (S^T_i) F and give every undecided k in S_j of each new F point
//  j lambda_k += 1, then lambda_j -= 1 for every undecided j in S_i.
//  Leftovers (ascending) become F if a strong dependency is C, else C.
//  second pass: F points ascending; a strong F dependency j of F point i
//  whose S_j misses C_i (strong C dependencies of i) makes j a tentative C
//  point; a second such j turns i into C and sends the tentative one back.
void rs_split(const Pattern& S, const Pattern& ST, std::vector<int8_t>& cf);

// Classical RS interpolation; see the order of operations in host_setup.cpp.
// Returns false if a denominator a_ii + (weak sum) is zero.
bool rs_interpolation(const HostCsr& A, const std::vector<uint8_t>& strong_mask, uint8_t bit,
                      const std::vector<int8_t>& cf, HostCsr& P);

// Explicit transpose; rows of the result list columns ascending.
HostCsr transpose(const HostCsr& A);

// C = A B: for row i, for k in row i of A (stored order), for j in row k of B
// (stored order), c_ij = c_ij + a_ik*b_kj starting from 0.0; every result row
// is sorted by column; no entry is dropped.
HostCsr spgemm_ordered(const HostCsr& A, const HostCsr& B);

// Dense LU with partial pivoting (row-major n x n, in place), pivot row
// indices in piv.  Returns false when a pivot is exactly zero.
bool dense_lu(int32_t n, std::vector<double>& a, std::vector<int32_t>& piv);

// Block ILU(0) of a 3x3-block matrix (the second stage R of eq. (CPR) that
// Section 3.1 names, with the level scheduling of Section 6), natural row
// order, no fill: the factors keep A's block pattern.  IKJ form: for each row
// i ascending, for each stored k < i ascending, L_ik = A_ik Uinv_k, then
// A_ij -= L_ik U_kj for every stored j > k of row k that row i also stores;
// then Uinv_i = inverse of the updated diagonal block (LU with partial
// pivoting of the 3x3 block, then its inverse column by column).  A 3x3
// product c = a b sums each entry from 0.0 over m = 0, 1, 2.  Rows of one
// forward level depend only on rows of earlier levels, so the levels are
// factored one after another, their rows in parallel.
//   rp, col: the block pattern (sorted columns, diagonal stored);
//   lu: on entry the blocks of A (nnz x 9, row-major), on exit L_ik (k < i)
//       and U_ij (j >= i);  uinv: n x 9;  flev: forward level of every row.
// Returns the first row whose pivot block is singular (a pivot below 1e-300
// times the block's largest entry), or -1.
int32_t bilu0_factor(int32_t n, const int32_t* rp, const int32_t* col, const std::vector<int32_t>& flev,
                     double* lu, double* uinv);

// Level of every row in the forward (lower) and backward (upper) triangular
// solve: 0 when the row has no stored entry on that side, else one more than
// the largest level among those entries.  Returns the number of levels.
int32_t bilu_forward_levels(int32_t n, const int32_t* rp, const int32_t* col, std::vector<int32_t>& lev);
int32_t bilu_backward_levels(int32_t n, const int32_t* rp, const int32_t* col, std::vector<int32_t>& lev);

// Inverse of a 3x3 block (row-major) by LU with partial pivoting, then the
// inverse column by column; false when a pivot is at most 1e-300 times the
// block's largest entry.
bool inverse3(const double* a, double* inv);

// Pairwise matching (one pass) of unsmoothed-aggregation AMG (the paper's
// NPAIR aggregation, Section 6).  Couplings s_ij = a_ij/2 + a_ji/2 (the half
// of the lower-numbered row added first, a missing entry counting as 0);
// S_i = {j != i : s_ij < -beta * max_k(-s_ik)} when that maximum is positive;
// m_i = number of unaggregated rows k with i in S_k.  Repeatedly the
// unaggregated row i of smallest m_i (ties: smallest index) is paired with its
// unaggregated j in S_i of most negative s_ij (ties: smallest index), or left
// alone; aggregates are numbered in formation order.  agg[i] = aggregate of
// row i; returns the aggregate count.
int32_t pairwise_matching(const HostCsr& A, double beta, std::vector<int32_t>& agg);

// npair successive matching passes (the second on P_1^T A P_1, formed by
// transpose and spgemm_ordered); agg composes the passes.
int32_t npair_aggregates(const HostCsr& A, double beta, int npair, std::vector<int32_t>& agg);

// The 0/1 prolongation of an aggregation (row i: a 1 in column agg[i]).
HostCsr aggregation_matrix(const std::vector<int32_t>& agg, int32_t n_agg);

// Host threads used by the row-parallel SETUP steps (at most 16).
int setup_threads();

// Runs f(chunk, slot) for chunk = 0..n_chunks-1 on the SETUP thread pool
// (the calling thread takes part); slot < min(setup_threads(), n_chunks)
// indexes per-call scratch.  Returns when every chunk has finished.
void parallel_for(int n_chunks, const std::function<void(int, int)>& f);

}  // namespace cpr
