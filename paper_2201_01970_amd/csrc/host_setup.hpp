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

// Host threads used by the row-parallel SETUP steps (at most 16).
int setup_threads();

// Runs f(chunk, slot) for chunk = 0..n_chunks-1 on the SETUP thread pool
// (the calling thread takes part); slot < min(setup_threads(), n_chunks)
// indexes per-call scratch.  Returns when every chunk has finished.
void parallel_for(int n_chunks, const std::function<void(int, int)>& f);

}  // namespace cpr
