// SETUP pipeline and the FP64 flexible GMRES driver with the adaptive-setup
// rule (Section 4, Algorithms "ASCPR-GMRES" and "ASCPR").
#include "solver.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <future>
#include <limits>
#include <numeric>

namespace cpr {

std::mutex& device_api_mutex() {
  static std::mutex m;
  return m;
}

void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e == hipSuccess) return;
  (void)hipGetLastError();
  const cpr_status st = (e == hipErrorOutOfMemory) ? CPR_ERR_OOM : CPR_ERR_HIP;
  throw Error(st, std::string(hipGetErrorString(e)) + " in " + what + " (" + file + ":" + std::to_string(line) + ")");
}

// ------------------------------------------------------------------ profiler
Profiler::~Profiler() {
  for (auto& r : pending_) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : free_) (void)hipEventDestroy(e);
  for (hipEvent_t e : open_ev_)
    if (e) (void)hipEventDestroy(e);
}

void Profiler::enable(bool on) {
  on_ = on;
  if (on)
    for (int k = 0; k < CPR_KSTAT_COUNT; ++k) {
      launches[k] = 0;
      total_ms[k] = 0.0;
      bytes[k] = 0.0;
    }
}

hipEvent_t Profiler::get_event() {
  if (!free_.empty()) {
    hipEvent_t e = free_.back();
    free_.pop_back();
    return e;
  }
  // Timing-only events: without the system-scope fence a recorded event
  // otherwise performs (a cache writeback and invalidation that would both
  // lengthen the measured interval and slow the next kernel); the profiler
  // reads them after synchronising the stream.
  hipEvent_t e;
  std::lock_guard<std::mutex> lk(device_api_mutex());
  HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  return e;
}

void Profiler::begin(int kind, hipStream_t s) {
  if (!on_) return;
  hipEvent_t e = get_event();
  HIPCHK(hipEventRecord(e, s));
  open_ev_[kind] = e;
}

void Profiler::end(int kind, hipStream_t s, double b) {
  if (!on_ || !open_ev_[kind]) return;
  hipEvent_t e = get_event();
  HIPCHK(hipEventRecord(e, s));
  pending_.push_back({kind, open_ev_[kind], e, b});
  open_ev_[kind] = nullptr;
}

void Profiler::collect() {
  for (auto& r : pending_) {
    HIPCHK(hipEventSynchronize(r.b));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    launches[r.kind] += 1;
    total_ms[r.kind] += ms;
    bytes[r.kind] += r.bytes;
    free_.push_back(r.a);
    free_.push_back(r.b);
  }
  pending_.clear();
}

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Rows of each colour in index order; returns the permutation (device
// position -> row) and colour offsets.  Index order keeps rows that are close
// in the grid close on the device, so the rows a workgroup takes share most
// of the vector entries they gather (sorting a colour by row length instead
// scatters them: 10% more solve time at 3.28M DOF).
void colour_order(int32_t n, const std::vector<int32_t>& colour, int32_t ncol, std::vector<int32_t>& perm,
                  std::vector<int32_t>& coff) {
  coff.assign(ncol + 1, 0);
  for (int32_t i = 0; i < n; ++i) coff[colour[i] + 1]++;
  for (int32_t c = 0; c < ncol; ++c) coff[c + 1] += coff[c];
  std::vector<int32_t> next(coff.begin(), coff.end() - 1);
  perm.resize(n);
  for (int32_t i = 0; i < n; ++i) perm[next[colour[i]]++] = i;
}

// Greedy colouring of one level (Algorithm VerticesGrouping) and its device
// row order; independent of the coarsening, so it runs on its own thread.
struct Colouring {
  std::vector<int32_t> colour, perm, coff;
  int32_t n_colours = 0;
};

Colouring colour_level(const Pattern& S) {
  Colouring c;
  c.n_colours = vertices_grouping(S, c.colour);
  colour_order(S.n, c.colour, c.n_colours, c.perm, c.coff);
  return c;
}

}  // namespace

}  // namespace cpr

using namespace cpr;

// ------------------------------------------------------------------ SETUP
// Pressure extraction (A_PP = Pi_P^T A Pi_P, the (0,0) entry of every stored
// block), then per level: strength masks on the GPU, RS split, interpolation
// and Galerkin product on the host, until the level is small enough; the
// colouring of every smoothed level (Algorithm VerticesGrouping on eq.
// (strong-matrix)) and the stage-2 block colouring (theta = 0 on the block
// graph) run on threads of their own meanwhile; then the coarsest LU and the
// device images.
void cpr_handle::build_precond() {
  const double t0 = now_ms();
  drop_graphs();
  // Everything is built into locals and swapped into the handle only when the
  // whole SETUP succeeded: a failed rebuild leaves the previous B in place.
  std::vector<HostLevel> hl;

  // SETUP's view of the values, prepared on the device from the handle's
  // copy of A: the pressure entry of every block, which blocks hold a nonzero
  // entry, and the first cell whose diagonal block admits no LU with partial
  // pivoting whose pivots exceed 1e-300 times the block's largest entry (the
  // test of the device inversion, made first so that no other SETUP step sees
  // a singular block).  67 MB come back to the host at 3.28M DOF instead of
  // the 534 MB of values.
  // Decoupling: B is built on W A (computed here on the device, freed once
  // the preconditioner holds its own images) and applied to W v.
  Arena dec;
  const double* d_vals_pc = d_vals_in;
  double* d_w = nullptr;
  if (prm.decoupling != 0) {
    d_w = dec.alloc<double>(static_cast<int64_t>(n_b) * 9);
    double* d_wa = dec.alloc<double>(static_cast<int64_t>(nnz_b) * 9);
    int32_t* d_bad = dec.alloc<int32_t>(1);
    int32_t bad = std::numeric_limits<int32_t>::max();
    HIPCHK(hipMemcpyAsync(d_bad, &bad, sizeof(int32_t), hipMemcpyHostToDevice, stream));
    launch_decouple(n_b, d_rp_pat, d_col_pat, d_vals_in, prm.decoupling, d_w, d_wa, d_bad, stream);
    HIPCHK(hipMemcpyAsync(&bad, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    if (bad != std::numeric_limits<int32_t>::max())
      throw Error(CPR_ERR_SINGULAR_BLOCK,
                  "the decoupling weights of cell " + std::to_string(bad) + " cannot be formed (singular diagonal block)");
    d_vals_pc = d_wa;
  }

  HostVec<double> pval(nnz_b);
  HostVec<uint8_t> nonzero(nnz_b);
  int32_t bad_row = std::numeric_limits<int32_t>::max();
  {
    Arena scratch;
    double* d_pval = scratch.alloc<double>(nnz_b);
    uint8_t* d_nonzero = scratch.alloc<uint8_t>(nnz_b);
    int32_t* d_bad = scratch.alloc<int32_t>(1);
    HIPCHK(hipMemcpyAsync(d_bad, &bad_row, sizeof(int32_t), hipMemcpyHostToDevice, stream));
    launch_setup_values(n_b, d_rp_pat, d_col_pat, d_vals_pc, d_pval, d_nonzero, d_bad, stream);
    HIPCHK(hipMemcpyAsync(pval.data(), d_pval, pval.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipMemcpyAsync(nonzero.data(), d_nonzero, nonzero.size(), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipMemcpyAsync(&bad_row, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
  }
  if (bad_row != std::numeric_limits<int32_t>::max())
    throw Error(CPR_ERR_SINGULAR_BLOCK, "diagonal block of cell " + std::to_string(bad_row) + " is singular");

  // The colourings depend only on each level's matrix and strength mask, not
  // on the coarsening that follows, so they run on threads of their own while
  // the levels are built: first the stage-2 block colouring (theta = 0 on the
  // block graph: every stored nonzero off-diagonal block couples two cells),
  // or, for the block ILU(0) second stage, the factorisation.
  const bool use_bilu = prm.second_stage == 1;
  std::future<HostBilu> bilu_task;
  if (use_bilu)
    bilu_task = std::async(std::launch::async, [this, d_vals_pc]() {
      HostBilu F;
      F.lu.resize(static_cast<size_t>(nnz_b) * 9);
      {
        std::lock_guard<std::mutex> lk(device_api_mutex());
        HIPCHK(hipMemcpy(F.lu.data(), d_vals_pc, F.lu.size() * sizeof(double), hipMemcpyDeviceToHost));
      }
      F.acol0.resize(static_cast<size_t>(nnz_b) * 3);
      for (int64_t k = 0; k < nnz_b; ++k)
        for (int r = 0; r < 3; ++r) F.acol0[3 * k + r] = F.lu[9 * k + 3 * r];
      F.n_flev = bilu_forward_levels(n_b, h_row_ptr.data(), h_col.data(), F.flev);
      F.n_blev = bilu_backward_levels(n_b, h_row_ptr.data(), h_col.data(), F.blev);
      F.uinv.resize(static_cast<size_t>(n_b) * 9);
      const int32_t bad = bilu0_factor(n_b, h_row_ptr.data(), h_col.data(), F.flev, F.lu.data(), F.uinv.data());
      if (bad >= 0)
        throw Error(CPR_ERR_SINGULAR_BLOCK, "block ILU(0) pivot block of cell " + std::to_string(bad) + " is singular");
      return F;
    });
  auto block_task = std::async(std::launch::async, [this, &nonzero, use_bilu]() {
    if (use_bilu) return Colouring{};
    Pattern B;
    B.n = n_b;
    B.ptr.assign(n_b + 1, 0);
    for (int32_t i = 0; i < n_b; ++i) {
      for (int32_t k = h_row_ptr[i]; k < h_row_ptr[i + 1]; ++k) {
        const int32_t j = h_col[k];
        if (j != i && nonzero[k]) B.col.push_back(j);
      }
      B.ptr[i + 1] = static_cast<int32_t>(B.col.size());
    }
    return colour_level(B);
  });
  std::vector<std::future<Colouring>> level_tasks;
  // SETUP phase times (ms), printed to stderr when CPR_SETUP_TRACE is set
  double t_strength = 0, t_split = 0, t_interp = 0, t_galerkin = 0;
  const double t_loop0 = now_ms();

  HostCsr A;
  A.n_rows = A.n_cols = n_b;
  A.ptr.assign(h_row_ptr.begin(), h_row_ptr.end());
  A.col.assign(h_col.begin(), h_col.end());
  A.val = std::move(pval);

  Arena tmp;
  int32_t *d_ptr = nullptr, *d_col = nullptr;
  double* d_val = nullptr;
  uint8_t* d_mask = nullptr;
  int64_t cap_n = 0, cap_nnz = 0;
  while (true) {
    HostLevel L;
    L.A = std::move(A);
    const int32_t n = L.A.n_rows;
    const bool last = n <= prm.coarse_max || static_cast<int>(hl.size()) + 1 >= prm.max_levels;
    if (last) {
      hl.push_back(std::move(L));
      break;
    }
    // strength masks on the device
    if (n + 1 > cap_n || L.A.nnz() > cap_nnz) {
      tmp.release();
      cap_n = n + 1;
      cap_nnz = std::max<int64_t>(1, L.A.nnz());
      d_ptr = tmp.alloc<int32_t>(cap_n);
      d_col = tmp.alloc<int32_t>(cap_nnz);
      d_val = tmp.alloc<double>(cap_nnz);
      d_mask = tmp.alloc<uint8_t>(cap_nnz);
    }
    double tp = now_ms();
    HIPCHK(hipMemcpyAsync(d_ptr, L.A.ptr.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(d_col, L.A.col.data(), L.A.nnz() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(d_val, L.A.val.data(), L.A.nnz() * sizeof(double), hipMemcpyHostToDevice, stream));
    launch_strength(n, d_ptr, d_col, d_val, prm.theta_rs, prm.theta_color, d_mask, stream);
    L.mask.resize(L.A.nnz());
    HIPCHK(hipMemcpyAsync(L.mask.data(), d_mask, L.A.nnz(), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    t_strength += now_ms() - tp;
    tp = now_ms();

    // colouring of this level (eq. (strong-matrix) pattern) on its own thread
    level_tasks.push_back(
        std::async(std::launch::async, [Sc = pattern_from_mask(L.A, L.mask, 2)]() { return colour_level(Sc); }));
    int32_t nc = 0;
    if (prm.amg_kind == 1) {
      // unsmoothed aggregation: npair passes of pairwise matching, P of 0/1
      nc = npair_aggregates(L.A, prm.pair_beta, prm.npair, L.agg);
    } else {
      const Pattern S = pattern_from_mask(L.A, L.mask, 1);
      const Pattern ST = transpose_pattern(S);
      rs_split(S, ST, L.cf);
      for (int8_t c : L.cf) nc += (c == 1);
    }
    t_split += now_ms() - tp;
    if (nc == 0 || static_cast<double>(nc) > 0.9 * n) {
      // coarsening stalled: this level becomes the coarsest and is not smoothed
      level_tasks.pop_back();
      L.cf.clear();
      L.agg.clear();
      hl.push_back(std::move(L));
      break;
    }
    tp = now_ms();
    if (prm.amg_kind == 1)
      L.P = aggregation_matrix(L.agg, nc);
    else if (!rs_interpolation(L.A, L.mask, 1, L.cf, L.P))
      throw Error(CPR_ERR_SINGULAR_COARSE, "zero interpolation denominator");
    t_interp += now_ms() - tp;
    tp = now_ms();
    const HostCsr R = transpose(L.P);
    const HostCsr AP = spgemm_ordered(L.A, L.P);
    A = spgemm_ordered(R, AP);
    t_galerkin += now_ms() - tp;
    hl.push_back(std::move(L));
  }
  tmp.release();

  const double t_loop = now_ms() - t_loop0;
  double tp = now_ms();
  const int nl = static_cast<int>(hl.size());
  for (int l = 0; l < nl; ++l) {
    HostLevel& L = hl[l];
    if (l + 1 < nl && prm.smoother == 1) {
      // PGS-NO: rows stay in natural order, one class holding them all
      (void)level_tasks[l].get();
      const int32_t n = L.A.n_rows;
      L.colour.assign(n, 0);
      L.n_colours = 1;
      L.perm.resize(n);
      std::iota(L.perm.begin(), L.perm.end(), 0);
      L.coff = {0, n};
    } else if (l + 1 < nl) {
      Colouring c = level_tasks[l].get();
      L.colour = std::move(c.colour);
      L.n_colours = c.n_colours;
      L.perm = std::move(c.perm);
      L.coff = std::move(c.coff);
    } else {
      L.perm.resize(L.A.n_rows);
      std::iota(L.perm.begin(), L.perm.end(), 0);
    }
  }
  // coarsest level, dense (FP64): LU-factored here for the single-workgroup
  // kernel; left unfactored when its inverse is formed on the device
  const bool coarse_inverse = prm.amg_kind == 1 || prm.coarse_solver == 1;
  const HostCsr& Ac = hl.back().A;
  const int32_t nc = Ac.n_rows;
  const int32_t dense_max = coarse_inverse ? 16384 : 8192;
  if (nc > dense_max)
    throw Error(CPR_ERR_INVALID_ARG, "the coarsest level has " + std::to_string(nc) + " rows, more than the " +
                                         std::to_string(dense_max) +
                                         " its dense direct solve takes (coarsening stalled, or coarse_max too large)");
  std::vector<double> lu(static_cast<size_t>(nc) * nc, 0.0);
  for (int32_t i = 0; i < nc; ++i)
    for (int32_t q = Ac.ptr[i]; q < Ac.ptr[i + 1]; ++q) lu[static_cast<size_t>(i) * nc + Ac.col[q]] += Ac.val[q];
  std::vector<int32_t> piv;
  if (!coarse_inverse && !dense_lu(nc, lu, piv))
    throw Error(CPR_ERR_SINGULAR_COARSE, "coarsest matrix is singular");

  // stage-2 block colouring or factorisation (computed on its own thread since the start)
  Colouring bc = block_task.get();
  HostBilu bf;
  if (use_bilu) bf = bilu_task.get();
  const double t_colour_wait = now_ms() - tp;
  tp = now_ms();
  std::vector<int32_t> bperm = std::move(bc.perm), bcoff = std::move(bc.coff);

  std::unique_ptr<PrecondBase> npc = make_precond(prm.precond_fp32 != 0, prm, n_b, hl, lu, piv, bperm, bcoff,
                                                  h_row_ptr, h_col, bc.colour, d_vals_pc, use_bilu ? &bf : nullptr,
                                                  d_w, stream);
  npc->timer = &prof;
  HIPCHK(hipStreamSynchronize(stream));
  pc = std::move(npc);
  this->hl.swap(hl);
  block_colour = std::move(bc.colour);
  n_block_colours = bc.n_colours;
  bilu_host = std::move(bf);
  values_changed = false;
  last_setup_ms = now_ms() - t0;
  if (std::getenv("CPR_SETUP_TRACE"))
    std::fprintf(stderr,
                 "[cpr setup] %.1f ms: levels %.1f (strength %.1f, split %.1f, interpolation %.1f, galerkin %.1f), "
                 "colouring wait %.1f, LU + device images %.1f\n",
                 last_setup_ms, t_loop, t_strength, t_split, t_interp, t_galerkin, t_colour_wait, now_ms() - tp);
}

void cpr_handle::spmv(const double* x, double* y) {
  launch_bsr_spmv<double, double>(outer.view(), x, nullptr, y, stream);
}

// Capture step j once; returns null (and leaves no error behind) when the
// runtime refuses the capture, in which case the step runs eagerly.
hipGraphExec_t cpr_handle::capture_step(int j) {
  std::lock_guard<std::mutex> lk(device_api_mutex());
  if (!cap_stream) HIPCHK(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  bool ok = true;
  try {
    step_body(j, kw, false, cap_stream);
  } catch (const Error&) {
    ok = false;
  }
  const hipError_t e_end = hipStreamEndCapture(cap_stream, &graph);
  hipGraphExec_t exec = nullptr;
  if (ok && e_end == hipSuccess && graph) {
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) exec = nullptr;
  }
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipGetLastError();
  return exec;
}

void cpr_handle::drop_graphs() {
  for (hipGraphExec_t& g : step_graph)
    if (g) (void)hipGraphExecDestroy(g);
  step_graph.clear();
}

// One FGMRES step j: z_j = B v_j; w = A z_j (written into v_{j+1});
// h_ij = (w, v_i) for i <= j (all against the same w: classical Gram-Schmidt);
// w -= sum h_ij v_i; h_{j+1,j} = ||w||; Givens update; v_{j+1} = w / h_{j+1,j};
// then |g_{j+1}| and h_{j+1,j} are copied to the host.
void cpr_handle::step_body(int j, const KrylovWork& w_, bool timed, hipStream_t s) {
  const int64_t N = 3 * static_cast<int64_t>(n_b);
  const int64_t ld = N;
  const int grid = krylov_grid(N);
  const bool f32 = pc->fp32();
  double* vj = V + j * ld;
  double* w = V + (j + 1) * ld;
  void* zj = f32 ? static_cast<void*>(static_cast<float*>(Z) + j * ld)
                 : static_cast<void*>(static_cast<double*>(Z) + j * ld);
  LaunchTimer* const saved_timer = pc->timer;
  if (!timed) pc->timer = nullptr;
  pc->apply(vj, zj, s);
  pc->timer = saved_timer;
  if (timed) prof.begin(CPR_KSTAT_SPMV, s);
  if (f32)
    launch_bsr_spmv<double, float>(outer.view(), static_cast<const float*>(zj), nullptr, w, s);
  else
    launch_bsr_spmv<double, double>(outer.view(), static_cast<const double*>(zj), nullptr, w, s);
  if (timed)
    prof.end(CPR_KSTAT_SPMV, s, 9.0 * nnz_b * 8 + 4.0 * nnz_b + 4.0 * (n_b + 1) + 3.0 * n_b * ((f32 ? 4 : 8) + 8));
  launch_multidot(N, w, V, ld, 0, j + 1, w_.partial, s);
  double* Hj = w_.H + static_cast<int64_t>(j) * (m + 1);
  launch_reduce_partials(w_.partial, grid, j + 1, Hj, s);
  launch_axpy_norm(N, w, V, ld, 0, j + 1, Hj, w_.norm_partial, s);
  launch_givens(m, j, w_.norm_partial, grid, w_.H, w_.cs, w_.sn, w_.g, w_.hnorm, w_.report, s);
  launch_scale_div(N, w, w_.hnorm, w, s);
  HIPCHK(hipMemcpyAsync(report_h, w_.report, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
}

// ------------------------------------------------------------------ SOLVE
// Flexible GMRES(m), classical Gram-Schmidt, Givens rotations.  Convergence:
// ||r|| / ||r_0|| < tol checked on the Givens estimate after every step and
// confirmed with the true residual; iterations = inner steps.
cpr_status cpr_handle::solve(const double* b, double* x, double tol, cpr_solve_info* info, const KrylovWork& kwork,
                             bool may_allocate) {
  // adaptive setup (Algorithm "ASCPR"); SETUP of cpr_setup counts as k = 1
  // k counts solves since the handle's SETUP.  Solve k = 1 always runs on a B
  // built from the matrix it solves: cpr_setup built it, unless new values
  // arrived before this first solve, in which case SETUP runs again.
  const int64_t k_this = k_solves + 1;
  bool rebuild = false;
  if (values_changed) {
    if (k_this == 1 || prm.reuse_mode == 0)
      rebuild = true;
    else if (prm.reuse_mode == 1)
      rebuild = !(it_prev <= prm.mu);
    else
      rebuild = !(static_cast<double>(it_prev) <= prm.reuse_factor * static_cast<double>(it_ref));
  }
  if (rebuild && !may_allocate)
    throw Error(CPR_ERR_INVALID_ARG,
                "the adaptive-setup rule asks for a SETUP before this solve, and SETUP allocates: call cpr_solve");
  k_solves = k_this;
  const bool timed = may_allocate && prof.on();
  double setup_ms = 0.0;
  if (rebuild) {
    build_precond();
    setup_ms = last_setup_ms;
  } else if (k_solves == 1) {
    setup_ms = 0.0;
  }
  const bool fresh = rebuild || k_solves == 1;

  const double t0 = now_ms();
  const int64_t N = 3 * static_cast<int64_t>(n_b);
  const int grid = krylov_grid(N);
  const bool f32 = pc->fp32();
  const int64_t ld = N;
  auto sync_report = [&]() {
    HIPCHK(hipMemcpyAsync(report_h, kwork.report, 4 * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
  };
  auto outer_spmv_resid = [&](const double* xx, const double* bb, double* rr) {
    if (timed) prof.begin(CPR_KSTAT_SPMV, stream);
    launch_bsr_spmv<double, double>(outer.view(), xx, bb, rr, stream);
    if (timed)
      prof.end(CPR_KSTAT_SPMV, stream, 9.0 * nnz_b * 8 + 4.0 * nnz_b + 4.0 * (n_b + 1) + 3.0 * n_b * (8 + 8 + 8));
  };

  // ||b|| (for the reported true relative residual), r0 = b - A x0, beta0 = ||r0||
  launch_norm_partial(N, b, kwork.norm_partial, stream);
  launch_reduce_partials(kwork.norm_partial, grid, 1, kwork.report + 2, stream);
  outer_spmv_resid(x, b, r);
  launch_norm_partial(N, r, kwork.norm_partial, stream);
  launch_start_cycle(m, kwork.norm_partial, grid, kwork.g, kwork.hnorm, kwork.report, stream);
  sync_report();
  const double beta0 = report_h[0];
  const double bnorm = std::sqrt(report_h[2]);
  int its = 0, cycles = 0;
  double est = 1.0, rel = 0.0, relb = 0.0;
  cpr_status st = CPR_NOT_CONVERGED;
  if (!std::isfinite(beta0)) {
    last_error = "NaN or Inf in the initial residual";
    st = CPR_ERR_NAN;
  } else if (beta0 == 0.0) {
    st = CPR_OK;
    rel = 0.0;
    est = 0.0;
  } else {
    for (int cycle = 0; cycle < prm.max_restarts; ++cycle) {
      cycles = cycle;
      // v_1 = r / ||r||, g = ||r|| e_1 (start_cycle already ran for this r)
      launch_scale_div(N, r, kwork.hnorm, V, stream);
      int k = 0;
      bool bad = false;
      for (int j = 0; j < m; ++j) {
        if (may_allocate && prm.use_graphs && !prof.on()) {
          if (step_graph.empty()) step_graph.assign(m, nullptr);
          if (!step_graph[j]) step_graph[j] = capture_step(j);
          if (step_graph[j])
            HIPCHK(hipGraphLaunch(step_graph[j], stream));
          else
            step_body(j, kwork, timed, stream);  // capture was refused: same kernels, launched one by one
        } else {
          step_body(j, kwork, timed, stream);
        }
        HIPCHK(hipStreamSynchronize(stream));
        ++its;
        k = j + 1;
        est = report_h[0] / beta0;
        const double hn = report_h[1];
        if (!std::isfinite(est) || !std::isfinite(hn)) {
          bad = true;
          break;
        }
        if (hn == 0.0) break;  // happy breakdown
        if (est < tol) break;
      }
      if (bad) {
        last_error = "NaN or Inf during the Arnoldi process";
        st = CPR_ERR_NAN;
        break;
      }
      launch_backsolve(m, k, kwork.H, kwork.g, kwork.y, stream);
      if (f32)
        launch_update_x<float>(N, x, static_cast<const float*>(Z), ld, k, kwork.y, stream);
      else
        launch_update_x<double>(N, x, static_cast<const double*>(Z), ld, k, kwork.y, stream);
      outer_spmv_resid(x, b, r);
      launch_norm_partial(N, r, kwork.norm_partial, stream);
      launch_start_cycle(m, kwork.norm_partial, grid, kwork.g, kwork.hnorm, kwork.report, stream);
      sync_report();
      rel = report_h[0] / beta0;
      relb = bnorm > 0.0 ? report_h[0] / bnorm : 0.0;
      if (!std::isfinite(rel)) {
        last_error = "NaN or Inf in the true residual";
        st = CPR_ERR_NAN;
        break;
      }
      if (rel < tol) {
        st = CPR_OK;
        break;
      }
    }
  }
  HIPCHK(hipStreamSynchronize(stream));
  if (timed) prof.collect();
  const double solve_ms = now_ms() - t0;

  it_prev = its;
  if (fresh) it_ref = its;

  if (info) {
    info->iterations = its;
    info->restarts = cycles;
    info->rebuilt = rebuild ? 1 : 0;
    info->n_levels = pc->n_levels();
    info->relres_true = relb;
    info->relres_est = est;
    info->setup_ms = setup_ms;
    info->solve_ms = solve_ms;
  }
  if (st == CPR_NOT_CONVERGED) last_error = "not converged within max_restarts";
  return st;
}
