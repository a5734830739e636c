// extern "C" entry points: argument checks, exception-to-status translation.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "solver.hpp"

using namespace cpr;

namespace {

thread_local std::string g_last_error;

cpr_status fail(cpr_handle* h, cpr_status st, const std::string& msg) {
  if (h) h->last_error = msg;
  g_last_error = msg;
  return st;
}

template <typename F>
cpr_status guarded(cpr_handle* h, F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    return fail(h, e.status, e.what());
  } catch (const std::bad_alloc&) {
    return fail(h, CPR_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(h, CPR_ERR_HIP, e.what());
  }
}

void copy_in(void* dst, const void* src, size_t bytes, int32_t location) {
  if (bytes == 0) return;
  if (location == CPR_MEM_DEVICE) {
    std::lock_guard<std::mutex> lk(device_api_mutex());
    HIPCHK(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
  } else
    std::memcpy(dst, src, bytes);
}

// Check sizes, ascending columns, range and the diagonal block of every row.
void validate_pattern(int32_t n, int32_t nnz, const HostVec<int32_t>& rp, const HostVec<int32_t>& col) {
  if (rp[0] != 0 || rp[n] != nnz) throw Error(CPR_ERR_INVALID_ARG, "row_ptr must start at 0 and end at nnz_blocks");
  for (int32_t i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) throw Error(CPR_ERR_INVALID_ARG, "row_ptr is not monotone");
    bool diag = false;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      if (col[k] < 0 || col[k] >= n) throw Error(CPR_ERR_INVALID_ARG, "column index out of range");
      if (k > rp[i] && col[k] <= col[k - 1]) throw Error(CPR_ERR_INVALID_ARG, "columns not strictly ascending");
      diag = diag || col[k] == i;
    }
    if (!diag) throw Error(CPR_ERR_INVALID_ARG, "missing diagonal block in row " + std::to_string(i));
  }
}

void check_bsr(const cpr_bsr* A) {
  if (!A || !A->row_ptr || !A->col_idx || !A->values) throw Error(CPR_ERR_INVALID_ARG, "null matrix array");
  if (A->block_dim != 3) throw Error(CPR_ERR_INVALID_ARG, "block_dim must be 3");
  if (A->n_block_rows <= 0 || A->nnz_blocks < A->n_block_rows)
    throw Error(CPR_ERR_INVALID_ARG, "invalid n_block_rows / nnz_blocks");
  if (A->n_block_rows >= (1 << 30)) throw Error(CPR_ERR_INVALID_ARG, "too many block rows");
  if (A->location != CPR_MEM_HOST && A->location != CPR_MEM_DEVICE)
    throw Error(CPR_ERR_INVALID_ARG, "location must be CPR_MEM_HOST or CPR_MEM_DEVICE");
}

// SETUP builds a new preconditioner aside and swaps it in only on success, so
// a handle that cpr_setup returned always holds one; checked anyway before any
// entry point dereferences it.
void need_pc(const cpr_handle* h) {
  if (!h->pc) throw Error(CPR_ERR_INVALID_ARG, "the handle holds no preconditioner");
}

// Outer FP64 block SELL in natural row order; pos[k] = lane-slot of block k.
void build_outer(cpr_handle* h) {
  const int32_t n = h->n_b;
  const int32_t ns = (n + kWave - 1) / kWave;
  std::vector<int32_t> sp(ns + 1, 0);
  for (int32_t s = 0; s < ns; ++s) {
    int32_t w = 0;
    for (int32_t i = s * kWave; i < std::min(n, (s + 1) * kWave); ++i)
      w = std::max(w, h->h_row_ptr[i + 1] - h->h_row_ptr[i]);
    sp[s + 1] = sp[s] + w;
  }
  const int64_t slots = sp[ns];
  HostVec<int32_t> col(static_cast<size_t>(slots) * kWave);  // written in full below
  HostVec<int64_t> pos(h->nnz_b);
  const int nch = static_cast<int>(std::min<int64_t>(256, std::max<int64_t>(1, ns / 64)));
  parallel_for(nch, [&](int ch, int) {
    const int32_t s1 = static_cast<int32_t>(static_cast<int64_t>(ns) * (ch + 1) / nch);
    for (int32_t s = static_cast<int32_t>(static_cast<int64_t>(ns) * ch / nch); s < s1; ++s)
      for (int32_t lane = 0; lane < kWave; ++lane) {
        const int32_t i = s * kWave + lane;
        int32_t k = i < n ? h->h_row_ptr[i] : 0;
        const int32_t k1 = i < n ? h->h_row_ptr[i + 1] : 0;
        for (int32_t t = sp[s]; t < sp[s + 1]; ++t) {
          const size_t e = static_cast<size_t>(t) * kWave + lane;
          if (k < k1) {
            col[e] = h->h_col[k];
            pos[k] = static_cast<int64_t>(e);
            ++k;
          } else {
            col[e] = kPadCol;
          }
        }
      }
  });
  h->outer.n_rows = n;
  h->outer.slots = slots;
  h->outer.slice_ptr = h->fine.upload(sp);
  h->outer.col = h->fine.upload(col);
  h->outer.val = h->fine.alloc<double>(slots * 9 * kWave);
  HIPCHK(hipMemsetAsync(h->outer.val, 0, static_cast<size_t>(slots) * 9 * kWave * sizeof(double), h->stream));
  h->d_pos_outer = h->fine.upload(pos);
}

void alloc_krylov(cpr_handle* h) {
  const int64_t N = 3 * static_cast<int64_t>(h->n_b);
  const int m = h->m;
  h->V = h->fine.alloc<double>((m + 1) * N);
  if (h->prm.precond_fp32)
    h->Z = h->fine.alloc<float>(m * N);
  else
    h->Z = h->fine.alloc<double>(m * N);
  h->kw = krylov_work_carve(h->fine.alloc<double>(krylov_work_doubles(m)), m);
  h->r = h->fine.alloc<double>(N);
  std::lock_guard<std::mutex> lk(device_api_mutex());
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&h->report_h), 4 * sizeof(double), hipHostMallocDefault));
}

}  // namespace

extern "C" {

void cpr_params_default(cpr_params* p) {
  if (!p) return;
  p->restart = 30;
  p->max_restarts = 100;
  p->theta_rs = 0.25;
  p->theta_color = 0.05;
  p->coarse_max = 50;
  p->max_levels = 25;
  p->pre_sweeps = 2;
  p->post_sweeps = 2;
  p->precond_fp32 = 0;
  p->reuse_mode = 2;
  p->mu = 20;
  p->reuse_factor = 1.3;
  p->use_graphs = 1;
  p->tail_nnz = 30000;
  p->row_layout = 0;
  p->second_stage = 0;
  p->decoupling = 0;
  p->smoother = 0;
  p->smoother_chunks = 256;
  p->amg_kind = 0;
  p->amli_inner = 2;
  p->npair = 2;
  p->pair_beta = 0.25;
  p->coarse_solver = 0;
}

cpr_status cpr_setup(const cpr_bsr* A, const cpr_params* p, void* hip_stream, cpr_handle** out) {
  if (!out) return fail(nullptr, CPR_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  cpr_handle* h = nullptr;
  cpr_status st = guarded(nullptr, [&]() -> cpr_status {
    check_bsr(A);
    cpr_params prm;
    cpr_params_default(&prm);
    if (p) prm = *p;
    if (prm.restart < 1 || prm.restart > 256 || prm.max_restarts < 1 || prm.coarse_max < 1 || prm.max_levels < 1 ||
        prm.pre_sweeps < 0 || prm.post_sweeps < 0 || !(prm.theta_rs >= 0.0) || !(prm.theta_color >= 0.0) ||
        prm.reuse_mode < 0 || prm.reuse_mode > 2 || prm.tail_nnz < 0 ||
        !(prm.row_layout == 0 || prm.row_layout == 1 || prm.row_layout == 2 || prm.row_layout == 4 ||
          prm.row_layout == 16 || prm.row_layout == 32 || prm.row_layout == 64) ||
        prm.second_stage < 0 || prm.second_stage > 1 || prm.decoupling < 0 || prm.decoupling > 2 ||
        prm.smoother < 0 || prm.smoother > 1 || prm.smoother_chunks < 1 || prm.amg_kind < 0 || prm.amg_kind > 1 ||
        prm.amli_inner < 1 || prm.amli_inner > 2 || prm.npair < 1 || prm.npair > 4 || !(prm.pair_beta >= 0.0) ||
        prm.coarse_solver < 0 || prm.coarse_solver > 1 || (prm.amg_kind == 1 && prm.smoother != 0))
      throw Error(CPR_ERR_INVALID_ARG, "invalid parameters");
    h = new cpr_handle();
    h->prm = prm;
    h->m = prm.restart;
    HIPCHK(hipGetDevice(&h->device));
    h->stream = static_cast<hipStream_t>(hip_stream);  // NULL = the default stream
    h->n_b = A->n_block_rows;
    h->nnz_b = A->nnz_blocks;
    // phase times (ms), printed to stderr when CPR_SETUP_TRACE is set
    auto clock_ms = []() {
      return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
    };
    const double t0 = clock_ms();
    h->h_row_ptr.resize(h->n_b + 1);
    h->h_col.resize(h->nnz_b);
    copy_in(h->h_row_ptr.data(), A->row_ptr, (h->n_b + 1) * sizeof(int32_t), A->location);
    copy_in(h->h_col.data(), A->col_idx, h->nnz_b * sizeof(int32_t), A->location);
    validate_pattern(h->n_b, h->nnz_b, h->h_row_ptr, h->h_col);
    h->d_rp_pat = h->fine.upload(h->h_row_ptr);
    h->d_col_pat = h->fine.upload(h->h_col);
    h->d_flag = h->fine.alloc<int32_t>(1);
    // the values go straight to the handle's device copy (SETUP reads what it
    // needs of them on the device)
    h->d_vals_in = h->fine.alloc<double>(static_cast<int64_t>(h->nnz_b) * 9);
    {
      std::lock_guard<std::mutex> lk(device_api_mutex());
      HIPCHK(hipMemcpy(h->d_vals_in, A->values, static_cast<size_t>(h->nnz_b) * 9 * sizeof(double),
                       A->location == CPR_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
    }
    const double t1 = clock_ms();
    build_outer(h);
    launch_bsr_values_to_sell<double>(h->nnz_b, h->d_vals_in, h->d_pos_outer, h->outer.val, h->stream);
    const double t2 = clock_ms();
    alloc_krylov(h);
    const double t3 = clock_ms();
    h->build_precond();
    if (std::getenv("CPR_SETUP_TRACE"))
      std::fprintf(stderr,
                   "[cpr setup] input copy, checks and upload %.1f ms, outer SpMV image %.1f, Krylov memory %.1f, "
                   "preconditioner %.1f\n",
                   t1 - t0, t2 - t1, t3 - t2, clock_ms() - t3);
    return CPR_OK;
  });
  if (st != CPR_OK) {
    cpr_destroy(h);
    return st;
  }
  *out = h;
  return CPR_OK;
}

cpr_status cpr_update_values(cpr_handle* h, const cpr_bsr* A) {
  if (!h) return fail(nullptr, CPR_ERR_INVALID_ARG, "null handle");
  return guarded(h, [&]() -> cpr_status {
    check_bsr(A);
    if (A->n_block_rows != h->n_b || A->nnz_blocks != h->nnz_b)
      throw Error(CPR_ERR_SIZE_MISMATCH, "matrix size differs from the handle's (a new SETUP is required)");
    // exact comparison with the SETUP pattern, where the new arrays live
    bool same = true;
    if (A->location == CPR_MEM_DEVICE) {
      // synchronising calls stay exclusive with step-graph captures in other threads
      std::lock_guard<std::mutex> lk(device_api_mutex());
      int32_t diff = 0;
      HIPCHK(hipMemsetAsync(h->d_flag, 0, sizeof(int32_t), h->stream));
      launch_int_diff(h->n_b + 1, A->row_ptr, h->d_rp_pat, h->d_flag, h->stream);
      launch_int_diff(h->nnz_b, A->col_idx, h->d_col_pat, h->d_flag, h->stream);
      HIPCHK(hipMemcpyAsync(&diff, h->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      same = diff == 0;
    } else {
      same = std::equal(A->row_ptr, A->row_ptr + h->n_b + 1, h->h_row_ptr.begin()) &&
             std::equal(A->col_idx, A->col_idx + h->nnz_b, h->h_col.begin());
    }
    if (!same) throw Error(CPR_ERR_PATTERN_MISMATCH, "sparsity pattern differs from the handle's");
    const size_t bytes = static_cast<size_t>(h->nnz_b) * 9 * sizeof(double);
    HIPCHK(hipMemcpyAsync(h->d_vals_in, A->values, bytes,
                          A->location == CPR_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          h->stream));
    launch_bsr_values_to_sell<double>(h->nnz_b, h->d_vals_in, h->d_pos_outer, h->outer.val, h->stream);
    HIPCHK(hipStreamSynchronize(h->stream));
    h->values_changed = true;
    return CPR_OK;
  });
}

cpr_status cpr_solve(cpr_handle* h, const double* b, double* x, double tol, cpr_solve_info* info) {
  if (!h) return fail(nullptr, CPR_ERR_INVALID_ARG, "null handle");
  if (!b || !x || !(tol > 0.0)) return fail(h, CPR_ERR_INVALID_ARG, "b, x must be device arrays and tol > 0");
  return guarded(h, [&]() -> cpr_status {
    need_pc(h);
    return h->solve(b, x, tol, info, h->kw, true);
  });
}

cpr_status cpr_solve_noalloc(cpr_handle* h, const double* b, double* x, double tol, cpr_solve_info* info) {
  if (!h) return fail(nullptr, CPR_ERR_INVALID_ARG, "null handle");
  if (!b || !x || !(tol > 0.0)) return fail(h, CPR_ERR_INVALID_ARG, "b, x must be device arrays and tol > 0");
  if (h->m > kNoAllocMaxRestart)
    return fail(h, CPR_ERR_INVALID_ARG,
                "restart " + std::to_string(h->m) + " exceeds the allocation-free solve's maximum of " +
                    std::to_string(kNoAllocMaxRestart));
  return guarded(h, [&]() -> cpr_status {
    need_pc(h);
    const KrylovWork w = krylov_work_carve(noalloc_scratch(h->device), h->m);
    return h->solve(b, x, tol, info, w, false);
  });
}

cpr_status cpr_set_stream(cpr_handle* h, void* hip_stream) {
  if (!h) return fail(nullptr, CPR_ERR_INVALID_ARG, "null handle");
  return guarded(h, [&]() -> cpr_status {
    HIPCHK(hipStreamSynchronize(h->stream));
    h->stream = static_cast<hipStream_t>(hip_stream);
    return CPR_OK;
  });
}

void cpr_destroy(cpr_handle* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  h->drop_graphs();
  h->pc.reset();
  h->fine.release();
  {
    std::lock_guard<std::mutex> lk(device_api_mutex());
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->report_h) (void)hipHostFree(h->report_h);
  }
  delete h;
}

const char* cpr_status_string(cpr_status s) {
  switch (s) {
    case CPR_OK: return "CPR_OK";
    case CPR_NOT_CONVERGED: return "CPR_NOT_CONVERGED";
    case CPR_ERR_INVALID_ARG: return "CPR_ERR_INVALID_ARG";
    case CPR_ERR_PATTERN_MISMATCH: return "CPR_ERR_PATTERN_MISMATCH";
    case CPR_ERR_SIZE_MISMATCH: return "CPR_ERR_SIZE_MISMATCH";
    case CPR_ERR_SINGULAR_BLOCK: return "CPR_ERR_SINGULAR_BLOCK";
    case CPR_ERR_SINGULAR_COARSE: return "CPR_ERR_SINGULAR_COARSE";
    case CPR_ERR_NAN: return "CPR_ERR_NAN";
    case CPR_ERR_OOM: return "CPR_ERR_OOM";
    case CPR_ERR_HIP: return "CPR_ERR_HIP";
  }
  return "CPR_UNKNOWN_STATUS";
}

const char* cpr_last_error(const cpr_handle* h) { return h ? h->last_error.c_str() : g_last_error.c_str(); }

int64_t cpr_device_bytes(const cpr_handle* h) {
  if (!h) return 0;
  return h->fine.bytes() + (h->pc ? h->pc->bytes() : 0);
}

// ---------------------------------------------------------------- inspection
cpr_status cpr_spmv(cpr_handle* h, const double* x, double* y) {
  if (!h || !x || !y) return fail(h, CPR_ERR_INVALID_ARG, "null argument");
  return guarded(h, [&]() -> cpr_status {
    h->spmv(x, y);
    HIPCHK(hipStreamSynchronize(h->stream));
    return CPR_OK;
  });
}

cpr_status cpr_precond_apply(cpr_handle* h, const double* v, double* z) {
  if (!h || !v || !z) return fail(h, CPR_ERR_INVALID_ARG, "null argument");
  return guarded(h, [&]() -> cpr_status {
    need_pc(h);
    if (h->pc->fp32()) {
      h->pc->apply(v, h->Z, h->stream);
      launch_copy_cast<float, double>(3 * static_cast<int64_t>(h->n_b), static_cast<const float*>(h->Z), z,
                                      h->stream);
    } else {
      h->pc->apply(v, z, h->stream);
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    return CPR_OK;
  });
}

cpr_status cpr_second_stage(cpr_handle* h, const double* v, const double* pe, double* z) {
  if (!h || !v || !pe || !z) return fail(h, CPR_ERR_INVALID_ARG, "null argument");
  return guarded(h, [&]() -> cpr_status {
    need_pc(h);
    h->pc->second_stage_own(v, pe, z, h->stream);
    HIPCHK(hipStreamSynchronize(h->stream));
    return CPR_OK;
  });
}

cpr_status cpr_vcycle(cpr_handle* h, const double* r, double* e) {
  if (!h || !r || !e) return fail(h, CPR_ERR_INVALID_ARG, "null argument");
  return guarded(h, [&]() -> cpr_status {
    need_pc(h);
    h->pc->vcycle_own(r, e, h->stream);
    HIPCHK(hipStreamSynchronize(h->stream));
    return CPR_OK;
  });
}

cpr_status cpr_smooth(cpr_handle* h, int32_t level, double* x, const double* b, int32_t n_sweeps,
                      int32_t zero_start) {
  if (!h || !x || !b || n_sweeps < 0) return fail(h, CPR_ERR_INVALID_ARG, "invalid argument");
  return guarded(h, [&]() -> cpr_status {
    need_pc(h);
    h->pc->smooth_own(level, x, b, n_sweeps, zero_start != 0, h->stream);
    HIPCHK(hipStreamSynchronize(h->stream));
    return CPR_OK;
  });
}

cpr_status cpr_level_info(const cpr_handle* h, int32_t level, int64_t out[8]) {
  if (!h || !out || level < 0 || level >= static_cast<int32_t>(h->hl.size()))
    return fail(const_cast<cpr_handle*>(h), CPR_ERR_INVALID_ARG, "invalid level");
  const HostLevel& L = h->hl[level];
  const bool last = level + 1 == static_cast<int32_t>(h->hl.size());
  out[0] = L.A.n_rows;
  out[1] = L.A.nnz();
  out[2] = L.n_colours;
  out[3] = last ? 0 : h->hl[level + 1].A.n_rows;
  out[4] = last ? 1 : 0;
  out[5] = static_cast<int64_t>(h->hl.size());
  out[6] = last ? 0 : L.P.nnz();
  out[7] = h->n_block_colours;
  return CPR_OK;
}

cpr_status cpr_level_arrays(const cpr_handle* h, int32_t level, int32_t* row_ptr, int32_t* col, double* val,
                            uint8_t* rs_strong, uint8_t* color_strong, int32_t* colour, int8_t* cf) {
  if (!h || level < 0 || level >= static_cast<int32_t>(h->hl.size()))
    return fail(const_cast<cpr_handle*>(h), CPR_ERR_INVALID_ARG, "invalid level");
  const HostLevel& L = h->hl[level];
  if (row_ptr) std::copy(L.A.ptr.begin(), L.A.ptr.end(), row_ptr);
  if (col) std::copy(L.A.col.begin(), L.A.col.end(), col);
  if (val) std::copy(L.A.val.begin(), L.A.val.end(), val);
  if (rs_strong)
    for (size_t k = 0; k < L.mask.size(); ++k) rs_strong[k] = (L.mask[k] & 1) ? 1 : 0;
  if (color_strong)
    for (size_t k = 0; k < L.mask.size(); ++k) color_strong[k] = (L.mask[k] & 2) ? 1 : 0;
  if (colour) std::copy(L.colour.begin(), L.colour.end(), colour);
  if (cf) std::copy(L.cf.begin(), L.cf.end(), cf);
  return CPR_OK;
}

cpr_status cpr_level_interp(const cpr_handle* h, int32_t level, int32_t* row_ptr, int32_t* col, double* val) {
  if (!h || level < 0 || level + 1 >= static_cast<int32_t>(h->hl.size()))
    return fail(const_cast<cpr_handle*>(h), CPR_ERR_INVALID_ARG, "level has no interpolation");
  const HostCsr& P = h->hl[level].P;
  if (row_ptr) std::copy(P.ptr.begin(), P.ptr.end(), row_ptr);
  if (col) std::copy(P.col.begin(), P.col.end(), col);
  if (val) std::copy(P.val.begin(), P.val.end(), val);
  return CPR_OK;
}

cpr_status cpr_level_aggregates(const cpr_handle* h, int32_t level, int32_t* agg) {
  if (!h || !agg || level < 0 || level >= static_cast<int32_t>(h->hl.size()) || h->hl[level].agg.empty())
    return fail(const_cast<cpr_handle*>(h), CPR_ERR_INVALID_ARG, "level has no aggregates");
  std::copy(h->hl[level].agg.begin(), h->hl[level].agg.end(), agg);
  return CPR_OK;
}

cpr_status cpr_block_colours(const cpr_handle* h, int32_t* colour) {
  if (!h || !colour) return fail(const_cast<cpr_handle*>(h), CPR_ERR_INVALID_ARG, "null argument");
  std::copy(h->block_colour.begin(), h->block_colour.end(), colour);
  return CPR_OK;
}

cpr_status cpr_bilu_factors(const cpr_handle* h, double* lu, double* uinv, int32_t* flev, int32_t* blev,
                            int32_t* n_levels) {
  if (!h) return fail(nullptr, CPR_ERR_INVALID_ARG, "null handle");
  const HostBilu& F = h->bilu_host;
  if (F.flev.empty()) return fail(const_cast<cpr_handle*>(h), CPR_ERR_INVALID_ARG, "the second stage is not block ILU(0)");
  if (lu) std::copy(F.lu.begin(), F.lu.end(), lu);
  if (uinv) std::copy(F.uinv.begin(), F.uinv.end(), uinv);
  if (flev) std::copy(F.flev.begin(), F.flev.end(), flev);
  if (blev) std::copy(F.blev.begin(), F.blev.end(), blev);
  if (n_levels) {
    n_levels[0] = F.n_flev;
    n_levels[1] = F.n_blev;
  }
  return CPR_OK;
}

// ---------------------------------------------------------------- host-only
static Pattern make_pattern(int32_t n, const int32_t* s_ptr, const int32_t* s_col) {
  Pattern S;
  S.n = n;
  S.ptr.assign(s_ptr, s_ptr + n + 1);
  S.col.assign(s_col, s_col + s_ptr[n]);
  return S;
}

cpr_status cpr_host_grouping(int32_t n, const int32_t* s_ptr, const int32_t* s_col, int32_t* colour,
                             int32_t* n_colours) {
  if (n < 0 || !s_ptr || (!s_col && n > 0 && s_ptr[n] > 0) || !colour || !n_colours)
    return fail(nullptr, CPR_ERR_INVALID_ARG, "invalid argument");
  return guarded(nullptr, [&]() -> cpr_status {
    const Pattern S = make_pattern(n, s_ptr, s_col);
    std::vector<int32_t> c;
    *n_colours = vertices_grouping(S, c);
    std::copy(c.begin(), c.end(), colour);
    return CPR_OK;
  });
}

cpr_status cpr_host_rs_split(int32_t n, const int32_t* s_ptr, const int32_t* s_col, int8_t* cf) {
  if (n < 0 || !s_ptr || !cf) return fail(nullptr, CPR_ERR_INVALID_ARG, "invalid argument");
  return guarded(nullptr, [&]() -> cpr_status {
    const Pattern S = make_pattern(n, s_ptr, s_col);
    const Pattern ST = transpose_pattern(S);
    std::vector<int8_t> c;
    rs_split(S, ST, c);
    std::copy(c.begin(), c.end(), cf);
    return CPR_OK;
  });
}

static HostCsr make_csr(int32_t n, int32_t ncols, const int32_t* ptr, const int32_t* col, const double* val) {
  HostCsr A;
  A.n_rows = n;
  A.n_cols = ncols;
  A.ptr.assign(ptr, ptr + n + 1);
  A.col.assign(col, col + ptr[n]);
  A.val.assign(val, val + ptr[n]);
  return A;
}

cpr_status cpr_host_interpolation(int32_t n, const int32_t* a_ptr, const int32_t* a_col, const double* a_val,
                                  const uint8_t* strong, const int8_t* cf, int32_t* p_ptr, int32_t* p_col,
                                  double* p_val, int32_t* n_coarse) {
  if (n < 0 || !a_ptr || !a_col || !a_val || !strong || !cf || !p_ptr || !p_col || !p_val || !n_coarse)
    return fail(nullptr, CPR_ERR_INVALID_ARG, "invalid argument");
  return guarded(nullptr, [&]() -> cpr_status {
    const HostCsr A = make_csr(n, n, a_ptr, a_col, a_val);
    std::vector<uint8_t> mask(strong, strong + a_ptr[n]);
    std::vector<int8_t> c(cf, cf + n);
    HostCsr P;
    if (!rs_interpolation(A, mask, 1, c, P)) throw Error(CPR_ERR_SINGULAR_COARSE, "zero interpolation denominator");
    std::copy(P.ptr.begin(), P.ptr.end(), p_ptr);
    std::copy(P.col.begin(), P.col.end(), p_col);
    std::copy(P.val.begin(), P.val.end(), p_val);
    *n_coarse = P.n_cols;
    return CPR_OK;
  });
}

cpr_status cpr_host_galerkin(int32_t n, int32_t n_coarse, const int32_t* a_ptr, const int32_t* a_col,
                             const double* a_val, const int32_t* p_ptr, const int32_t* p_col, const double* p_val,
                             int32_t* c_ptr, int32_t* c_col, double* c_val) {
  if (n < 0 || n_coarse < 0 || !a_ptr || !a_col || !a_val || !p_ptr || !p_col || !p_val || !c_ptr)
    return fail(nullptr, CPR_ERR_INVALID_ARG, "invalid argument");
  return guarded(nullptr, [&]() -> cpr_status {
    const HostCsr A = make_csr(n, n, a_ptr, a_col, a_val);
    const HostCsr P = make_csr(n, n_coarse, p_ptr, p_col, p_val);
    const HostCsr R = transpose(P);
    const HostCsr C = spgemm_ordered(R, spgemm_ordered(A, P));
    std::copy(C.ptr.begin(), C.ptr.end(), c_ptr);
    if (c_col) std::copy(C.col.begin(), C.col.end(), c_col);
    if (c_val) std::copy(C.val.begin(), C.val.end(), c_val);
    return CPR_OK;
  });
}

cpr_status cpr_host_aggregates(int32_t n, const int32_t* a_ptr, const int32_t* a_col, const double* a_val,
                               double beta, int32_t npair, int32_t* agg, int32_t* n_agg) {
  if (n < 0 || !a_ptr || !a_col || !a_val || !agg || !n_agg || npair < 1)
    return fail(nullptr, CPR_ERR_INVALID_ARG, "invalid argument");
  return guarded(nullptr, [&]() -> cpr_status {
    const HostCsr A = make_csr(n, n, a_ptr, a_col, a_val);
    std::vector<int32_t> a;
    *n_agg = npair_aggregates(A, beta, npair, a);
    std::copy(a.begin(), a.end(), agg);
    return CPR_OK;
  });
}

cpr_status cpr_host_bilu0(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* vals, double* lu,
                          double* uinv, int32_t* flev, int32_t* blev) {
  if (n < 0 || !row_ptr || !col || !vals || !lu || !uinv || !flev || !blev)
    return fail(nullptr, CPR_ERR_INVALID_ARG, "invalid argument");
  return guarded(nullptr, [&]() -> cpr_status {
    std::vector<int32_t> fl, bl;
    bilu_forward_levels(n, row_ptr, col, fl);
    bilu_backward_levels(n, row_ptr, col, bl);
    std::copy(vals, vals + static_cast<int64_t>(row_ptr[n]) * 9, lu);
    const int32_t bad = bilu0_factor(n, row_ptr, col, fl, lu, uinv);
    std::copy(fl.begin(), fl.end(), flev);
    std::copy(bl.begin(), bl.end(), blev);
    if (bad >= 0) throw Error(CPR_ERR_SINGULAR_BLOCK, "pivot block of row " + std::to_string(bad) + " is singular");
    return CPR_OK;
  });
}

// ---------------------------------------------------------------- measurement
cpr_status cpr_profile_enable(cpr_handle* h, int32_t enable) {
  if (!h) return fail(nullptr, CPR_ERR_INVALID_ARG, "null handle");
  h->prof.enable(enable != 0);
  return CPR_OK;
}

cpr_status cpr_profile_read(cpr_handle* h, int32_t kind, int64_t* launches, double* total_ms, double* bytes) {
  if (!h || kind < 0 || kind >= CPR_KSTAT_COUNT) return fail(h, CPR_ERR_INVALID_ARG, "invalid kernel class");
  if (launches) *launches = h->prof.launches[kind];
  if (total_ms) *total_ms = h->prof.total_ms[kind];
  if (bytes) *bytes = h->prof.bytes[kind];
  return CPR_OK;
}

cpr_status cpr_copy_kernel(void* dst, const void* src, int64_t n_bytes, void* hip_stream) {
  if (!dst || !src || n_bytes < 0) return fail(nullptr, CPR_ERR_INVALID_ARG, "invalid argument");
  return guarded(nullptr, [&]() -> cpr_status {
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    launch_copy_bytes(n_bytes, src, dst, s);
    HIPCHK(hipStreamSynchronize(s));
    return CPR_OK;
  });
}

}  // extern "C"
