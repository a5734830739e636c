// Request-serving runtime: worker threads with their own streams, admission
// by device-memory budget, resident cases with LRU eviction.  See cpr_serve.h.
#include "../../include/cpr_serve.h"

#include <hip/hip_runtime.h>

#include "solver.hpp"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Req {
  int64_t ticket = 0;
  cpr_request r{};
  double t_submit = 0.0;
  bool done = false;
  cpr_status status = CPR_OK;
  cpr_solve_info info{};
  double latency_ms = 0.0;
};

struct Case {
  cpr_handle* h = nullptr;
  hipStream_t stream = nullptr;  // the case's own stream (its handle never changes stream)
  double* d_b = nullptr;
  double* d_x = nullptr;
  int32_t n_b = 0, nnz_b = 0;
  int64_t bytes = 0;  // device bytes charged to the budget
  bool busy = false;
  uint64_t last_use = 0;
};

// Device bytes a case will need before it is set up (upper estimate): outer
// matrix with its staging copy and slot map, stage-2 copy, AMG hierarchy (up to
// five times the pressure entries), Krylov bases and vectors.
int64_t estimate_bytes(const cpr_bsr& A, const cpr_params& p) {
  const int64_t nnz = A.nnz_blocks, n = A.n_block_rows;
  const int64_t sv = p.precond_fp32 ? 4 : 8;
  const int64_t m = p.restart;
  int64_t b = 0;
  b += nnz * (72 + 72 + 4 + 8) * 11 / 10;  // outer SELL (+padding), values, columns, slot map
  b += nnz * (9 * sv + 4 + 8) * 11 / 10;   // stage-2 copy, columns, slot map
  b += 5 * nnz * (sv + 4) * 2;              // hierarchy: A_l, P, R over all levels
  b += n * (9 * sv + 64);                   // D^-1, permutations, level vectors
  b += 3 * n * (8 * (m + 1) + sv * m + 8 * 4);  // V, Z, residual, b, x
  return b + (16 << 20);
}

}  // namespace

struct cpr_server {
  cpr_params prm{};
  int device = 0;
  int64_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Req>> pending;
  std::unordered_map<int64_t, std::shared_ptr<Req>> tickets;
  std::unordered_map<int64_t, Case> cases;
  int64_t used = 0, peak = 0;
  int64_t next_ticket = 1;
  uint64_t clock = 0;
  int running = 0;
  bool stop = false;
  cpr_server_stats st{};
  std::string last_error;  // text of the most recent failed request
  std::vector<std::thread> workers;

  // Under the lock: the first pending request that can start now, or null.
  std::shared_ptr<Req> pick() {
    for (auto it = pending.begin(); it != pending.end(); ++it) {
      std::shared_ptr<Req> rq = *it;
      auto cit = cases.find(rq->r.case_id);
      if (cit != cases.end() && cit->second.busy) continue;
      const bool resident = cit != cases.end() && cit->second.h && cit->second.n_b == rq->r.A.n_block_rows &&
                            cit->second.nnz_b == rq->r.A.nnz_blocks;
      int64_t need = 0;
      if (!resident) {
        need = estimate_bytes(rq->r.A, prm);
        const int64_t freed_by_replace = cit != cases.end() ? cit->second.bytes : 0;
        while (used - freed_by_replace + need > budget && evict_one(rq->r.case_id)) {
        }
        if (used - freed_by_replace + need > budget) {
          // nothing left to evict: if nothing runs either, it can never fit
          bool others_resident = false;
          for (auto& kv : cases)
            if (kv.first != rq->r.case_id && kv.second.h) others_resident = true;
          if (running == 0 && !others_resident) {
            rq->status = CPR_ERR_OOM;
            rq->done = true;
            rq->latency_ms = now_ms() - rq->t_submit;
            st.rejected += 1;
            pending.erase(it);
            cv_done.notify_all();
            return pick();
          }
          continue;
        }
      }
      Case& c = cases[rq->r.case_id];
      if (!resident) {
        used -= c.bytes;
        c.bytes = need;  // charged now, corrected after SETUP
        used += need;
        peak = std::max(peak, used);
      }
      c.busy = true;
      pending.erase(it);
      return rq;
    }
    return nullptr;
  }

  // Evict the least recently used idle resident case other than `keep`.
  bool evict_one(int64_t keep) {
    int64_t victim = 0;
    bool found = false;
    uint64_t best = ~0ull;
    for (auto& kv : cases)
      if (kv.first != keep && !kv.second.busy && kv.second.h && kv.second.last_use < best) {
        best = kv.second.last_use;
        victim = kv.first;
        found = true;
      }
    if (!found) return false;
    Case& c = cases[victim];
    release(c);
    cases.erase(victim);
    st.evictions += 1;
    return true;
  }

  static void free_case(Case& c) {
    if (c.h) cpr_destroy(c.h);
    {
      std::lock_guard<std::mutex> lk(cpr::device_api_mutex());
      if (c.d_b) (void)hipFree(c.d_b);
      if (c.d_x) (void)hipFree(c.d_x);
      if (c.stream) (void)hipStreamDestroy(c.stream);
    }
    c.h = nullptr;
    c.d_b = c.d_x = nullptr;
    c.stream = nullptr;
  }

  void release(Case& c) {
    free_case(c);
    used -= c.bytes;
    c = Case();
  }

  void worker(int wid) {
    (void)wid;
    (void)hipSetDevice(device);
    while (true) {
      std::shared_ptr<Req> rq;
      Case snapshot;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] {
          if (stop && pending.empty()) return true;
          rq = pick();
          return rq != nullptr;
        });
        if (!rq) break;
        running += 1;
        snapshot = cases[rq->r.case_id];
      }
      cpr_status s = run(rq, snapshot);
      {
        std::lock_guard<std::mutex> lk(mu);
        Case& c = cases[rq->r.case_id];
        const int64_t charged = c.bytes;
        c = snapshot;
        c.busy = false;
        c.last_use = ++clock;
        if (c.h) {
          c.bytes = cpr_device_bytes(c.h) + 2 * 3 * static_cast<int64_t>(c.n_b) * 8;
          used += c.bytes - charged;
        } else {
          free_case(c);  // SETUP failed: nothing stays resident
          used -= charged;
          c.bytes = 0;
        }
        peak = std::max(peak, used);
        running -= 1;
        if (s != CPR_OK && s != CPR_NOT_CONVERGED)
          last_error = "case " + std::to_string(rq->r.case_id) + ": " + cpr_status_string(s) + ": " +
                       (c.h ? cpr_last_error(c.h) : cpr_last_error(nullptr));
        rq->status = s;
        rq->done = true;
        rq->latency_ms = now_ms() - rq->t_submit;
        st.completed += 1;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }

  // One request on its case's stream: SETUP or value update, then the solve.
  cpr_status run(const std::shared_ptr<Req>& rq, Case& c) {
    const cpr_request& r = rq->r;
    const int32_t n = r.A.n_block_rows;
    const size_t vec = 3 * static_cast<size_t>(n) * sizeof(double);
    cpr_status s = CPR_OK;
    bool reused = false;
    if (c.h && c.n_b == n && c.nnz_b == r.A.nnz_blocks) {
      s = cpr_update_values(c.h, &r.A);
      if (s == CPR_OK) reused = true;
      if (s == CPR_ERR_PATTERN_MISMATCH) s = CPR_OK;  // new pattern: the case is replaced
    }
    if (!reused) {
      free_case(c);
      hipError_t e;
      {
        std::lock_guard<std::mutex> lk(cpr::device_api_mutex());
        e = hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking);
      }
      if (e != hipSuccess) {
        (void)hipGetLastError();
        c.stream = nullptr;
        return CPR_ERR_HIP;
      }
      s = cpr_setup(&r.A, &prm, c.stream, &c.h);
      if (s != CPR_OK) {
        c.h = nullptr;
        return s;
      }
      c.n_b = n;
      c.nnz_b = r.A.nnz_blocks;
      {
        std::lock_guard<std::mutex> lk(cpr::device_api_mutex());
        e = hipMalloc(&c.d_b, vec);
        if (e == hipSuccess) e = hipMalloc(&c.d_x, vec);
      }
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return CPR_ERR_OOM;
      }
      std::lock_guard<std::mutex> lk(mu);
      st.setups += 1;
    } else {
      std::lock_guard<std::mutex> lk(mu);
      st.reuses += 1;
    }
    if (hipMemcpyAsync(c.d_b, r.b, vec, hipMemcpyHostToDevice, c.stream) != hipSuccess ||
        hipMemsetAsync(c.d_x, 0, vec, c.stream) != hipSuccess)
      return CPR_ERR_HIP;
    s = cpr_solve(c.h, c.d_b, c.d_x, r.tol, &rq->info);
    if (s == CPR_OK || s == CPR_NOT_CONVERGED) {
      if (hipMemcpyAsync(r.x, c.d_x, vec, hipMemcpyDeviceToHost, c.stream) != hipSuccess ||
          hipStreamSynchronize(c.stream) != hipSuccess)
        return CPR_ERR_HIP;
    }
    return s;
  }
};

extern "C" {

cpr_status cpr_server_create(int64_t budget_bytes, int32_t max_slots, const cpr_params* p, cpr_server** out) {
  if (!out || budget_bytes <= 0 || max_slots < 1 || max_slots > 64) return CPR_ERR_INVALID_ARG;
  *out = nullptr;
  cpr_server* s = new cpr_server();
  cpr_params_default(&s->prm);
  if (p) s->prm = *p;
  s->budget = budget_bytes;
  s->st.budget_bytes = budget_bytes;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return CPR_ERR_HIP;
  }
  for (int w = 0; w < max_slots; ++w) s->workers.emplace_back([s, w] { s->worker(w); });
  *out = s;
  return CPR_OK;
}

cpr_status cpr_server_submit(cpr_server* s, const cpr_request* r, int64_t* ticket) {
  if (!s || !r || !ticket || !r->b || !r->x || !(r->tol > 0.0) || r->A.location != CPR_MEM_HOST ||
      r->A.block_dim != 3 || r->A.n_block_rows <= 0 || !r->A.row_ptr || !r->A.col_idx || !r->A.values)
    return CPR_ERR_INVALID_ARG;
  auto rq = std::make_shared<Req>();
  rq->r = *r;
  rq->t_submit = now_ms();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    rq->ticket = s->next_ticket++;
    s->tickets[rq->ticket] = rq;
    s->pending.push_back(rq);
    s->st.submitted += 1;
    *ticket = rq->ticket;
  }
  s->cv_work.notify_all();
  return CPR_OK;
}

cpr_status cpr_server_wait(cpr_server* s, int64_t ticket, cpr_solve_info* info, double* latency_ms) {
  if (!s) return CPR_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return CPR_ERR_INVALID_ARG;
  std::shared_ptr<Req> rq = it->second;
  s->cv_done.wait(lk, [&] { return rq->done; });
  s->tickets.erase(ticket);
  if (info) *info = rq->info;
  if (latency_ms) *latency_ms = rq->latency_ms;
  return rq->status;
}

const char* cpr_server_last_error(cpr_server* s) {
  if (!s) return "";
  std::lock_guard<std::mutex> lk(s->mu);
  return s->last_error.c_str();
}

cpr_status cpr_server_stats_get(cpr_server* s, cpr_server_stats* out) {
  if (!s || !out) return CPR_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->resident_cases = 0;
  for (auto& kv : s->cases)
    if (kv.second.h) out->resident_cases += 1;
  out->bytes_in_use = s->used;
  out->bytes_peak = s->peak;
  out->budget_bytes = s->budget;
  return CPR_OK;
}

void cpr_server_destroy(cpr_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  for (auto& kv : s->cases) s->release(kv.second);
  delete s;
}

}  // extern "C"
