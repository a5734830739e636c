// Host-side SETUP algorithms; see host_setup.hpp for the contracts.
#include "host_setup.hpp"

#include <algorithm>
#include <limits>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <queue>
#include <set>
#include <thread>
#include <utility>

namespace cpr {

int setup_threads() {
  const unsigned hw = std::thread::hardware_concurrency();
  return static_cast<int>(std::max(1u, std::min(hw, 16u)));
}

namespace {

// Persistent worker threads shared by every SETUP in the process (the
// serving runtime runs several at once).  A parallel call posts a job; the
// caller and idle workers join it, each under a slot index below the job's
// slot count (per-call scratch is indexed by slot), and claim chunks until
// none is left; the caller returns when every claimed chunk has finished.
// Spawning fresh threads per call instead cost ~0.3 ms a call, dozens of
// calls per SETUP: most of the SETUP time of a 10^4-cell case.
class SetupPool {
 public:
  static SetupPool& get() {
    static SetupPool* pool = new SetupPool();  // never destroyed: workers live until the process ends
    return *pool;
  }

  void run(int n_chunks, int n_slots, const std::function<void(int, int)>& f) {
    auto job = std::make_shared<Job>();
    job->f = &f;
    job->n_chunks = n_chunks;
    job->n_slots = n_slots;
    {
      std::lock_guard<std::mutex> lk(m_);
      queue_.push_back(job);
    }
    cv_.notify_all();
    work(*job);
    {
      std::unique_lock<std::mutex> lk(job->m);
      job->cv.wait(lk, [&] { return job->done == job->n_chunks; });
    }
    std::lock_guard<std::mutex> lk(m_);
    for (auto it = queue_.begin(); it != queue_.end(); ++it)
      if (it->get() == job.get()) {
        queue_.erase(it);
        break;
      }
  }

 private:
  struct Job {
    const std::function<void(int, int)>* f = nullptr;
    int n_chunks = 0, n_slots = 0;
    std::atomic<int> next_chunk{0}, next_slot{0};
    std::mutex m;
    std::condition_variable cv;
    int done = 0;  // finished chunks, under m
  };

  SetupPool() {
    const int nt = setup_threads() - 1;  // the caller is the remaining thread
    for (int t = 0; t < nt; ++t) std::thread([this]() { worker(); }).detach();
  }

  // Join a job under a free slot and run chunks until none is left.
  static void work(Job& job) {
    const int slot = job.next_slot++;
    if (slot >= job.n_slots) return;
    int finished = 0;
    for (int c = job.next_chunk++; c < job.n_chunks; c = job.next_chunk++) {
      (*job.f)(c, slot);
      ++finished;
    }
    if (finished > 0) {
      std::lock_guard<std::mutex> lk(job.m);
      job.done += finished;
      if (job.done == job.n_chunks) job.cv.notify_all();
    }
  }

  void worker() {
    for (;;) {
      std::shared_ptr<Job> job;
      {
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [&] {
          while (!queue_.empty() && (queue_.front()->next_chunk.load() >= queue_.front()->n_chunks ||
                                     queue_.front()->next_slot.load() >= queue_.front()->n_slots))
            queue_.pop_front();  // nothing left to join
          return !queue_.empty();
        });
        job = queue_.front();
      }
      work(*job);
    }
  }

  std::mutex m_;
  std::condition_variable cv_;
  std::deque<std::shared_ptr<Job>> queue_;
};

// Run f(chunk, slot) for chunk = 0..n_chunks-1 on up to setup_threads()
// threads; `slot` (below n_workers(n_chunks)) indexes per-call scratch.
template <typename F>
void parallel_chunks(int n_chunks, F&& f) {
  const int nt = std::min(setup_threads(), n_chunks);
  if (nt <= 1) {
    for (int c = 0; c < n_chunks; ++c) f(c, 0);
    return;
  }
  const std::function<void(int, int)> fn = [&f](int c, int t) { f(c, t); };
  SetupPool::get().run(n_chunks, nt, fn);
}

int n_workers(int n_chunks) { return std::max(1, std::min(setup_threads(), n_chunks)); }

// Rows [0, n) split into contiguous chunks for parallel_chunks.  Every row's
// result depends only on that row, so results do not depend on the thread
// count.
struct RowChunks {
  int32_t n_rows = 0, n_chunks = 0;
  explicit RowChunks(int32_t n) : n_rows(n) {
    n_chunks = static_cast<int32_t>(std::min<int64_t>(std::max<int64_t>(1, n / 2048), 256));
  }
  int32_t begin(int c) const { return static_cast<int32_t>(static_cast<int64_t>(n_rows) * c / n_chunks); }
  int32_t end(int c) const { return static_cast<int32_t>(static_cast<int64_t>(n_rows) * (c + 1) / n_chunks); }
};

}  // namespace

void parallel_for(int n_chunks, const std::function<void(int, int)>& f) { parallel_chunks(n_chunks, f); }

namespace {
// Transpose of an n x m pattern (ptr, col) in blocks of rows: each block
// counts its entries per column, a column's blocks then take consecutive
// ranges of the column in block order, and each block writes its rows in
// ascending order, so every column of the result lists its rows in
// ascending order whatever the thread count (as a sequential transpose
// does).  tptr (m + 1 entries, zero on entry) receives the row pointers;
// put(w, i, p) stores entry p (row i) of the input at position w.
template <typename Put>
void transpose_blocks(int32_t n, int32_t m, int64_t nnz, const int32_t* ptr, const int32_t* col, int32_t* tptr,
                      Put&& put) {
  const int nb = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(setup_threads(), nnz / 262144)));
  auto row0 = [&](int b) { return static_cast<int32_t>(static_cast<int64_t>(n) * b / nb); };
  std::vector<std::vector<int32_t>> cnt(nb);
  parallel_chunks(nb, [&](int b, int) {
    std::vector<int32_t>& c = cnt[b];
    c.assign(static_cast<size_t>(m), 0);
    for (int32_t p = ptr[row0(b)]; p < ptr[row0(b + 1)]; ++p) c[col[p]]++;
  });
  // cnt[b][j] becomes block b's first slot within column j
  const int ncb = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(64, m / 4096)));
  parallel_chunks(ncb, [&](int cb, int) {
    const int32_t j1 = static_cast<int32_t>(static_cast<int64_t>(m) * (cb + 1) / ncb);
    for (int32_t j = static_cast<int32_t>(static_cast<int64_t>(m) * cb / ncb); j < j1; ++j) {
      int32_t sum = 0;
      for (int b = 0; b < nb; ++b) {
        const int32_t c = cnt[b][j];
        cnt[b][j] = sum;
        sum += c;
      }
      tptr[j + 1] = sum;
    }
  });
  for (int32_t j = 0; j < m; ++j) tptr[j + 1] += tptr[j];
  parallel_chunks(nb, [&](int b, int) {
    std::vector<int32_t>& c = cnt[b];
    for (int32_t i = row0(b); i < row0(b + 1); ++i)
      for (int32_t p = ptr[i]; p < ptr[i + 1]; ++p) {
        const int32_t j = col[p];
        put(static_cast<int64_t>(tptr[j]) + c[j]++, i, p);
      }
  });
}
}  // namespace

Pattern pattern_from_mask(const HostCsr& A, const std::vector<uint8_t>& mask, uint8_t bit) {
  Pattern S;
  const int32_t n = A.n_rows;
  S.n = n;
  S.ptr.assign(static_cast<size_t>(n) + 1, 0);
  RowChunks rc(n);
  parallel_chunks(rc.n_chunks, [&](int ch, int) {
    for (int32_t i = rc.begin(ch); i < rc.end(ch); ++i) {
      int32_t c = 0;
      for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) c += (mask[p] & bit) ? 1 : 0;
      S.ptr[i + 1] = c;
    }
  });
  for (int32_t i = 0; i < n; ++i) S.ptr[i + 1] += S.ptr[i];
  S.col.resize(S.ptr[n]);
  parallel_chunks(rc.n_chunks, [&](int ch, int) {
    for (int32_t i = rc.begin(ch); i < rc.end(ch); ++i) {
      int32_t w = S.ptr[i];
      for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p)
        if (mask[p] & bit) S.col[w++] = A.col[p];
    }
  });
  return S;
}

Pattern transpose_pattern(const Pattern& S) {
  Pattern T;
  T.n = S.n;
  T.ptr.assign(static_cast<size_t>(S.n) + 1, 0);
  T.col.resize(S.col.size());
  transpose_blocks(S.n, S.n, static_cast<int64_t>(S.col.size()), S.ptr.data(), S.col.data(), T.ptr.data(),
                   [&](int64_t w, int32_t i, int32_t) { T.col[w] = i; });
  return T;
}

// ------------------------------------------------------------ grouping
namespace {
enum : int8_t { kOutside = 0, kUndecided = 1, kInW = 2, kInWbar = 3 };

// Max-heap on (influence, -index): largest influence first, then smallest index.
struct InflKey {
  int32_t infl, v;
};
struct InflLess {
  bool operator()(const InflKey& a, const InflKey& b) const {
    if (a.infl != b.infl) return a.infl < b.infl;
    return a.v > b.v;
  }
};
using InflHeap = std::priority_queue<InflKey, std::vector<InflKey>, InflLess>;
}  // namespace

int32_t vertices_grouping(const Pattern& S, std::vector<int32_t>& colour) {
  const int32_t n = S.n;
  colour.assign(n, -1);
  std::vector<int32_t> infl(n);
  for (int32_t i = 0; i < n; ++i) infl[i] = S.ptr[i + 1] - S.ptr[i];
  std::vector<int8_t> state(n, kOutside);
  std::vector<int32_t> in_front(n, -1);  // round in which the vertex entered the frontier
  std::vector<int32_t> V(n);
  for (int32_t i = 0; i < n; ++i) V[i] = i;
  std::vector<int32_t> Wbar;
  int32_t c = 0;
  while (!V.empty()) {
    for (int32_t v : V) state[v] = kUndecided;
    int64_t remaining = static_cast<int64_t>(V.size());
    std::vector<InflKey> init;
    init.reserve(V.size());
    for (int32_t v : V) init.push_back({infl[v], v});
    InflHeap heap_v(InflLess(), std::move(init));
    InflHeap heap_f;
    Wbar.clear();
    auto pop = [&](InflHeap& h) -> int32_t {
      while (!h.empty()) {
        int32_t v = h.top().v;
        h.pop();
        if (state[v] == kUndecided) return v;
      }
      return -1;
    };
    while (remaining > 0) {
      int32_t v = pop(heap_f);
      if (v < 0) v = pop(heap_v);
      bool touches_w = false;
      for (int32_t p = S.ptr[v]; p < S.ptr[v + 1]; ++p)
        if (state[S.col[p]] == kInW) {
          touches_w = true;
          break;
        }
      if (!touches_w) {
        state[v] = kInW;
        colour[v] = c;
        --remaining;
        for (int32_t p = S.ptr[v]; p < S.ptr[v + 1]; ++p) {
          int32_t j = S.col[p];
          if (state[j] == kUndecided) {
            state[j] = kInWbar;
            Wbar.push_back(j);
            --remaining;
          }
        }
        for (int32_t p = S.ptr[v]; p < S.ptr[v + 1]; ++p) {
          int32_t k = S.col[p];
          for (int32_t q = S.ptr[k]; q < S.ptr[k + 1]; ++q) {
            int32_t j = S.col[q];
            // keys are static, so one frontier entry per vertex and round suffices
            if (state[j] == kUndecided && in_front[j] != c) {
              in_front[j] = c;
              heap_f.push({infl[j], j});
            }
          }
        }
      } else {
        state[v] = kInWbar;
        Wbar.push_back(v);
        --remaining;
      }
    }
    // W-bar (ascending) is the next round's vertex set; reset visited marks.
    for (int32_t v : V) state[v] = kOutside;
    std::sort(Wbar.begin(), Wbar.end());
    V.swap(Wbar);
    ++c;
  }
  return c;
}

// ------------------------------------------------------------ RS split
namespace {
// A set of indices in [0, n) with insert, erase and smallest-member queries in
// O(log_64 n): a 64-ary tree of occupancy words (bit b of word w on a level
// says whether word 64w + b of the level below has any bit set).
class IndexSet {
 public:
  explicit IndexSet(int32_t n) {
    int64_t words = (static_cast<int64_t>(n) + 63) / 64;
    do {
      lv_.emplace_back(static_cast<size_t>(std::max<int64_t>(words, 1)), 0ull);
      words = (words + 63) / 64;
    } while (lv_.back().size() > 1);
  }
  void insert(int32_t i) {
    uint64_t idx = static_cast<uint64_t>(i);
    for (auto& w : lv_) {
      const bool was_empty = w[idx >> 6] == 0;
      w[idx >> 6] |= 1ull << (idx & 63);
      if (!was_empty) break;
      idx >>= 6;
    }
  }
  void erase(int32_t i) {
    uint64_t idx = static_cast<uint64_t>(i);
    for (auto& w : lv_) {
      w[idx >> 6] &= ~(1ull << (idx & 63));
      if (w[idx >> 6] != 0) break;
      idx >>= 6;
    }
  }
  bool empty() const { return lv_.back()[0] == 0; }
  int32_t first() const {  // smallest member; the set must not be empty
    uint64_t idx = 0;
    for (size_t l = lv_.size(); l-- > 0;) idx = (idx << 6) | static_cast<uint64_t>(__builtin_ctzll(lv_[l][idx]));
    return static_cast<int32_t>(idx);
  }

 private:
  std::vector<std::vector<uint64_t>> lv_;  // lv_[0]: one bit per index
};
}  // namespace

// First pass: repeatedly take the undecided point of largest lambda (ties to
// the smallest index).  Points are kept in one IndexSet per lambda value;
// lambda_i never exceeds 2|S^T_i| (it grows by one for each strong dependent
// that turns F), which bounds the number of sets.
void rs_split(const Pattern& S, const Pattern& ST, std::vector<int8_t>& cf) {
  constexpr int8_t U = 0, C = 1, F = 2;
  const int32_t n = S.n;
  cf.assign(n, U);
  std::vector<int32_t> lam(n, 0);
  int32_t max_st = 0;
  for (int32_t i = 0; i < n; ++i) max_st = std::max(max_st, ST.ptr[i + 1] - ST.ptr[i]);
  std::vector<IndexSet> bucket;
  bucket.reserve(2 * static_cast<size_t>(max_st) + 1);
  for (int32_t v = 0; v <= 2 * max_st; ++v) bucket.emplace_back(n);
  int32_t top = 0;
  for (int32_t i = 0; i < n; ++i) {
    const bool no_s = S.ptr[i + 1] == S.ptr[i];
    const bool no_st = ST.ptr[i + 1] == ST.ptr[i];
    if (no_s && no_st) {
      cf[i] = F;
    } else {
      lam[i] = ST.ptr[i + 1] - ST.ptr[i];
      bucket[lam[i]].insert(i);
      top = std::max(top, lam[i]);
    }
  }
  while (true) {
    while (top > 0 && bucket[top].empty()) --top;
    if (top == 0) break;  // every undecided point left has lambda = 0
    const int32_t i = bucket[top].first();
    bucket[top].erase(i);
    cf[i] = C;
    for (int32_t p = ST.ptr[i]; p < ST.ptr[i + 1]; ++p) {
      const int32_t j = ST.col[p];
      if (cf[j] != U) continue;
      cf[j] = F;
      bucket[lam[j]].erase(j);
      for (int32_t q = S.ptr[j]; q < S.ptr[j + 1]; ++q) {
        const int32_t k = S.col[q];
        if (cf[k] == U) {
          bucket[lam[k]].erase(k);
          lam[k] += 1;
          bucket[lam[k]].insert(k);
          top = std::max(top, lam[k]);
        }
      }
    }
    for (int32_t p = S.ptr[i]; p < S.ptr[i + 1]; ++p) {
      const int32_t j = S.col[p];
      if (cf[j] == U) {
        bucket[lam[j]].erase(j);
        lam[j] -= 1;
        bucket[lam[j]].insert(j);
      }
    }
  }
  for (int32_t i = 0; i < n; ++i) {
    if (cf[i] != U) continue;
    bool has_c = false;
    for (int32_t p = S.ptr[i]; p < S.ptr[i + 1]; ++p)
      if (cf[S.col[p]] == C) {
        has_c = true;
        break;
      }
    cf[i] = has_c ? F : C;
  }
  // second pass: membership of C_i tracked with a stamp array
  std::vector<int32_t> stamp(n, -1);
  for (int32_t i = 0; i < n; ++i) {
    if (cf[i] != F) continue;
    for (int32_t p = S.ptr[i]; p < S.ptr[i + 1]; ++p)
      if (cf[S.col[p]] == C) stamp[S.col[p]] = i;
    int32_t tentative = -1;
    for (int32_t p = S.ptr[i]; p < S.ptr[i + 1]; ++p) {
      const int32_t j = S.col[p];
      if (cf[j] != F) continue;
      bool shares = false;
      for (int32_t q = S.ptr[j]; q < S.ptr[j + 1]; ++q)
        if (stamp[S.col[q]] == i) {
          shares = true;
          break;
        }
      if (shares) continue;
      if (tentative < 0) {
        tentative = j;
        cf[j] = C;
        stamp[j] = i;
      } else {
        cf[tentative] = F;
        stamp[tentative] = -1;
        cf[i] = C;
        break;
      }
    }
  }
}

// ------------------------------------------------------------ interpolation
// For F point i with interpolatory set C_i = strong C dependencies (stored order):
//   d = a_ii; then d = d + a_ij for each weak j != i in stored order;
//   num_j = a_ij for j in C_i;
//   for each strong F dependency m of i (stored order):
//     den = 0 + sum of a_mk over k in C_i (row m, stored order);
//     den == 0 -> d = d + a_im; otherwise num_k = num_k + (a_im*a_mk)/den for
//     each k in C_i met in row m (stored order);
//   w_ij = -num_j / d.
// C points get the unit row of their coarse index; F points without a strong C
// dependency get an empty row.
bool rs_interpolation(const HostCsr& A, const std::vector<uint8_t>& mask, uint8_t bit,
                      const std::vector<int8_t>& cf, HostCsr& P) {
  constexpr int8_t C = 1, F = 2;
  const int32_t n = A.n_rows;
  std::vector<int32_t> coarse(n, -1);
  int32_t nc = 0;
  for (int32_t i = 0; i < n; ++i)
    if (cf[i] == C) coarse[i] = nc++;
  P = HostCsr();
  P.n_rows = n;
  P.n_cols = nc;
  RowChunks rc(n);
  std::atomic<bool> ok{true};
  // Row lengths first (a C point interpolates from itself; an F point from
  // each strong C neighbour, or not at all), then one allocation of P, then
  // the weights written straight into place.
  P.ptr.assign(static_cast<size_t>(n) + 1, 0);
  parallel_chunks(rc.n_chunks, [&](int ch, int) {
    for (int32_t i = rc.begin(ch); i < rc.end(ch); ++i) {
      int32_t len = 0;
      if (cf[i] == C) {
        len = 1;
      } else {
        for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p)
          if ((mask[p] & bit) && cf[A.col[p]] == C) ++len;
      }
      P.ptr[i + 1] = len;
    }
  });
  for (int32_t i = 0; i < n; ++i) P.ptr[i + 1] += P.ptr[i];
  P.col.resize(P.ptr[n]);
  P.val.resize(P.ptr[n]);
  // per-thread marks, indexed by fine row and stamped with the current row
  const int nw = n_workers(rc.n_chunks);
  std::vector<std::vector<int32_t>> in_ci_t(nw);
  std::vector<std::vector<double>> num_t(nw);
  parallel_chunks(rc.n_chunks, [&](int ch, int t) {
    if (in_ci_t[t].empty()) {
      in_ci_t[t].assign(n, -1);
      num_t[t].assign(n, 0.0);
    }
    std::vector<int32_t>& in_ci = in_ci_t[t];
    std::vector<double>& num = num_t[t];
    for (int32_t i = rc.begin(ch); i < rc.end(ch); ++i) {
      int32_t* pc = P.col.data() + P.ptr[i];
      double* pv = P.val.data() + P.ptr[i];
      const int32_t a0 = A.ptr[i], a1 = A.ptr[i + 1];
      if (cf[i] == C) {
        pc[0] = coarse[i];
        pv[0] = 1.0;
        continue;
      }
      bool any_c = false;
      for (int32_t p = a0; p < a1; ++p)
        if ((mask[p] & bit) && cf[A.col[p]] == C) {
          in_ci[A.col[p]] = i;
          num[A.col[p]] = A.val[p];
          any_c = true;
        }
      if (!any_c) continue;
      double d = 0.0;
      for (int32_t p = a0; p < a1; ++p)
        if (A.col[p] == i) d = A.val[p];
      for (int32_t p = a0; p < a1; ++p)
        if (A.col[p] != i && !(mask[p] & bit)) d = d + A.val[p];
      for (int32_t p = a0; p < a1; ++p) {
        const int32_t m = A.col[p];
        if (!(mask[p] & bit) || cf[m] != F) continue;
        const double a_im = A.val[p];
        double den = 0.0;
        for (int32_t q = A.ptr[m]; q < A.ptr[m + 1]; ++q)
          if (in_ci[A.col[q]] == i) den = den + A.val[q];
        if (den == 0.0) {
          d = d + a_im;
          continue;
        }
        for (int32_t q = A.ptr[m]; q < A.ptr[m + 1]; ++q) {
          const int32_t k = A.col[q];
          if (in_ci[k] == i) num[k] = num[k] + (a_im * A.val[q]) / den;
        }
      }
      if (d == 0.0) ok = false;
      int32_t w = 0;
      for (int32_t p = a0; p < a1; ++p) {
        const int32_t j = A.col[p];
        if ((mask[p] & bit) && cf[j] == C) {
          pc[w] = coarse[j];
          pv[w] = -num[j] / d;
          ++w;
        }
      }
    }
  });
  return ok;
}

HostCsr transpose(const HostCsr& A) {
  HostCsr T;
  T.n_rows = A.n_cols;
  T.n_cols = A.n_rows;
  T.ptr.assign(static_cast<size_t>(A.n_cols) + 1, 0);
  T.col.resize(A.col.size());
  T.val.resize(A.val.size());
  transpose_blocks(A.n_rows, A.n_cols, A.nnz(), A.ptr.data(), A.col.data(), T.ptr.data(),
                   [&](int64_t w, int32_t i, int32_t p) {
                     T.col[w] = i;
                     T.val[w] = A.val[p];
                   });
  return T;
}

// Two passes over row chunks: the number of distinct columns of every result
// row, then (after one allocation of the result) the values, written straight
// into place.  Growing per-chunk buffers instead made every thread allocate and
// fault in fresh pages and serialised them (slower than one thread).
HostCsr spgemm_ordered(const HostCsr& A, const HostCsr& B) {
  HostCsr Cm;
  const int32_t n = A.n_rows;
  Cm.n_rows = n;
  Cm.n_cols = B.n_cols;
  Cm.ptr.assign(static_cast<size_t>(n) + 1, 0);
  RowChunks rc(n);
  const int nw = n_workers(rc.n_chunks);
  std::vector<std::vector<int32_t>> seen_t(nw);
  parallel_chunks(rc.n_chunks, [&](int ch, int t) {
    std::vector<int32_t>& seen = seen_t[t];
    if (seen.empty()) seen.assign(B.n_cols, -1);
    for (int32_t i = rc.begin(ch); i < rc.end(ch); ++i) {
      int32_t cnt = 0;
      for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
        const int32_t k = A.col[p];
        for (int32_t q = B.ptr[k]; q < B.ptr[k + 1]; ++q) {
          const int32_t j = B.col[q];
          if (seen[j] != i) {
            seen[j] = i;
            ++cnt;
          }
        }
      }
      Cm.ptr[i + 1] = cnt;
    }
  });
  for (int32_t i = 0; i < n; ++i) Cm.ptr[i + 1] += Cm.ptr[i];
  Cm.col.resize(Cm.ptr[n]);
  Cm.val.resize(Cm.ptr[n]);
  for (auto& seen : seen_t) std::fill(seen.begin(), seen.end(), -1);
  std::vector<std::vector<double>> acc_t(nw);
  parallel_chunks(rc.n_chunks, [&](int ch, int t) {
    std::vector<int32_t>& seen = seen_t[t];
    std::vector<double>& acc = acc_t[t];
    if (seen.empty()) seen.assign(B.n_cols, -1);
    if (acc.empty()) acc.assign(B.n_cols, 0.0);
    for (int32_t i = rc.begin(ch); i < rc.end(ch); ++i) {
      int32_t* cols = Cm.col.data() + Cm.ptr[i];
      int32_t m = 0;
      for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
        const int32_t k = A.col[p];
        const double a = A.val[p];
        for (int32_t q = B.ptr[k]; q < B.ptr[k + 1]; ++q) {
          const int32_t j = B.col[q];
          if (seen[j] != i) {
            seen[j] = i;
            acc[j] = 0.0;
            cols[m++] = j;
          }
          const double prod = a * B.val[q];
          acc[j] = acc[j] + prod;
        }
      }
      std::sort(cols, cols + m);
      double* vals = Cm.val.data() + Cm.ptr[i];
      for (int32_t e = 0; e < m; ++e) vals[e] = acc[cols[e]];
    }
  });
  return Cm;
}

bool dense_lu(int32_t n, std::vector<double>& a, std::vector<int32_t>& piv) {
  piv.assign(n, 0);
  for (int32_t k = 0; k < n; ++k) {
    int32_t p = k;
    double best = std::fabs(a[static_cast<size_t>(k) * n + k]);
    for (int32_t r = k + 1; r < n; ++r) {
      const double v = std::fabs(a[static_cast<size_t>(r) * n + k]);
      if (v > best) {
        best = v;
        p = r;
      }
    }
    piv[k] = p;
    if (best == 0.0) return false;
    if (p != k)
      for (int32_t c = 0; c < n; ++c) std::swap(a[static_cast<size_t>(k) * n + c], a[static_cast<size_t>(p) * n + c]);
    const double inv = a[static_cast<size_t>(k) * n + k];
    for (int32_t r = k + 1; r < n; ++r) {
      double& l = a[static_cast<size_t>(r) * n + k];
      l = l / inv;
      for (int32_t c = k + 1; c < n; ++c) {
        const double prod = l * a[static_cast<size_t>(k) * n + c];
        a[static_cast<size_t>(r) * n + c] = a[static_cast<size_t>(r) * n + c] - prod;
      }
    }
  }
  return true;
}

// ------------------------------------------------------------ block ILU(0)
bool inverse3(const double* src, double* out) {
  double a[3][3];
  double amax = 0.0;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      a[r][c] = src[3 * r + c];
      amax = std::max(amax, std::fabs(a[r][c]));
    }
  int perm[3] = {0, 1, 2};
  bool ok = amax > 0.0;
  for (int k = 0; k < 3; ++k) {
    int p = k;
    double best = std::fabs(a[k][k]);
    for (int r = k + 1; r < 3; ++r)
      if (std::fabs(a[r][k]) > best) {
        best = std::fabs(a[r][k]);
        p = r;
      }
    if (!(best > 1e-300 * amax)) ok = false;
    if (p != k) {
      for (int c = 0; c < 3; ++c) std::swap(a[k][c], a[p][c]);
      std::swap(perm[k], perm[p]);
    }
    for (int r = k + 1; r < 3; ++r) {
      a[r][k] = a[r][k] / a[k][k];
      for (int c = k + 1; c < 3; ++c) a[r][c] = a[r][c] - a[r][k] * a[k][c];
    }
  }
  if (!ok) return false;
  // column c of the inverse solves (L U) x = P e_c
  for (int c = 0; c < 3; ++c) {
    double y[3];
    for (int r = 0; r < 3; ++r) {
      double t = perm[r] == c ? 1.0 : 0.0;
      for (int m = 0; m < r; ++m) t = t - a[r][m] * y[m];
      y[r] = t;
    }
    for (int r = 2; r >= 0; --r) {
      double t = y[r];
      for (int m = r + 1; m < 3; ++m) t = t - a[r][m] * y[m];
      y[r] = t / a[r][r];
    }
    for (int r = 0; r < 3; ++r) out[3 * r + c] = y[r];
  }
  return true;
}

namespace {

// c = a b for row-major 3x3 blocks, each entry summed from 0.0 over m.
inline void mul3(const double* a, const double* b, double* c) {
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) {
      double t = 0.0;
      for (int m = 0; m < 3; ++m) t = t + a[3 * r + m] * b[3 * m + q];
      c[3 * r + q] = t;
    }
}

}  // namespace

int32_t bilu_forward_levels(int32_t n, const int32_t* rp, const int32_t* col, std::vector<int32_t>& lev) {
  lev.assign(n, 0);
  int32_t nlev = 0;
  for (int32_t i = 0; i < n; ++i) {
    int32_t m = -1;
    for (int32_t p = rp[i]; p < rp[i + 1] && col[p] < i; ++p) m = std::max(m, lev[col[p]]);
    lev[i] = m + 1;
    nlev = std::max(nlev, m + 2);
  }
  return nlev;
}

int32_t bilu_backward_levels(int32_t n, const int32_t* rp, const int32_t* col, std::vector<int32_t>& lev) {
  lev.assign(n, 0);
  int32_t nlev = 0;
  for (int32_t i = n - 1; i >= 0; --i) {
    int32_t m = -1;
    for (int32_t p = rp[i + 1] - 1; p >= rp[i] && col[p] > i; --p) m = std::max(m, lev[col[p]]);
    lev[i] = m + 1;
    nlev = std::max(nlev, m + 2);
  }
  return nlev;
}

int32_t bilu0_factor(int32_t n, const int32_t* rp, const int32_t* col, const std::vector<int32_t>& flev,
                     double* lu, double* uinv) {
  // rows grouped by forward level (ascending index inside a level)
  int32_t nlev = 0;
  for (int32_t i = 0; i < n; ++i) nlev = std::max(nlev, flev[i] + 1);
  std::vector<int32_t> off(nlev + 1, 0), rows(n);
  for (int32_t i = 0; i < n; ++i) off[flev[i] + 1]++;
  for (int32_t l = 0; l < nlev; ++l) off[l + 1] += off[l];
  {
    std::vector<int32_t> next(off.begin(), off.end() - 1);
    for (int32_t i = 0; i < n; ++i) rows[next[flev[i]]++] = i;
  }
  std::atomic<int32_t> bad{std::numeric_limits<int32_t>::max()};
  auto factor_row = [&](int32_t i) {
    const int32_t a = rp[i], b = rp[i + 1];
    int32_t dpos = -1;
    for (int32_t p = a; p < b; ++p) {
      const int32_t k = col[p];
      if (k == i) dpos = p;
      if (k >= i) continue;
      double l[9];
      mul3(lu + 9 * static_cast<int64_t>(p), uinv + 9 * static_cast<int64_t>(k), l);
      std::copy(l, l + 9, lu + 9 * static_cast<int64_t>(p));
      // A_ij -= L_ik U_kj over the j > k that both rows store (both sorted)
      int32_t t = p + 1;
      for (int32_t q = rp[k]; q < rp[k + 1]; ++q) {
        const int32_t j = col[q];
        if (j <= k) continue;
        while (t < b && col[t] < j) ++t;
        if (t == b) break;
        if (col[t] != j) continue;
        double prod[9];
        mul3(l, lu + 9 * static_cast<int64_t>(q), prod);
        double* dst = lu + 9 * static_cast<int64_t>(t);
        for (int e = 0; e < 9; ++e) dst[e] = dst[e] - prod[e];
      }
    }
    if (dpos < 0 || !inverse3(lu + 9 * static_cast<int64_t>(dpos), uinv + 9 * static_cast<int64_t>(i))) {
      int32_t cur = bad.load();
      while (i < cur && !bad.compare_exchange_weak(cur, i)) {
      }
    }
  };
  for (int32_t l = 0; l < nlev; ++l) {
    const int32_t r0 = off[l], r1 = off[l + 1], cnt = r1 - r0;
    if (cnt < 4096) {
      for (int32_t q = r0; q < r1; ++q) factor_row(rows[q]);
    } else {
      const int nch = std::min(64, cnt / 1024);
      parallel_for(nch, [&](int ch, int) {
        const int32_t q0 = r0 + static_cast<int32_t>(static_cast<int64_t>(cnt) * ch / nch);
        const int32_t q1 = r0 + static_cast<int32_t>(static_cast<int64_t>(cnt) * (ch + 1) / nch);
        for (int32_t q = q0; q < q1; ++q) factor_row(rows[q]);
      });
    }
    if (bad.load() != std::numeric_limits<int32_t>::max()) break;
  }
  const int32_t first_bad = bad.load();
  return first_bad == std::numeric_limits<int32_t>::max() ? -1 : first_bad;
}

// ------------------------------------------------------------ pairwise matching
int32_t pairwise_matching(const HostCsr& A, double beta, std::vector<int32_t>& agg) {
  const int32_t n = A.n_rows;
  const HostCsr T = transpose(A);
  // Strong set of row i: with s_ij = a_ij/2 + a_ji/2 over the merged
  // columns j != i of row i of A and of A^T (ascending), the j with
  // s_ij < -beta max_k(-s_ik), when that maximum is positive.  Rows are
  // independent: a counting pass, then a filling pass, over row chunks.
  std::vector<int64_t> Sp(static_cast<size_t>(n) + 1, 0);
  std::vector<int32_t> Sc;
  std::vector<double> Sv;  // s_ij of each strong entry
  RowChunks rc(n);
  // mc, mv: the chunk's own scratch for the merged row
  auto strong_row = [&](int32_t i, std::vector<int32_t>& mc, std::vector<double>& mv, int32_t* out_c,
                        double* out_v) -> int64_t {
    mc.clear();
    mv.clear();
    int32_t p = A.ptr[i], q = T.ptr[i];
    const int32_t pe = A.ptr[i + 1], qe = T.ptr[i + 1];
    while (p < pe || q < qe) {
      const int32_t jp = p < pe ? A.col[p] : std::numeric_limits<int32_t>::max();
      const int32_t jq = q < qe ? T.col[q] : std::numeric_limits<int32_t>::max();
      const int32_t j = std::min(jp, jq);
      const bool has_ij = jp == j, has_ji = jq == j;
      const double h_ij = has_ij ? A.val[p] / 2.0 : 0.0;
      const double h_ji = has_ji ? T.val[q] / 2.0 : 0.0;
      if (has_ij) ++p;
      if (has_ji) ++q;
      if (j == i) continue;
      // the half-entry of the lower-numbered row first
      const bool lo_first = i < j;
      const bool has_lo = lo_first ? has_ij : has_ji, has_hi = lo_first ? has_ji : has_ij;
      const double h_lo = lo_first ? h_ij : h_ji, h_hi = lo_first ? h_ji : h_ij;
      double acc = 0.0;
      if (has_lo) acc = acc + h_lo;
      if (has_hi) acc = acc + h_hi;
      mc.push_back(j);
      mv.push_back(acc);
    }
    double top = 0.0;
    for (size_t e = 0; e < mv.size(); ++e) top = e == 0 ? -mv[e] : std::max(top, -mv[e]);
    int64_t c = 0;
    if (!mv.empty() && top > 0.0)
      for (size_t e = 0; e < mv.size(); ++e)
        if (mv[e] < -beta * top) {
          if (out_c) {
            out_c[c] = mc[e];
            out_v[c] = mv[e];
          }
          ++c;
        }
    return c;
  };
  parallel_chunks(rc.n_chunks, [&](int ch, int) {
    std::vector<int32_t> mc;
    std::vector<double> mv;
    for (int32_t i = rc.begin(ch); i < rc.end(ch); ++i) Sp[i + 1] = strong_row(i, mc, mv, nullptr, nullptr);
  });
  for (int32_t i = 0; i < n; ++i) Sp[i + 1] += Sp[i];
  Sc.resize(static_cast<size_t>(Sp[n]));
  Sv.resize(static_cast<size_t>(Sp[n]));
  parallel_chunks(rc.n_chunks, [&](int ch, int) {
    std::vector<int32_t> mc;
    std::vector<double> mv;
    for (int32_t i = rc.begin(ch); i < rc.end(ch); ++i) strong_row(i, mc, mv, Sc.data() + Sp[i], Sv.data() + Sp[i]);
  });
  std::vector<int64_t> m(n, 0);
  for (int32_t i = 0; i < n; ++i)
    for (int64_t e = Sp[i]; e < Sp[i + 1]; ++e) m[Sc[e]] += 1;
  // The unaggregated nodes in ascending (m_i, i).  m_i only falls, so one
  // IndexSet per value of m up to kCap holds them, with a pointer to the
  // lowest non-empty set; the rarer nodes of larger m wait in an ordered set
  // and move into the sets once m_i reaches kCap.
  constexpr int64_t kCap = 63;
  int64_t max_m = 0;
  for (int32_t i = 0; i < n; ++i) max_m = std::max(max_m, m[i]);
  const int64_t n_sets = std::min(max_m, kCap) + 1;
  std::vector<IndexSet> bucket;
  bucket.reserve(static_cast<size_t>(n_sets));
  for (int64_t v = 0; v < n_sets; ++v) bucket.emplace_back(n);
  std::set<std::pair<int64_t, int32_t>> high;
  for (int32_t i = 0; i < n; ++i) {
    if (m[i] <= kCap)
      bucket[m[i]].insert(i);
    else
      high.insert({m[i], i});
  }
  auto take_out = [&](int32_t k) {
    if (m[k] <= kCap)
      bucket[m[k]].erase(k);
    else
      high.erase({m[k], k});
  };
  int64_t low = 0;
  agg.assign(n, -1);
  int32_t n_agg = 0;
  while (true) {
    while (low < n_sets && bucket[low].empty()) ++low;
    int32_t i;
    if (low < n_sets) {
      i = bucket[low].first();
    } else if (!high.empty()) {
      i = high.begin()->second;
    } else {
      break;
    }
    take_out(i);
    int32_t best = -1;
    double best_v = 0.0;
    for (int64_t e = Sp[i]; e < Sp[i + 1]; ++e) {
      const int32_t j = Sc[e];
      if (agg[j] >= 0) continue;
      if (best < 0 || Sv[e] < best_v) {
        best = j;
        best_v = Sv[e];
      }
    }
    if (best >= 0) take_out(best);
    const int32_t members[2] = {i, best};
    const int nm = best < 0 ? 1 : 2;
    for (int t = 0; t < nm; ++t) agg[members[t]] = n_agg;
    for (int t = 0; t < nm; ++t)
      for (int64_t e = Sp[members[t]]; e < Sp[members[t] + 1]; ++e) {
        const int32_t k = Sc[e];
        if (agg[k] >= 0) {
          m[k] -= 1;
          continue;
        }
        take_out(k);
        m[k] -= 1;
        if (m[k] <= kCap) {
          bucket[m[k]].insert(k);
          low = std::min(low, m[k]);
        } else {
          high.insert({m[k], k});
        }
      }
    ++n_agg;
  }
  return n_agg;
}

HostCsr aggregation_matrix(const std::vector<int32_t>& agg, int32_t n_agg) {
  HostCsr P;
  const int32_t n = static_cast<int32_t>(agg.size());
  P.n_rows = n;
  P.n_cols = n_agg;
  P.ptr.resize(n + 1);
  P.col.resize(n);
  P.val.resize(n);
  for (int32_t i = 0; i <= n; ++i) P.ptr[i] = i;
  for (int32_t i = 0; i < n; ++i) {
    P.col[i] = agg[i];
    P.val[i] = 1.0;
  }
  return P;
}

int32_t npair_aggregates(const HostCsr& A, double beta, int npair, std::vector<int32_t>& agg) {
  const int32_t n = A.n_rows;
  agg.resize(n);
  for (int32_t i = 0; i < n; ++i) agg[i] = i;
  int32_t n_agg = n;
  HostCsr Ak;
  const HostCsr* cur = &A;
  for (int pass = 0; pass < npair; ++pass) {
    std::vector<int32_t> a;
    const int32_t na = pairwise_matching(*cur, beta, a);
    for (int32_t i = 0; i < n; ++i) agg[i] = a[agg[i]];
    n_agg = na;
    if (pass + 1 < npair) {
      const HostCsr P = aggregation_matrix(a, na);
      const HostCsr R = transpose(P);
      Ak = spgemm_ordered(R, spgemm_ordered(*cur, P));
      cur = &Ak;
    }
  }
  return n_agg;
}

}  // namespace cpr
