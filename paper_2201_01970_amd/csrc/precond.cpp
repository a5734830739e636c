// The CPR preconditioner on the device (Section 3.1, Algorithm "CPR method"):
// stage 1 = one V-cycle of the pressure AMG smoothed by PGS-SCM (Section 5.2),
// stage 2 = one forward multi-colour block Gauss-Seidel sweep, fused with the
// prolongation Pi_P and the residual r = v - A z.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <future>
#include <numeric>

#include "solver.hpp"

namespace cpr {

namespace {

// Host SELL-64 image of a CSR matrix with rows in `order` and columns mapped
// through `colmap`; entries keep their stored order.
template <typename T>
struct SellHost {
  int32_t n_rows = 0;
  int32_t uniform = 0;  // width of every slice when all are equal, else 0
  HostVec<int32_t> slice_ptr, col;
  HostVec<T> val;
};

// Chunks of about `per` items for parallel_for (at most 256).
int chunks_of(int64_t n, int64_t per) {
  return static_cast<int>(std::min<int64_t>(256, std::max<int64_t>(1, n / per)));
}

// When padding every slice to the widest one costs at most 5% more slots, all
// slices get that width (uniform = the width), which lets the kernels compute
// a slice's slot range instead of loading it.  The slots are filled slice by
// slice in parallel, padding included (column -1, value 0).
template <typename T>
SellHost<T> build_sell(const HostCsr& A, const std::vector<int32_t>& order, const std::vector<int32_t>& colmap) {
  SellHost<T> S;
  const int32_t n = static_cast<int32_t>(order.size());
  S.n_rows = n;
  const int32_t ns = (n + kWave - 1) / kWave;
  std::vector<int32_t> width(ns, 0);
  int32_t wmax = 0;
  int64_t wsum = 0;
  for (int32_t s = 0; s < ns; ++s) {
    int32_t w = 0;
    for (int32_t p = s * kWave; p < std::min(n, (s + 1) * kWave); ++p) {
      const int32_t i = order[p];
      w = std::max(w, A.ptr[i + 1] - A.ptr[i]);
    }
    width[s] = w;
    wmax = std::max(wmax, w);
    wsum += w;
  }
  if (ns > 0 && wmax > 0 && static_cast<int64_t>(ns) * wmax * 20 <= wsum * 21) {
    S.uniform = wmax;
    std::fill(width.begin(), width.end(), wmax);
  }
  S.slice_ptr.assign(ns + 1, 0);
  for (int32_t s = 0; s < ns; ++s) S.slice_ptr[s + 1] = S.slice_ptr[s] + width[s];
  const int64_t slots = S.slice_ptr[ns];
  S.col.resize(static_cast<size_t>(slots) * kWave);
  S.val.resize(static_cast<size_t>(slots) * kWave);
  const int nch = chunks_of(ns, 64);
  parallel_for(nch, [&](int ch, int) {
    const int32_t s0 = static_cast<int32_t>(static_cast<int64_t>(ns) * ch / nch);
    const int32_t s1 = static_cast<int32_t>(static_cast<int64_t>(ns) * (ch + 1) / nch);
    for (int32_t s = s0; s < s1; ++s)
      for (int32_t lane = 0; lane < kWave; ++lane) {
        const int32_t p = s * kWave + lane;
        int32_t q = 0, q1 = 0;
        if (p < n) {
          q = A.ptr[order[p]];
          q1 = A.ptr[order[p] + 1];
        }
        for (int32_t t = S.slice_ptr[s]; t < S.slice_ptr[s + 1]; ++t) {
          const size_t e = static_cast<size_t>(t) * kWave + lane;
          if (q < q1) {
            S.col[e] = colmap.empty() ? A.col[q] : colmap[A.col[q]];
            S.val[e] = static_cast<T>(A.val[q]);
            ++q;
          } else {
            S.col[e] = kPadCol;
            S.val[e] = static_cast<T>(0);
          }
        }
      }
  });
  return S;
}

// A level matrix on the device in the form its size and row lengths call for.
// One lane per row (SELL-64) costs two ALU operations per entry and streams
// perfectly, but walks each row serially, so it needs short rows and many rows
// in flight; a 16-lane group per row (CSR) issues up to 64 entries of a row at
// once, so long rows and small levels finish in one memory round trip, at the
// price of the in-order broadcast sum.  Measured at 3.28M DOF on MI355X: SELL
// wins on the finest levels (about 7 and 15 entries per row) and on P and R at
// scale, 16-lane groups win on every Galerkin level with 30-90 entries per row
// (about 2x faster than 32- or 64-lane groups) and on all small matrices.
// Quad-vector rows (four lanes, 16 entries per chunk, sixteen rows per
// wavefront) win over 16-lane rows while rows average at most 24 entries or
// all fit two quad chunks (32 entries: a 16-lane chunk of 64 would leave most
// lanes idle).
constexpr int32_t kSellRows = 32768;
constexpr double kSellAvg = 10.0;
constexpr double kQuadAvg = 24.0;
constexpr int32_t kQuadMax = 32;

int32_t layout_for(int32_t policy, int32_t n, double avg, int32_t max_len) {
  if (policy != 0) return policy;
  if (n >= kSellRows && avg <= kSellAvg) return 1;
  return (avg <= kQuadAvg || max_len <= kQuadMax) ? 4 : 2;
}

// Requests a row keeps in flight.  SELL and one-entry-per-lane CSR: enough
// that nine rows (or slices) in ten finish in one batch (each further batch
// costs two dependent memory round trips), no more (the registers held per
// lane limit the waves in flight); SELL: slots of a slice, 8/16/32; 16-lane
// CSR: chunks of 16 entries, 4/8/16.  The quad-vector layouts take every row
// in one batch up to 128 (quad: chunks of 16 entries, 2/4/8) or 512 entries
// (16 lanes x 4: chunks of 64, 1/2/4/8): a colour kernel lasts as long as
// its longest row, and on the Galerkin levels the longest rows are about
// twice the 90th percentile, so a p90-sized batch would give them a second
// pass of loads and gathers (1-1.5 us per colour at 3.28M DOF).
int32_t p90(std::vector<int32_t> v) {
  if (v.empty()) return 0;
  const size_t k = static_cast<size_t>(0.9 * (v.size() - 1));
  std::nth_element(v.begin(), v.begin() + k, v.end());
  return v[k];
}

int32_t csr_depth(const HostCsr& A, int32_t group) {
  std::vector<int32_t> len(A.n_rows);
  int32_t wmax = 0;
  for (int32_t i = 0; i < A.n_rows; ++i) {
    len[i] = A.ptr[i + 1] - A.ptr[i];
    wmax = std::max(wmax, (len[i] + 3) / 4 * 4);  // padded to a multiple of four
  }
  if (group == 4) return wmax <= 32 ? 2 : (wmax <= 64 ? 4 : 8);
  if (group == 2) return wmax <= 64 ? 1 : (wmax <= 128 ? 2 : (wmax <= 256 ? 4 : 8));
  const int32_t w = p90(std::move(len));
  return w <= 64 ? 4 : (w <= 128 ? 8 : 16);
}

int32_t sell_depth(const HostVec<int32_t>& slice_ptr) {
  std::vector<int32_t> width(slice_ptr.size() > 0 ? slice_ptr.size() - 1 : 0);
  for (size_t s = 0; s < width.size(); ++s) width[s] = slice_ptr[s + 1] - slice_ptr[s];
  const int32_t w = p90(std::move(width));
  return w <= 8 ? 8 : (w <= 16 ? 16 : 32);
}

template <typename T>
struct DevMat {
  int32_t n_rows = 0;
  int32_t group = 1;
  int32_t depth = 8;
  int32_t width = 0;
  int64_t stored = 0;  // stored entries including SELL padding
  int32_t* ptr = nullptr;
  int32_t* col = nullptr;
  T* val = nullptr;
  MatView<T> view() const { return MatView<T>{n_rows, group, depth, width, ptr, col, val}; }
};

// Host image of a level matrix in the storage form its size and row lengths
// call for (built on a worker thread, uploaded afterwards).
template <typename T>
struct HostMat {
  int32_t n_rows = 0, group = 1, depth = 8, width = 0;
  HostVec<int32_t> ptr, col;
  HostVec<T> val;
};

template <typename T>
HostMat<T> build_mat(const HostCsr& A, const std::vector<int32_t>& order, const std::vector<int32_t>& colmap,
                     int32_t policy, bool force_csr = false) {
  HostMat<T> M;
  const int32_t n = static_cast<int32_t>(order.size());
  M.n_rows = n;
  const double avg = n > 0 ? static_cast<double>(A.nnz()) / n : 0.0;
  int32_t max_len = 0;
  for (int32_t i = 0; i < A.n_rows; ++i) max_len = std::max(max_len, A.ptr[i + 1] - A.ptr[i]);
  int32_t layout = layout_for(policy, n, avg, max_len);
  if (force_csr) layout = 4;
  if (layout == 1) {
    SellHost<T> S = build_sell<T>(A, order, colmap);
    M.group = 1;
    M.depth = sell_depth(S.slice_ptr);
    M.width = S.uniform;
    M.ptr = std::move(S.slice_ptr);
    M.col = std::move(S.col);
    M.val = std::move(S.val);
    return M;
  }
  // Quad-vector CSR pads every row to a multiple of four entries (column -1,
  // value 0), so each row starts on a 16-byte boundary of the column array.
  // Row offsets first, then the rows filled in parallel.
  const int32_t pad = (layout == 4 || layout == 2) ? 4 : 1;
  M.ptr.assign(n + 1, 0);
  for (int32_t p = 0; p < n; ++p) {
    const int32_t i = order[p];
    M.ptr[p + 1] = M.ptr[p] + (A.ptr[i + 1] - A.ptr[i] + pad - 1) / pad * pad;
  }
  M.col.resize(M.ptr[n]);
  M.val.resize(M.ptr[n]);
  const int nch = chunks_of(n, 2048);
  parallel_for(nch, [&](int ch, int) {
    const int32_t p0 = static_cast<int32_t>(static_cast<int64_t>(n) * ch / nch);
    const int32_t p1 = static_cast<int32_t>(static_cast<int64_t>(n) * (ch + 1) / nch);
    for (int32_t p = p0; p < p1; ++p) {
      const int32_t i = order[p];
      int32_t e = M.ptr[p];
      for (int32_t q = A.ptr[i]; q < A.ptr[i + 1]; ++q, ++e) {
        M.col[e] = colmap.empty() ? A.col[q] : colmap[A.col[q]];
        M.val[e] = static_cast<T>(A.val[q]);
      }
      for (; e < M.ptr[p + 1]; ++e) {
        M.col[e] = kPadCol;
        M.val[e] = static_cast<T>(0);
      }
    }
  });
  M.group = layout;
  M.depth = csr_depth(A, layout);
  return M;
}

template <typename T>
DevMat<T> upload_mat(Arena& ar, const HostMat<T>& M) {
  DevMat<T> D;
  D.n_rows = M.n_rows;
  D.group = M.group;
  D.depth = M.depth;
  D.width = M.width;
  D.stored = static_cast<int64_t>(M.col.size());
  D.ptr = ar.upload(M.ptr);
  D.col = ar.upload(M.col);
  D.val = ar.upload(M.val);
  return D;
}

// Stored entries of A in the quad-vector layout (rows padded to a multiple
// of four).
int64_t quad_stored(const HostCsr& A) {
  int64_t m = 0;
  for (int32_t i = 0; i < A.n_rows; ++i) m += (A.ptr[i + 1] - A.ptr[i] + 3) / 4 * 4;
  return m;
}

// LDS layout of the tail kernel when it starts at level `first` and stages
// the sweep matrices of the smoothed levels from `staged` down (see
// TailLayout): the image holds the coarsest LU factors (n_c <= 64), then per
// smoothed level, from an even word, its diagonal (T), colour offsets and the
// row pointers of A and P (n + 1 each, rows padded in the quad-vector layout
// keep their count) and of R (next level's n + 1), then rperm (n_c), padded to
// a multiple of four words, then per staged level the columns and the values
// of its sweep matrix (each a multiple of four words).  Vectors: x, b, r, s0,
// s1 of each smoothed level (5 n + 3 elements: x, s0 and s1 carry the zero
// entry), x and b of the coarsest level.
template <typename T>
TailLayout tail_layout(const std::vector<HostLevel>& hl, int first, int staged) {
  const int nl = static_cast<int>(hl.size());
  const int64_t nc = hl[nl - 1].A.n_rows;
  int64_t w = nc <= kWave ? 2 * nc * nc : 0;
  int64_t t = 2 * nc;
  for (int l = first; l + 1 < nl; ++l) {
    const int64_t n = hl[l].A.n_rows;
    w += w & 1;
    w += (n * static_cast<int64_t>(sizeof(T)) + 3) / 4;
    w += static_cast<int64_t>(hl[l].coff.size()) + 2 * (n + 1) + (hl[l + 1].A.n_rows + 1);
    t += 5 * n + 3;
  }
  TailLayout lay;
  lay.w_rperm = static_cast<int32_t>(w);
  w += nc;
  w = (w + 3) / 4 * 4;
  for (int l = std::max(first, staged); l + 1 < nl; ++l) {
    const int64_t m = quad_stored(hl[l].A);
    w += m + m * static_cast<int64_t>(sizeof(T)) / 4;
  }
  lay.img_words = static_cast<int32_t>(w);
  lay.xs_off = static_cast<int32_t>(w);
  lay.v_off = static_cast<int32_t>(w + (nc > kWave ? 2 * nc : 0));
  lay.lds_bytes = 4 * static_cast<size_t>(lay.v_off) + static_cast<size_t>(t) * sizeof(T);
  return lay;
}

std::vector<int32_t> inverse_perm(const std::vector<int32_t>& perm) {
  std::vector<int32_t> inv(perm.size());
  for (size_t p = 0; p < perm.size(); ++p) inv[perm[p]] = static_cast<int32_t>(p);
  return inv;
}

// Rows grouped by level (ascending index inside a level): order[q] = row,
// off[l] = first position of level l.
void level_order(const std::vector<int32_t>& lev, int32_t nlev, std::vector<int32_t>& order,
                 std::vector<int32_t>& off) {
  const int32_t n = static_cast<int32_t>(lev.size());
  off.assign(nlev + 1, 0);
  for (int32_t i = 0; i < n; ++i) off[lev[i] + 1]++;
  for (int32_t l = 0; l < nlev; ++l) off[l + 1] += off[l];
  std::vector<int32_t> next(off.begin(), off.end() - 1);
  order.resize(n);
  for (int32_t i = 0; i < n; ++i) order[next[lev[i]]++] = i;
}

// Block SELL-64 image of the rows order[q]: for row i, the stored blocks k of
// [rp[i], rp[i+1]) whose column passes keep(i, col[k]), in stored order; a
// block contributes `planes` values src[k*stride + e] (e < planes), one plane
// each; rows are padded at the end with column -1 and zero values.
template <typename T>
struct BlockSellHost {
  std::vector<int32_t> sp;
  HostVec<int32_t> col;
  HostVec<T> val;
};

template <typename T, typename Keep>
BlockSellHost<T> build_block_sell(const std::vector<int32_t>& order, const HostVec<int32_t>& rp,
                                  const HostVec<int32_t>& col, const double* src, int stride, int planes, Keep keep) {
  BlockSellHost<T> S;
  const int32_t n = static_cast<int32_t>(order.size());
  const int32_t ns = (n + kWave - 1) / kWave;
  S.sp.assign(ns + 1, 0);
  for (int32_t s = 0; s < ns; ++s) {
    int32_t w = 0;
    for (int32_t q = s * kWave; q < std::min(n, (s + 1) * kWave); ++q) {
      const int32_t i = order[q];
      int32_t c = 0;
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k) c += keep(i, col[k]) ? 1 : 0;
      w = std::max(w, c);
    }
    S.sp[s + 1] = S.sp[s] + w;
  }
  const int64_t slots = S.sp[ns];
  S.col.resize(static_cast<size_t>(slots) * kWave);
  S.val.resize(static_cast<size_t>(slots) * kWave * planes);
  parallel_for(chunks_of(ns, 64), [&](int ch, int) {
    const int nch = chunks_of(ns, 64);
    const int32_t s0 = static_cast<int32_t>(static_cast<int64_t>(ns) * ch / nch);
    const int32_t s1 = static_cast<int32_t>(static_cast<int64_t>(ns) * (ch + 1) / nch);
    for (int32_t s = s0; s < s1; ++s)
      for (int32_t lane = 0; lane < kWave; ++lane) {
        const int32_t q = s * kWave + lane;
        int32_t k = 0, k1 = 0, i = -1;
        if (q < n) {
          i = order[q];
          k = rp[i];
          k1 = rp[i + 1];
        }
        for (int32_t t = S.sp[s]; t < S.sp[s + 1]; ++t) {
          while (k < k1 && !keep(i, col[k])) ++k;
          const size_t e = static_cast<size_t>(t) * kWave + lane;
          if (k < k1) {
            S.col[e] = col[k];
            for (int p = 0; p < planes; ++p)
              S.val[(static_cast<size_t>(t) * planes + p) * kWave + lane] =
                  static_cast<T>(src[static_cast<int64_t>(k) * stride + p]);
            ++k;
          } else {
            S.col[e] = kPadCol;
            for (int p = 0; p < planes; ++p) S.val[(static_cast<size_t>(t) * planes + p) * kWave + lane] = T(0);
          }
        }
      }
  });
  return S;
}

}  // namespace

template <typename T>
class Precond final : public PrecondBase {
 public:
  struct Level {
    int32_t n = 0;
    int64_t nnz = 0, nnz_p = 0, nnz_r = 0;
    std::vector<int32_t> coff;
    std::vector<double> colour_bytes;  // algorithmic bytes of each colour launch
    DevMat<T> A, P, R;
    T *diag = nullptr, *x = nullptr, *b = nullptr, *r = nullptr, *s0 = nullptr, *s1 = nullptr;
    int32_t* perm = nullptr;
  };

  Precond(const cpr_params& prm, int32_t n_b, const std::vector<HostLevel>& hl, const std::vector<double>& lu,
          const std::vector<int32_t>& piv, const std::vector<int32_t>& bperm, const std::vector<int32_t>& bcoff,
          const HostVec<int32_t>& h_row_ptr, const HostVec<int32_t>& h_col,
          const std::vector<int32_t>& bcolour, const double* d_vals_in, const HostBilu* bilu, const double* d_w,
          hipStream_t s)
      : pre_(prm.pre_sweeps),
        post_(prm.post_sweeps),
        n_b_(n_b),
        bilu_(bilu != nullptr),
        pgs_no_(prm.smoother == 1),
        chunks_(prm.smoother_chunks),
        ua_(prm.amg_kind == 1),
        cinv_mode_(prm.amg_kind == 1 || prm.coarse_solver == 1),
        inner_(prm.amli_inner) {
    const int nl = static_cast<int>(hl.size());
    lv_.resize(nl);
    const double sv = sizeof(T);
    // host image of the stage-2 matrix (SELL-64 in block-colour order, with a
    // flag on columns of earlier colours), built while the levels are prepared
    struct Stage2Image {
      std::vector<int32_t> sp, col;
      HostVec<int64_t> pos, diag_pos;  // written in full below
      std::vector<double> bytes;
    };
    std::future<Stage2Image> stage2_task;
    if (!bilu_) stage2_task = std::async(std::launch::async, [&]() {
      Stage2Image S;
      const int32_t n = n_b;
      const int32_t ns = (n + kWave - 1) / kWave;
      S.sp.assign(ns + 1, 0);
      for (int32_t s2 = 0; s2 < ns; ++s2) {
        int32_t w = 0;
        for (int32_t q = s2 * kWave; q < std::min(n, (s2 + 1) * kWave); ++q) {
          const int32_t i = bperm[q];
          w = std::max(w, h_row_ptr[i + 1] - h_row_ptr[i]);
        }
        S.sp[s2 + 1] = S.sp[s2] + w;
      }
      const int64_t slots = S.sp[ns];
      S.col.assign(static_cast<size_t>(slots) * kWave, kPadCol);
      S.pos.resize(h_col.size());
      S.diag_pos.resize(n);
      S.bytes.assign(bcoff.size() > 0 ? bcoff.size() - 1 : 0, 0.0);
      for (int32_t q = 0; q < n; ++q) {
        const int32_t i = bperm[q], s2 = q / kWave, lane = q % kWave;
        int32_t t = S.sp[s2];
        const int cidx = bcolour[i];
        for (int32_t k = h_row_ptr[i]; k < h_row_ptr[i + 1]; ++k, ++t) {
          const size_t e = static_cast<size_t>(t) * kWave + lane;
          const int32_t j = h_col[k];
          const bool earlier = bcolour[j] < bcolour[i];
          S.col[e] = j | (earlier ? kEarlierBit : 0);
          S.pos[k] = static_cast<int64_t>(e);
          if (j == i) S.diag_pos[q] = k;
          S.bytes[cidx] += (earlier ? 9.0 : 3.0) * sv + 4.0;
        }
        S.bytes[cidx] += 24.0 + 13.0 * sv;
      }
      return S;
    });
    std::vector<std::vector<int32_t>> inv(nl);
    for (int l = 0; l < nl; ++l) inv[l] = inverse_perm(hl[l].perm);
    // First level of the one-workgroup tail: every level from it down has at
    // most tail_nnz stored entries and the tail's LDS layout fits one
    // workgroup.
    const int32_t n_last = hl[nl - 1].A.n_rows;
    const size_t lds_limit = tail_lds_limit();
    auto lds_for = [&](int first, int staged) { return tail_layout<T>(hl, first, staged).lds_bytes; };
    tail_ = nl - 1;
    // the one-workgroup tail runs PGS-SCM sweeps of a V-cycle; PGS-NO keeps
    // every smoothed level on its own kernels; a coarsest level solved by its
    // inverse (always for the aggregation AMG) leaves no tail
    if (cinv_mode_) tail_ = nl;
    if (prm.tail_nnz > 0 && !pgs_no_ && !cinv_mode_)
      while (tail_ > 0 && hl[tail_ - 1].A.nnz() <= prm.tail_nnz && lds_for(tail_ - 1, nl) <= lds_limit) --tail_;
    if (!cinv_mode_ && lds_for(tail_, nl) > lds_limit)
      throw Error(CPR_ERR_INVALID_ARG, "the coarsest level does not fit one workgroup's LDS (lower coarse_max)");
    // the sweep matrices staged in LDS: as many levels, coarsest first, as fit
    int staged = nl - 1;
    while (staged > tail_ && lds_for(tail_, staged - 1) <= lds_limit) --staged;
    tail_lay_ = tail_layout<T>(hl, tail_, staged);
    // host images of every smoothed level, built concurrently, then uploaded
    struct LevelImage {
      HostMat<T> A, P, R;
      std::vector<T> diag;
      int64_t nnz_p = 0, nnz_r = 0;
      std::vector<double> colour_bytes;
    };
    // phase times (ms), printed to stderr when CPR_SETUP_TRACE is set
    auto clock_ms = []() {
      return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
    };
    const double t_start = clock_ms();
    double t_wait = 0.0;
    std::vector<std::future<LevelImage>> images;
    for (int l = 0; l + 1 < nl; ++l)
      images.push_back(std::async(std::launch::async, [&, l]() {
        LevelImage I;
        const HostLevel& H = hl[l];
        const bool in_tail = l >= tail_;
        const int32_t n = H.A.n_rows;
        // PGS-NO walks rows in natural order from CSR row pointers
        I.A = build_mat<T>(H.A, H.perm, inv[l], prm.row_layout, in_tail || pgs_no_);
        I.diag.resize(n);
        const int nch = chunks_of(n, 4096);
        parallel_for(nch, [&](int ch, int) {
          const int32_t p1 = static_cast<int32_t>(static_cast<int64_t>(n) * (ch + 1) / nch);
          for (int32_t p = static_cast<int32_t>(static_cast<int64_t>(n) * ch / nch); p < p1; ++p) {
            const int32_t i = H.perm[p];
            double d = 0.0;
            for (int32_t q = H.A.ptr[i]; q < H.A.ptr[i + 1]; ++q)
              if (H.A.col[q] == i) d = H.A.val[q];
            I.diag[p] = static_cast<T>(d);
          }
        });
        I.P = build_mat<T>(H.P, H.perm, inv[l + 1], prm.row_layout, in_tail);
        const HostCsr R = transpose(H.P);
        I.R = build_mat<T>(R, hl[l + 1].perm, inv[l], prm.row_layout, in_tail);
        I.nnz_p = H.P.nnz();
        I.nnz_r = R.nnz();
        for (size_t c = 0; c + 1 < H.coff.size(); ++c) {
          int64_t nz = 0;
          for (int32_t p = H.coff[c]; p < H.coff[c + 1]; ++p) {
            const int32_t i = H.perm[p];
            nz += H.A.ptr[i + 1] - H.A.ptr[i];
          }
          const int64_t rows = H.coff[c + 1] - H.coff[c];
          I.colour_bytes.push_back(nz * (sv + 4.0) + 4.0 * rows + 4.0 * rows * sv);
        }
        return I;
      }));
    // LDS image of the tail: FP64 LU factors of a coarsest level of at most 64
    // rows, then per level the diagonal, colour offsets and row pointers of A,
    // P and R, then rperm (layout as in tail_layout)
    std::vector<uint32_t> img;
    auto put = [&img](const void* p, size_t bytes) {
      const size_t w0 = img.size();
      img.resize(w0 + (bytes + 3) / 4, 0u);
      std::memcpy(img.data() + w0, p, bytes);
      return static_cast<int32_t>(w0);
    };
    auto align_even = [&img]() {
      if (img.size() & 1) img.push_back(0u);
    };
    if (n_last <= kWave) put(lu.data(), lu.size() * sizeof(double));
    std::vector<TailLevel<T>> td(nl - tail_);
    std::vector<std::vector<int32_t>> h_wcol(nl);
    std::vector<std::vector<T>> h_wval(nl);
    for (int l = 0; l < nl; ++l) {
      Level& L = lv_[l];
      const HostLevel& H = hl[l];
      L.n = H.A.n_rows;
      L.nnz = H.A.nnz();
      L.coff = H.coff;
      L.perm = ar_.upload(H.perm);
      L.x = ar_.alloc<T>(L.n);
      L.b = ar_.alloc<T>(L.n);
      if (l + 1 < nl) {
        const double tw = clock_ms();
        LevelImage I = images[l].get();
        t_wait += clock_ms() - tw;
        if (l >= tail_) {
          // the sweep matrix of the tail: diagonal and padding point at the
          // zero entry n with value 0
          TailLevel<T>& d = td[l - tail_];
          std::vector<int32_t> wcol(I.A.col.size());
          std::vector<T> wval(I.A.val.size());
          for (int32_t p = 0; p < L.n; ++p)
            for (int32_t k = I.A.ptr[p]; k < I.A.ptr[p + 1]; ++k) {
              const bool off = I.A.col[k] != kPadCol && I.A.col[k] != p;
              wcol[k] = off ? I.A.col[k] : L.n;
              wval[k] = off ? I.A.val[k] : static_cast<T>(0);
            }
          d.w_col = ar_.upload(wcol);
          d.w_val = ar_.upload(wval);
          if (l >= staged) {
            h_wcol[l] = std::move(wcol);
            h_wval[l] = std::move(wval);
          }
          align_even();
          d.w_diag = put(I.diag.data(), I.diag.size() * sizeof(T));
          d.w_coff = put(H.coff.data(), H.coff.size() * sizeof(int32_t));
          d.w_arp = put(I.A.ptr.data(), I.A.ptr.size() * sizeof(int32_t));
          d.w_prp = put(I.P.ptr.data(), I.P.ptr.size() * sizeof(int32_t));
          d.w_rrp = put(I.R.ptr.data(), I.R.ptr.size() * sizeof(int32_t));
        }
        L.A = upload_mat<T>(ar_, I.A);
        L.diag = ar_.upload(I.diag);
        L.r = ar_.alloc<T>(L.n);
        L.s0 = ar_.alloc<T>(L.n);
        L.s1 = ar_.alloc<T>(L.n);
        L.P = upload_mat<T>(ar_, I.P);
        L.R = upload_mat<T>(ar_, I.R);
        L.nnz_p = I.nnz_p;
        L.nnz_r = I.nnz_r;
        L.colour_bytes = std::move(I.colour_bytes);
      }
    }
    nL_ = lv_.back().n;
    if (cinv_mode_) build_coarse_inverse(lu, s);  // no tail kernel
    if (ua_) build_gcr();
    if (!cinv_mode_) {
    lu_ = ar_.upload(lu);
    // compose the factorisation's row swaps: (P b)_i = b[rperm[i]]
    std::vector<int32_t> rperm(piv.size());
    std::iota(rperm.begin(), rperm.end(), 0);
    for (size_t k = 0; k < piv.size(); ++k) std::swap(rperm[k], rperm[piv[k]]);
    piv_ = ar_.upload(rperm);
    const int32_t w_rperm = put(rperm.data(), rperm.size() * sizeof(int32_t));
    while (img.size() % 4 != 0) img.push_back(0u);
    for (int l = staged; l + 1 < nl; ++l) {
      TailLevel<T>& d = td[l - tail_];
      d.w_wcol = put(h_wcol[l].data(), h_wcol[l].size() * sizeof(int32_t));
      d.w_wval = put(h_wval[l].data(), h_wval[l].size() * sizeof(T));
    }
    if (static_cast<int32_t>(img.size()) != tail_lay_.img_words || w_rperm != tail_lay_.w_rperm)
      throw Error(CPR_ERR_HIP, "internal: the tail LDS image does not match its layout");
    tail_img_ = ar_.upload(img);
    // device descriptors of the tail levels, with their LDS vector offsets
    // (x, s0 and s1 of a smoothed level hold the zero entry n as well)
    int32_t off = 0;
    for (int l = tail_; l < nl; ++l) {
      Level& L = lv_[l];
      TailLevel<T>& d = td[l - tail_];
      d.n = L.n;
      if (l == tail_) {
        d.gx = L.x;
        d.gb = L.b;
      }
      if (l + 1 < nl) {
        d.off_x = off;
        d.off_b = off + L.n + 1;
        d.off_r = off + 2 * L.n + 1;
        d.off_s0 = off + 3 * L.n + 1;
        d.off_s1 = off + 4 * L.n + 2;
        off += 5 * L.n + 3;
        d.ncol = static_cast<int32_t>(L.coff.size()) - 1;
        d.a_col = L.A.col;
        d.a_val = L.A.val;
        d.p_col = L.P.col;
        d.p_val = L.P.val;
        d.r_col = L.R.col;
        d.r_val = L.R.val;
      } else {
        d.off_x = off;
        d.off_b = off + L.n;
        off += 2 * L.n;
      }
    }
    tail_dev_ = ar_.upload(td);
    tail_bytes_ = 0.0;
    for (int l = tail_; l + 1 < nl; ++l) {
      const Level& L = lv_[l];
      const double sweep = L.nnz * (sv + 4.0) + 4.0 * L.n + 4.0 * L.n * sv;
      tail_bytes_ += (pre_ + post_) * sweep + L.nnz * (sv + 4) + 4.0 * L.n + 3.0 * L.n * sv +
                     (L.nnz_r + L.nnz_p) * (sv + 4.0) + 4.0 * (L.n + lv_[l + 1].n) + 4.0 * L.n * sv;
    }
    tail_bytes_ += 8.0 * nL_ * nL_;
    }

    const double t_levels = clock_ms();
    const int32_t n = n_b;
    pe_ = ar_.alloc<T>(n);
    if (d_w) {
      wt_ = ar_.alloc<T>(static_cast<int64_t>(9) * n);
      launch_copy_cast<double, T>(static_cast<int64_t>(9) * n, d_w, wt_, s);
      wv_ = ar_.alloc<double>(static_cast<int64_t>(3) * n);
    }
    if (bilu_) {
      build_bilu(*bilu, h_row_ptr, h_col);
      if (std::getenv("CPR_SETUP_TRACE"))
        std::fprintf(stderr, "[cpr setup] device images: levels %.1f ms, block ILU(0) images %.1f\n",
                     t_levels - t_start, clock_ms() - t_levels);
      return;
    }
    // ---- fine level for stage 2: cells in block-colour order
    bcoff_ = bcoff;
    cell_ = ar_.upload(bperm);
    Stage2Image S2 = stage2_task.get();
    const double t_s2wait = clock_ms();
    std::vector<int32_t>& sp = S2.sp;
    std::vector<int32_t>& col = S2.col;
    const auto& pos = S2.pos;
    const auto& diag_pos = S2.diag_pos;
    stage2_bytes_ = std::move(S2.bytes);
    const int64_t slots = sp.back();
    fine_.n_rows = n;
    fine_.slots = slots;
    fine_.slice_ptr = ar_.upload(sp);
    fine_.col = ar_.upload(col);
    fine_.val = ar_.alloc<T>(slots * 9 * kWave);
    HIPCHK(hipMemsetAsync(fine_.val, 0, static_cast<size_t>(slots) * 9 * kWave * sizeof(T), s));
    int64_t* d_pos = ar_.upload(pos);
    launch_bsr_values_to_sell<T>(static_cast<int64_t>(pos.size()), d_vals_in, d_pos, fine_.val, s);
    int64_t* d_diag_pos = ar_.upload(diag_pos);
    dinv_ld_ = n;
    dinv_ = ar_.alloc<T>(static_cast<int64_t>(9) * n);
    int32_t* d_sing = ar_.alloc<int32_t>(1);
    HIPCHK(hipMemsetAsync(d_sing, 0, sizeof(int32_t), s));
    launch_block_inverse<T>(n, d_vals_in, d_diag_pos, dinv_, dinv_ld_, d_sing, s);
    int32_t sing = 0;
    HIPCHK(hipMemcpyAsync(&sing, d_sing, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (sing) throw Error(CPR_ERR_SINGULAR_BLOCK, "a 3x3 diagonal block is singular");
    if (std::getenv("CPR_SETUP_TRACE"))
      std::fprintf(stderr,
                   "[cpr setup] device images: levels %.1f ms (waiting for host images %.1f), stage-2 image wait "
                   "%.1f, stage 2 upload and D^-1 %.1f\n",
                   t_levels - t_start, t_wait, t_s2wait - t_levels, clock_ms() - t_s2wait);
  }

  void apply(const double* v_in, void* zv, hipStream_t s) override {
    T* z = static_cast<T*>(zv);
    const double* v = v_in;
    if (wt_) {  // decoupled rows: B acts on W v
      launch_block_gemv<T>(n_b_, wt_, v_in, wv_, s);
      v = wv_;
    }
    Level& L0 = lv_[0];
    const ZeroStart<T> zs = zero_start(0);
    launch_restrict_pressure<T>(L0.n, v, L0.perm, L0.b, zs, s);
    cycle(0, s, zs.n_first > 0);
    launch_scatter<T>(L0.n, L0.x, L0.perm, pe_, s);
    second_stage(v, z, s);
  }

  void second_stage_own(const double* v, const double* pe, double* z, hipStream_t s) override {
    launch_copy_cast<double, T>(n_b_, pe, pe_, s);
    T* zt = sizeof(T) == sizeof(double) ? reinterpret_cast<T*>(z) : work_z();
    second_stage(v, zt, s);
    if (sizeof(T) != sizeof(double)) launch_copy_cast<T, double>(3 * static_cast<int64_t>(n_b_), zt, z, s);
  }

  void vcycle_own(const double* r, double* e, hipStream_t s) override {
    Level& L0 = lv_[0];
    launch_gather<double, T>(L0.n, r, L0.perm, L0.b, s);
    cycle(0, s, false);
    launch_scatter_cast<T, double>(L0.n, L0.x, L0.perm, e, s);
  }

  void smooth_own(int l, double* x, const double* b, int sweeps, bool zero_start, hipStream_t s) override {
    if (l < 0 || l + 1 >= static_cast<int>(lv_.size())) throw Error(CPR_ERR_INVALID_ARG, "level has no smoother");
    Level& L = lv_[l];
    launch_gather<double, T>(L.n, b, L.perm, L.b, s);
    launch_gather<double, T>(L.n, x, L.perm, L.x, s);
    int cur = 0;
    if (!zero_start) launch_copy_cast<T, T>(L.n, L.x, L.s0, s);
    for (int w = 0; w < sweeps; ++w) {
      sweep(l, cur, zero_start && w == 0, s);
      cur ^= 1;
    }
    launch_scatter_cast<T, double>(L.n, L.x, L.perm, x, s);
  }

  int n_levels() const override { return static_cast<int>(lv_.size()); }
  bool fp32() const override { return sizeof(T) == 4; }
  int64_t bytes() const override { return ar_.bytes(); }

 private:
  // z = Pi_P pe_ + R (v - A Pi_P pe_), R = multi-colour block Gauss-Seidel
  // (fused per colour) or block ILU(0) (level-scheduled solves).
  void second_stage(const double* v, T* z, hipStream_t s) {
    if (bilu_) {
      const SellView<T> R = fres_.view(), Lo = flow_.view(), U = bup_.view();
      if (timer) timer->begin(CPR_KSTAT_STAGE2, s);
      launch_bilu_residual<T>(R, v, pe_, rv_, s);
      if (timer) timer->end(CPR_KSTAT_STAGE2, s, rbytes_);
      for (size_t l = 0; l + 1 < flev_off_.size(); ++l) {
        if (timer) timer->begin(CPR_KSTAT_STAGE2, s);
        launch_bilu_forward<T>(flev_off_[l], flev_off_[l + 1], Lo, frow_, rv_, yv_, s);
        if (timer) timer->end(CPR_KSTAT_STAGE2, s, fbytes_[l]);
      }
      for (size_t l = 0; l + 1 < blev_off_.size(); ++l) {
        if (timer) timer->begin(CPR_KSTAT_STAGE2, s);
        launch_bilu_backward<T>(blev_off_[l], blev_off_[l + 1], U, buinv_, n_b_, brow_, yv_, pe_, dv_, z, s);
        if (timer) timer->end(CPR_KSTAT_STAGE2, s, bbytes_[l]);
      }
      return;
    }
    const SellView<T> F = fine_.view();
    for (size_t c = 0; c + 1 < bcoff_.size(); ++c) {
      if (timer) timer->begin(CPR_KSTAT_STAGE2, s);
      launch_stage2<T>(F, bcoff_[c], bcoff_[c + 1], cell_, dinv_, dinv_ld_, v, pe_, z, s);
      if (timer) timer->end(CPR_KSTAT_STAGE2, s, stage2_bytes_[c]);
    }
  }

  T* work_z() {
    if (!zbuf_) zbuf_ = ar_.alloc<T>(3 * static_cast<int64_t>(n_b_));
    return zbuf_;
  }

  // Device images of the block ILU(0) second stage: the residual reads column
  // 0 of every block, rows in natural order; the forward solve the lower
  // factor blocks, rows in forward-level order; the backward solve the upper
  // factor blocks and the inverted pivot blocks, rows in backward-level order.
  void build_bilu(const HostBilu& F, const HostVec<int32_t>& rp, const HostVec<int32_t>& col) {
    const int32_t n = n_b_;
    const double sv = sizeof(T);
    std::vector<int32_t> forder, border;
    level_order(F.flev, F.n_flev, forder, flev_off_);
    level_order(F.blev, F.n_blev, border, blev_off_);
    auto up = [&](const BlockSellHost<T>& H, DevSell<T>& D) {
      D.n_rows = n;
      D.slots = H.sp.empty() ? 0 : H.sp.back();
      D.slice_ptr = ar_.upload(H.sp);
      D.col = ar_.upload(H.col);
      D.val = ar_.upload(H.val);
    };
    {
      std::vector<int32_t> natural(n);
      std::iota(natural.begin(), natural.end(), 0);
      auto R = build_block_sell<T>(natural, rp, col, F.acol0.data(), 3, 3, [](int32_t, int32_t) { return true; });
      up(R, fres_);
    }
    {
      auto L = build_block_sell<T>(forder, rp, col, F.lu.data(), 9, 9, [](int32_t i, int32_t j) { return j < i; });
      up(L, flow_);
    }
    {
      auto U = build_block_sell<T>(border, rp, col, F.lu.data(), 9, 9, [](int32_t i, int32_t j) { return j > i; });
      up(U, bup_);
    }
    HostVec<T> ui(static_cast<size_t>(9) * n);
    for (int32_t q = 0; q < n; ++q)
      for (int e = 0; e < 9; ++e) ui[static_cast<size_t>(e) * n + q] = static_cast<T>(F.uinv[9 * static_cast<size_t>(border[q]) + e]);
    buinv_ = ar_.upload(ui);
    frow_ = ar_.upload(forder);
    brow_ = ar_.upload(border);
    rv_ = ar_.alloc<T>(3 * static_cast<int64_t>(n));
    yv_ = ar_.alloc<T>(3 * static_cast<int64_t>(n));
    dv_ = ar_.alloc<T>(3 * static_cast<int64_t>(n));
    // algorithmic bytes per level launch: row index, blocks read, vectors
    auto level_bytes = [&](const std::vector<int32_t>& order, const std::vector<int32_t>& off, bool fwd) {
      std::vector<double> b(off.size() > 0 ? off.size() - 1 : 0, 0.0);
      for (size_t l = 0; l + 1 < off.size(); ++l)
        for (int32_t q = off[l]; q < off[l + 1]; ++q) {
          const int32_t i = order[q];
          double r = 4.0;
          for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int32_t j = col[k];
            if (fwd && j < i) r += 9.0 * sv + 4.0 + 3 * sv;   // L_ij, y_j
            if (!fwd && j > i) r += 9.0 * sv + 4.0 + 3 * sv;  // U_ij, d_j
          }
          // forward: r_i in, y_i out; backward: Uinv_i, y_i, pe_i in, d_i, z_i out
          r += fwd ? 6.0 * sv : 9.0 * sv + 3.0 * sv + sv + 6.0 * sv;
          b[l] += r;
        }
      return b;
    };
    fbytes_ = level_bytes(forder, flev_off_, true);
    bbytes_ = level_bytes(border, blev_off_, false);
    // residual: column 0 of every block with its column, pe gathers, v in, r out
    rbytes_ = static_cast<double>(rp[n]) * (3.0 * sv + 4.0 + sv) + 4.0 * n + 24.0 * n + 3.0 * sv * n;
  }

  // The first pre-sweep of a level below the tail's start begins from x = 0;
  // its first colour is then fused into the kernel that writes the level's b.
  ZeroStart<T> zero_start(int l) const {
    ZeroStart<T> zs;
    if (!pgs_no_ && !ua_ && l < tail_ && pre_ > 0 && lv_[l].coff.size() > 1) {
      const Level& L = lv_[l];
      zs.n_first = L.coff[1];
      zs.diag = L.diag;
      zs.x = L.x;
      zs.snap = L.s1;  // the output snapshot of the first sweep (S[cur ^ 1] with cur = 0)
    }
    return zs;
  }

  // first_done: the first colour was already computed by the producer of b
  void sweep(int l, int cur, bool zero, hipStream_t s, bool first_done = false) {
    Level& L = lv_[l];
    T* S[2] = {L.s0, L.s1};
    const MatView<T> A = L.A.view();
    const int kind = l == 0 ? CPR_KSTAT_SMOOTH_L0 : CPR_KSTAT_SMOOTH_COARSE;
    if (pgs_no_) {  // sweep-start snapshot, then the chunked Gauss-Seidel
      if (zero)
        launch_fill<T>(L.n, (T)0, L.x, s);
      else
        launch_copy_cast<T, T>(L.n, L.x, L.s0, s);
      if (timer) timer->begin(kind, s);
      launch_gs_chunks<T>(A, L.diag, chunks_, L.b, L.x, zero ? nullptr : L.s0, s);
      if (timer) timer->end(kind, s, L.colour_bytes.empty() ? 0.0 : L.colour_bytes[0]);
      return;
    }
    for (size_t c = first_done ? 1 : 0; c + 1 < L.coff.size(); ++c) {
      if (timer) timer->begin(kind, s);
      launch_gs_colour<T>(A, L.diag, L.coff[c], L.coff[c + 1], L.b, L.x, S[cur], S[cur ^ 1], zero, s);
      if (timer) timer->end(kind, s, L.colour_bytes[c]);
    }
  }

  void cycle(int l, hipStream_t s, bool first_done) {
    if (ua_)
      kcycle(l, s);
    else
      vcycle(l, s, first_done);
  }

  // The coarsest level solved by its explicit inverse: x = A_L^{-1} b.
  void coarse_solve(hipStream_t s) {
    Level& L = lv_.back();
    if (timer) timer->begin(CPR_KSTAT_TAIL, s);
    launch_dense_gemv<T>(L.n, cinv_, L.b, L.x, s);
    if (timer) timer->end(CPR_KSTAT_TAIL, s, 8.0 * L.n * L.n + 2.0 * sizeof(T) * L.n);
  }

  // Nonlinear AMLI-cycle on level l from x = 0, right-hand side lv_[l].b,
  // result in lv_[l].x: pre-smoothing, residual, restriction, the coarse
  // correction (the inverse on the coarsest level, else inner_ flexible GCR
  // steps preconditioned by the next level's cycle), prolongation,
  // post-smoothing.
  void kcycle(int l, hipStream_t s) {
    const int nl = static_cast<int>(lv_.size());
    if (l == nl - 1) {
      coarse_solve(s);
      return;
    }
    Level& L = lv_[l];
    const double sv = sizeof(T);
    int cur = 0;
    if (pre_ == 0) launch_fill<T>(L.n, (T)0, L.x, s);
    for (int w = 0; w < pre_; ++w) {
      sweep(l, cur, w == 0, s);
      cur ^= 1;
    }
    Level& C = lv_[l + 1];
    const int kind = l == 0 ? CPR_KSTAT_TRANSFER_L0 : CPR_KSTAT_TRANSFER_COARSE;
    if (timer) timer->begin(kind, s);
    launch_csr_residual<T>(L.A.view(), L.b, L.x, L.r, s);
    if (timer) timer->end(kind, s, L.nnz * (sv + 4) + 4.0 * L.n + 3.0 * L.n * sv);
    if (timer) timer->begin(kind, s);
    launch_csr_restrict<T>(L.R.view(), L.r, C.b, ZeroStart<T>{}, s);
    if (timer) timer->end(kind, s, L.nnz_r * (sv + 4) + 4.0 * C.n + L.n * sv + C.n * sv);
    if (l + 1 == nl - 1)
      coarse_solve(s);
    else
      gcr(l + 1, s);
    T* S[2] = {L.s0, L.s1};
    if (timer) timer->begin(kind, s);
    launch_prolong_add<T>(L.P.view(), C.x, L.x, S[cur], s);
    if (timer) timer->end(kind, s, L.nnz_p * (sv + 4) + 4.0 * L.n + C.n * sv + 2.0 * L.n * sv);
    for (int w = 0; w < post_; ++w) {
      sweep(l, cur, false, s);
      cur ^= 1;
    }
  }

  // inner_ flexible GCR steps on A_c e = f (f = lv_[c].b on entry, e left in
  // lv_[c].x), preconditioned by the cycle on level c.
  void gcr(int c, hipStream_t s) {
    Level& C = lv_[c];
    Gcr& g = gcr_[c];
    const int64_t n = C.n;
    const MatView<T> A = C.A.view();
    const int kind = CPR_KSTAT_TRANSFER_COARSE;
    kcycle(c, s);                                   // z1 = B(f)   (in C.x)
    launch_csr_spmv<T>(A, C.x, g.w1, s);            // w1 = A z1
    if (timer) timer->begin(kind, s);
    launch_gcr_dots<T>(n, g.w1, g.w1, C.b, g.w1, g.part, s);
    if (inner_ == 1) {
      launch_gcr_single<T>(n, g.part, C.x, s);      // e = alpha1 z1
      if (timer) timer->end(kind, s, 4.0 * n * sizeof(T));
      return;
    }
    launch_gcr_step1<T>(n, g.part, C.x, g.z1, C.b, g.w1, g.scal, s);  // z1 kept, f -> r1
    if (timer) timer->end(kind, s, 7.0 * n * sizeof(T));
    kcycle(c, s);                                   // z2 = B(r1)  (in C.x)
    launch_csr_spmv<T>(A, C.x, g.w2, s);            // w2 = A z2
    if (timer) timer->begin(kind, s);
    launch_gcr_dots<T>(n, g.w2, g.w1, static_cast<const T*>(nullptr), static_cast<const T*>(nullptr), g.part, s);
    launch_gcr_orth<T>(n, g.part, g.scal, g.w2, g.w1, C.x, g.z1, C.b, g.part2, s);
    launch_gcr_finish<T>(n, g.part2, g.scal, C.x, g.z1, s);  // e = alpha1 z1 + alpha2 z2
    if (timer) timer->end(kind, s, 13.0 * n * sizeof(T));
  }

  // The explicit inverse of the coarsest matrix (dense, row-major) by
  // Gauss-Jordan elimination with partial pivoting on the device, in
  // SETUP-only memory; only the inverse stays resident.
  void build_coarse_inverse(const std::vector<double>& dense, hipStream_t s) {
    const int n = nL_;
    Arena work;  // released when SETUP returns
    double* a = work.upload(dense);
    double* gj = work.alloc<double>(gj_workspace_doubles(n));
    int32_t* igj = work.alloc<int32_t>(gj_workspace_ints(n));
    int32_t* piv = work.alloc<int32_t>(n);
    int32_t* bad = work.alloc<int32_t>(1);
    launch_fill<int32_t>(1, 0, bad, s);
    launch_gj_inverse(n, a, gj, igj, piv, bad, s);
    std::vector<int32_t> hpiv(n);
    int32_t hbad = 0;
    HIPCHK(hipMemcpyAsync(hpiv.data(), piv, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hbad) throw Error(CPR_ERR_SINGULAR_COARSE, "coarsest matrix is singular");
    // undo the row interchanges as column interchanges, in reverse order
    std::vector<int32_t> cols(n);
    std::iota(cols.begin(), cols.end(), 0);
    for (int k = n - 1; k >= 0; --k) std::swap(cols[k], cols[hpiv[k]]);
    int32_t* dcols = work.upload(cols);
    cinv_ = ar_.alloc<double>(static_cast<int64_t>(n) * n);
    launch_permute_cols(n, a, dcols, cinv_, s);
    HIPCHK(hipStreamSynchronize(s));
  }

  // The GCR vectors of every level of the AMLI-cycle that gets a coarse
  // correction by GCR.
  void build_gcr() {
    const int nl = static_cast<int>(lv_.size());
    gcr_.resize(nl);
    for (int c = 1; c + 1 < nl; ++c) {
      Gcr& g = gcr_[c];
      const int64_t nc = lv_[c].n;
      g.z1 = ar_.alloc<T>(nc);
      g.w1 = ar_.alloc<T>(nc);
      g.w2 = ar_.alloc<T>(nc);
      const int G = amli_dot_grid(nc);
      g.part = ar_.alloc<double>(2 * G);
      g.part2 = ar_.alloc<double>(2 * G);
      g.scal = ar_.alloc<double>(4);
    }
  }

  // first_done: colour 0 of the first pre-sweep was fused into the producer of b
  void vcycle(int l, hipStream_t s, bool first_done) {
    Level& L = lv_[l];
    const int nl = static_cast<int>(lv_.size());
    if (cinv_mode_ && l == nl - 1) {
      coarse_solve(s);
      return;
    }
    if (l == tail_) {
      if (timer) timer->begin(CPR_KSTAT_TAIL, s);
      launch_tail_vcycle<T>(tail_dev_, nl - tail_, pre_, post_, nL_, lu_, tail_img_, tail_lay_, s);
      if (timer) timer->end(CPR_KSTAT_TAIL, s, tail_bytes_);
      return;
    }
    const double sv = sizeof(T);
    int cur = 0;
    if (pre_ == 0) launch_fill<T>(L.n, (T)0, L.x, s);
    for (int w = 0; w < pre_; ++w) {
      sweep(l, cur, w == 0, s, w == 0 && first_done);
      cur ^= 1;
    }
    Level& C = lv_[l + 1];
    const int kind = l == 0 ? CPR_KSTAT_TRANSFER_L0 : CPR_KSTAT_TRANSFER_COARSE;
    if (timer) timer->begin(kind, s);
    launch_csr_residual<T>(L.A.view(), L.b, L.x, L.r, s);
    if (timer) timer->end(kind, s, L.nnz * (sv + 4) + 4.0 * L.n + 3.0 * L.n * sv);
    const ZeroStart<T> zs = zero_start(l + 1);
    if (timer) timer->begin(kind, s);
    launch_csr_restrict<T>(L.R.view(), L.r, C.b, zs, s);
    if (timer)
      timer->end(kind, s, L.nnz_r * (sv + 4) + 4.0 * C.n + L.n * sv + C.n * sv + 3.0 * sv * zs.n_first);
    vcycle(l + 1, s, zs.n_first > 0);
    T* S[2] = {L.s0, L.s1};
    if (timer) timer->begin(kind, s);
    launch_prolong_add<T>(L.P.view(), C.x, L.x, S[cur], s);
    if (timer) timer->end(kind, s, L.nnz_p * (sv + 4) + 4.0 * L.n + C.n * sv + 2.0 * L.n * sv);
    for (int w = 0; w < post_; ++w) {
      sweep(l, cur, false, s);
      cur ^= 1;
    }
  }

  Arena ar_;
  std::vector<Level> lv_;
  int tail_ = 0;
  TailLayout tail_lay_;
  uint32_t* tail_img_ = nullptr;
  TailLevel<T>* tail_dev_ = nullptr;
  double tail_bytes_ = 0.0;
  int pre_, post_;
  int32_t n_b_;
  int32_t nL_ = 0;
  double* lu_ = nullptr;
  int32_t* piv_ = nullptr;
  std::vector<int32_t> bcoff_;
  int32_t* cell_ = nullptr;
  DevSell<T> fine_;
  T* dinv_ = nullptr;
  int32_t dinv_ld_ = 0;
  T* pe_ = nullptr;
  std::vector<double> stage2_bytes_;
  // block ILU(0) second stage
  bool bilu_ = false;
  std::vector<int32_t> flev_off_, blev_off_;
  DevSell<T> fres_, flow_, bup_;
  T* buinv_ = nullptr;
  int32_t *frow_ = nullptr, *brow_ = nullptr;
  T *rv_ = nullptr, *yv_ = nullptr, *dv_ = nullptr, *zbuf_ = nullptr;
  std::vector<double> fbytes_, bbytes_;
  double rbytes_ = 0.0;
  // decoupling weights W (n x 9 in T) and W v
  T* wt_ = nullptr;
  double* wv_ = nullptr;
  // PGS-NO smoother (natural order, chunked Gauss-Seidel)
  bool pgs_no_ = false;
  int32_t chunks_ = 1;
  // aggregation AMG with the nonlinear AMLI-cycle
  struct Gcr {
    T *z1 = nullptr, *w1 = nullptr, *w2 = nullptr;
    double *part = nullptr, *part2 = nullptr, *scal = nullptr;
  };
  bool ua_ = false;
  bool cinv_mode_ = false;  // the coarsest level is solved by its explicit inverse
  int inner_ = 2;
  double* cinv_ = nullptr;
  std::vector<Gcr> gcr_;
};

std::unique_ptr<PrecondBase> make_precond(bool fp32, const cpr_params& prm, int32_t n_b,
                                          const std::vector<HostLevel>& hl, const std::vector<double>& lu,
                                          const std::vector<int32_t>& piv, const std::vector<int32_t>& bperm,
                                          const std::vector<int32_t>& bcoff, const HostVec<int32_t>& h_row_ptr,
                                          const HostVec<int32_t>& h_col, const std::vector<int32_t>& bcolour,
                                          const double* d_vals, const HostBilu* bilu, const double* d_w,
                                          hipStream_t s) {
  if (fp32)
    return std::make_unique<Precond<float>>(prm, n_b, hl, lu, piv, bperm, bcoff, h_row_ptr, h_col, bcolour,
                                            d_vals, bilu, d_w, s);
  return std::make_unique<Precond<double>>(prm, n_b, hl, lu, piv, bperm, bcoff, h_row_ptr, h_col, bcolour,
                                           d_vals, bilu, d_w, s);
}

}  // namespace cpr
