// The solver handle: SETUP (host greedy steps + device data), the CPR apply,
// the pressure V-cycle and the FP64 flexible GMRES with the adaptive-setup rule.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/cpr.h"
#include "../../include/cpr_inspect.h"
#include "device.hpp"
#include "host_setup.hpp"

namespace cpr {

struct Error : std::runtime_error {
  cpr_status status;
  Error(cpr_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

void hip_check(hipError_t e, const char* what, const char* file, int line);
#define HIPCHK(x) ::cpr::hip_check((x), #x, __FILE__, __LINE__)

// Graph capture on one thread is invalidated by device-synchronising runtime
// calls (blocking copies, allocation and release, stream creation) issued by
// another thread meanwhile.  Every such call of the library and every capture
// holds this process-wide mutex, so handles used from different threads (the
// serving runtime) never interfere.
std::mutex& device_api_mutex();

// Owns a list of device allocations.
class Arena {
 public:
  ~Arena() { release(); }
  template <typename T>
  T* alloc(int64_t n) {
    if (n <= 0) n = 1;
    void* p = nullptr;
    const size_t bytes = static_cast<size_t>(n) * sizeof(T);
    hipError_t e;
    {
      std::lock_guard<std::mutex> lk(device_api_mutex());
      e = hipMalloc(&p, bytes);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(CPR_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    ptrs_.push_back(p);
    bytes_ += static_cast<int64_t>(bytes);
    return static_cast<T*>(p);
  }
  template <typename T, typename Alloc>
  T* upload(const std::vector<T, Alloc>& v) {
    T* p = alloc<T>(static_cast<int64_t>(v.size()));
    if (!v.empty()) {
      std::lock_guard<std::mutex> lk(device_api_mutex());
      HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    }
    return p;
  }
  void release() {
    std::lock_guard<std::mutex> lk(device_api_mutex());
    for (void* p : ptrs_) (void)hipFree(p);
    ptrs_.clear();
    bytes_ = 0;
  }
  int64_t bytes() const { return bytes_; }

 private:
  std::vector<void*> ptrs_;
  int64_t bytes_ = 0;
};

template <typename T>
struct DevSell {
  int32_t n_rows = 0;
  int64_t slots = 0;
  int32_t* slice_ptr = nullptr;
  int32_t* col = nullptr;
  T* val = nullptr;
  SellView<T> view() const { return SellView<T>{n_rows, slice_ptr, col, val}; }
};

// Host products of SETUP for one AMG level (kept for inspection).
struct HostLevel {
  HostCsr A;
  std::vector<uint8_t> mask;  // bit 1: RS strength, bit 2: eq. (strong-matrix)
  std::vector<int32_t> colour;
  int32_t n_colours = 0;
  std::vector<int8_t> cf;
  std::vector<int32_t> agg;  // aggregation AMG: aggregate of every row
  HostCsr P;
  std::vector<int32_t> perm;  // device row p -> level row perm[p]
  std::vector<int32_t> coff;  // colour offsets in device order
};

// Host products of the block ILU(0) second stage (kept for inspection): the
// factors in the input block order (lu: L_ik for k < i, U_ij for j >= i;
// uinv: inverted pivot blocks), the forward and backward level of every row,
// and column 0 of every block of the matrix B is built on (the CPR residual
// r = v - A Pi_P e only reads that column).
struct HostBilu {
  HostVec<double> lu, uinv, acol0;
  std::vector<int32_t> flev, blev;
  int32_t n_flev = 0, n_blev = 0;
};

// Event timing of kernel classes.
class Profiler : public LaunchTimer {
 public:
  ~Profiler() override;
  void enable(bool on);
  bool on() const { return on_; }
  void begin(int kind, hipStream_t s) override;
  void end(int kind, hipStream_t s, double bytes) override;
  void collect();  // after the stream has drained
  int64_t launches[CPR_KSTAT_COUNT] = {0};
  double total_ms[CPR_KSTAT_COUNT] = {0};
  double bytes[CPR_KSTAT_COUNT] = {0};

 private:
  struct Rec {
    int kind;
    hipEvent_t a, b;
    double bytes;
  };
  hipEvent_t get_event();
  bool on_ = false;
  std::vector<Rec> pending_;
  std::vector<hipEvent_t> free_;
  hipEvent_t open_ev_[CPR_KSTAT_COUNT] = {};
};

class PrecondBase {
 public:
  virtual ~PrecondBase() = default;
  // z = B v; z is a T* of 3n (T = the preconditioner precision)
  virtual void apply(const double* v, void* z, hipStream_t s) = 0;
  virtual void vcycle_own(const double* r, double* e, hipStream_t s) = 0;
  virtual void smooth_own(int level, double* x, const double* b, int sweeps, bool zero_start, hipStream_t s) = 0;
  // z = Pi_P pe + R (v - A Pi_P pe): the second stage of Algorithm "CPR method"
  // given the stage-1 pressure correction pe (FP64 in, FP64 out; n_b and 3 n_b)
  virtual void second_stage_own(const double* v, const double* pe, double* z, hipStream_t s) = 0;
  virtual int n_levels() const = 0;
  virtual bool fp32() const = 0;
  virtual int64_t bytes() const = 0;
  LaunchTimer* timer = nullptr;
};

// d_vals: the 3x3 blocks B is built on (device, input order; W A when the
// rows are decoupled, then d_w holds W, n x 9 FP64, else null); bilu: the
// block ILU(0) factors when the second stage is block ILU(0), else null (then
// bperm/bcoff/bcolour give the block colouring of the Gauss-Seidel stage).
std::unique_ptr<PrecondBase> make_precond(bool fp32, const cpr_params& prm, int32_t n_b,
                                          const std::vector<HostLevel>& hl,
                                          const std::vector<double>& lu, const std::vector<int32_t>& piv,
                                          const std::vector<int32_t>& bperm, const std::vector<int32_t>& bcoff,
                                          const HostVec<int32_t>& h_row_ptr, const HostVec<int32_t>& h_col,
                                          const std::vector<int32_t>& bcolour, const double* d_vals,
                                          const HostBilu* bilu, const double* d_w, hipStream_t s);

}  // namespace cpr

struct cpr_handle {
  cpr_params prm{};
  hipStream_t stream = nullptr;  // caller's stream (NULL = default stream)
  int device = 0;
  int32_t n_b = 0, nnz_b = 0;
  int32_t *d_rp_pat = nullptr, *d_col_pat = nullptr;  // the input pattern on the device
  int32_t* d_flag = nullptr;                           // pattern comparison result
  cpr::HostVec<int32_t> h_row_ptr, h_col;  // resize() leaves entries uninitialised

  cpr::Arena fine;  // outer matrix, input values, Krylov workspace
  cpr::DevSell<double> outer;
  int64_t* d_pos_outer = nullptr;
  double* d_vals_in = nullptr;
  int32_t* d_singular = nullptr;

  std::unique_ptr<cpr::PrecondBase> pc;
  std::vector<cpr::HostLevel> hl;
  std::vector<int32_t> block_colour;
  int32_t n_block_colours = 0;
  cpr::HostBilu bilu_host;  // block ILU(0) factors (second_stage 1)

  // Krylov workspace (FP64 except Z in FP32 mode): the bases V and Z, the
  // residual r, and the scalars and partial sums of the handle's own solves
  int m = 30;
  double *V = nullptr, *r = nullptr;
  void* Z = nullptr;
  cpr::KrylovWork kw;
  double* report_h = nullptr;  // pinned

  // adaptive setup state (Algorithm "ASCPR")
  int64_t k_solves = 0;
  int32_t it_prev = 0, it_ref = 0;
  bool values_changed = false;
  double last_setup_ms = 0.0;

  cpr::Profiler prof;
  std::string last_error;

  // one captured graph per FGMRES step index j (dropped whenever SETUP reruns)
  std::vector<hipGraphExec_t> step_graph;
  hipStream_t cap_stream = nullptr;
  void drop_graphs();
  void step_body(int j, const cpr::KrylovWork& w, bool timed, hipStream_t s);
  hipGraphExec_t capture_step(int j);

  void build_precond();
  // The FGMRES solve with the adaptive-setup rule.  w: the scalars and partial
  // sums to use; may_allocate = false runs every step eagerly (no graph
  // capture or instantiation, no event timing) and refuses a solve for which
  // the rule asks a SETUP (SETUP allocates) with CPR_ERR_INVALID_ARG, before
  // any state changes.
  cpr_status solve(const double* b, double* x, double tol, cpr_solve_info* info, const cpr::KrylovWork& w,
                   bool may_allocate);
  void spmv(const double* x, double* y);
};
