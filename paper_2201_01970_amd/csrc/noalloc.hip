// The Krylov workspace layout and the static scratch array of the
// allocation-free solve (cpr_solve_noalloc).
//
// cpr_solve keeps the FGMRES scalars and partial sums (KrylovWork) in memory
// the handle allocated at SETUP and replays each step as a captured graph;
// cpr_solve_noalloc runs the same kernels eagerly with that workspace carved
// out of `scratch`, a file-scope device array that every GPU the library runs
// on holds until the process ends.  Its device address on each GPU is looked
// up once, with that GPU current, and kept per device: in host code the
// array's name is only a host-side stand-in and never reaches a kernel.
#include <mutex>

#include "kernels_common.hpp"
#include "solver.hpp"

namespace cpr {

KrylovWork krylov_work_carve(double* base, int m) {
  const int64_t m1 = m + 1;
  KrylovWork w;
  double* p = base;
  auto take = [&p](int64_t n) {
    double* q = p;
    p += krylov_round_up(n);
    return q;
  };
  w.H = take(m1 * m);
  w.cs = take(m);
  w.sn = take(m);
  w.g = take(m1);
  w.y = take(m);
  w.hnorm = take(1);
  w.partial = take(m1 * kKrylovGridMax);
  w.norm_partial = take(kKrylovGridMax);
  w.report = take(4);
  return w;
}

namespace {

// Room for the workspace of the largest accepted restart: 139,680 doubles
// (1.07 MiB) per GPU.
constexpr int64_t kScratchDoubles = krylov_work_doubles(kNoAllocMaxRestart);
static_assert(kScratchDoubles * 8 <= (2 << 20), "the static scratch stays below 2 MiB");

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

double* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) throw Error(CPR_ERR_INVALID_ARG, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  if (g_scratch_ptr[device]) return g_scratch_ptr[device];
  int current = 0;
  HIPCHK(hipGetDevice(&current));
  if (current != device) HIPCHK(hipSetDevice(device));
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (current != device) HIPCHK(hipSetDevice(current));
  HIPCHK(e);
  if (!ptr) throw Error(CPR_ERR_HIP, "hipGetSymbolAddress returned a null scratch address");
  g_scratch_ptr[device] = static_cast<double*>(ptr);
  return g_scratch_ptr[device];
}

}  // namespace cpr
