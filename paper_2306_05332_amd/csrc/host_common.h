// Host-side error handling shared by the library's source files: every C-ABI
// entry point runs its body under guarded(), which turns a Fail thrown by
// fail() (or a HIP error caught by HIPCHK / check_launch) into the returned
// rkl_status and leaves the message for rkl_last_error().
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <new>
#include <string>

#include "../../include/rkl_poisson.h"

namespace rkl {

extern thread_local std::string g_err;  // message of the calling thread's last failure

struct Fail {
  rkl_status st;
};

[[noreturn]] void fail(rkl_status st, const std::string& msg);

#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) fail(RKL_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) fail(RKL_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

template <typename Fn>
rkl_status guarded(Fn&& fn) {
  try {
    return fn();
  } catch (const Fail& f) {
    return f.st;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return RKL_ENOMEM;
  } catch (...) {
    g_err = "unexpected internal error";
    return RKL_EHIP;
  }
}

// Workgroups of `kernel` (blocks of `threads`) the current device holds at
// once, from the kernel's occupancy and the compute-unit count; cached per
// device in `cache` (one per kernel instantiation).
template <typename K>
int resident_wgs(K kernel, int threads, std::atomic<int> (&cache)[64]) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) fail(RKL_EINVAL, "device index out of range");
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v > 0) return v;
  int cus = 0, per_cu = 0;
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0));
  v = std::max(1, cus * per_cu);
  cache[dev].store(v, std::memory_order_relaxed);
  return v;
}

// a two-dimensional grid: nz = 1 with hz = +inf
bool flat_grid(const rkl_grid& g);
// RKL_EINVAL (via fail) for malformed geometry or face data on a periodic grid
void validate_grid(const rkl_grid* g, const double* bc_faces);

}  // namespace rkl
