// rkl_residual_noalloc: the finest-level residual r = f - M phi and its norm
// (Sec. 2.1 eq. residual, with the opposite sign; Sec. 4.1 stop metric) for
// callers that cannot allocate device memory -- code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc.
//
// It runs the kernels of rkl_residual (the LDS-tiled residual kernel with its
// float64 partial sums per workgroup, then the fixed-order reduction), but the
// partial sums live in `scratch`, a fixed array in this file, instead of a
// plan buffer, and Dirichlet face data is applied inside the stencil (ghost
// 2 g - u, eq. solution_ghost) instead of being folded into a copy of f.  No
// call here allocates, frees or synchronises.
//
// `scratch` exists once per GPU, for the life of the process.  Its device
// address is looked up once per device (hipGetSymbolAddress with that device
// current) and only that address is handed to kernels: in host code the
// array's name is a host-side stand-in, not a device pointer.  Every call on a
// GPU writes the same array, so calls that overlap in time on one GPU race;
// each call overwrites every slot it reads (each workgroup writes its own
// partial pair, the reduction writes the sum), so nothing needs clearing.
#include <cmath>
#include <mutex>
#include <string>

#include "host_common.h"
#include "kernels.h"

namespace rkl {

// Partial-sum pairs the residual kernels of one call may write.  A 3-D
// residual workgroup covers a 64 x 16 tile over up to 16 planes, so 65536
// pairs cover grids up to 1024^3 cells; 2-D grids take one pair per
// workgroup of their row-pair chunks.
constexpr size_t NOALLOC_MAX_PAIRS = 65536;
constexpr size_t NOALLOC_SUM = 2 * NOALLOC_MAX_PAIRS;  // slot of the reduced sum of r^2
constexpr size_t NOALLOC_DOUBLES = NOALLOC_SUM + 32;   // 1 MiB + 256 B

static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch` (looked up on the
// first call on that device, with it current).
double* scratch_ptr() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    fail(RKL_EINVAL, "device index " + std::to_string(dev) + " is beyond the no-allocation table (64 devices)");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[dev] == nullptr) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) fail(RKL_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_noalloc_ptr[dev] = (double*)p;
  }
  return g_noalloc_ptr[dev];
}

// out[0] = sqrt(sum[0]) (correctly rounded, as the host's std::sqrt)
__global__ __launch_bounds__(64) void k_sqrt_to(const double* __restrict__ sum, double* __restrict__ out) {
  if (threadIdx.x == 0) out[0] = sqrt(sum[0]);
}

}  // namespace
}  // namespace rkl

using namespace rkl;

extern "C" rkl_status rkl_residual_noalloc(const rkl_grid* grid, const double* f, const double* bc_faces,
                                           const double* phi, double* r_out, double* norm_dev,
                                           void* hip_stream) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, bc_faces);
    if (!f || !phi) fail(RKL_EINVAL, "f and phi must be non-NULL");
    const size_t pairs = resid_blocks(grid->nx, grid->ny, grid->nz);
    if (pairs > NOALLOC_MAX_PAIRS)
      fail(RKL_EINVAL, "grid needs " + std::to_string(pairs) + " partial-sum pairs; the no-allocation residual "
                       "holds at most " + std::to_string(NOALLOC_MAX_PAIRS) + " (about 1024^3 cells in 3-D)");
    double* const ptr = scratch_ptr();
    hipStream_t st = (hipStream_t)hip_stream;
    LevelView<double> V;
    V.nx = grid->nx;
    V.ny = grid->ny;
    V.nz = grid->nz;
    V.ihx2 = 1.0 / (grid->hx * grid->hx);
    V.ihy2 = 1.0 / (grid->hy * grid->hy);
    V.ihz2 = 1.0 / (grid->hz * grid->hz);  // 0 for a two-dimensional grid (hz = inf)
    V.periodic = grid->bc == RKL_BC_PERIODIC ? 1 : 0;
    V.faces = bc_faces;
    launch_residual<double, double>(V, phi, f, r_out, ptr, nullptr, st);
    check_launch();
    if (norm_dev != nullptr) {
      launch_reduce(ptr, (int)pairs, 2, 1, ptr + NOALLOC_SUM, nullptr, st);
      hipLaunchKernelGGL(k_sqrt_to, dim3(1), dim3(64), 0, st, ptr + NOALLOC_SUM, norm_dev);
      check_launch();
    }
    return RKL_OK;
  });
}
