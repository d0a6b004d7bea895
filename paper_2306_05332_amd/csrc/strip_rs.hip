// Restriction fusion of the strip tau-step (strip_body.h, RS = true): the
// last pre-smoothing relaxation of a level (App. A eq.
// RKL_intermediate_source) also writes the next level's right-hand side
// R(b - M Y_S), the 8-child average of eq. restriction_example_3D applied
// to the residual (Sec. 2.1 steps 2a-2b), with the float64 partials of the
// separate residual + restriction pass: per workgroup (sum of fine r^2, sum
// of the coarse values).  Y_S is never read back: 3 words per fine cell
// plus the coarse write, against 3 + 2 for the tau-step and the separate
// pass.
//
// Tiles: 64 - 2(S + 1) output columns per wavefront (one halo lane more on
// either side than the plain strip), R WY - 2 output rows per workgroup (its
// first and last computed rows are the residual's halo), chunks of an even
// number of planes (a coarse plane's two fine planes in one chunk).  Built
// for S >= 2: a wavefront's last row pair takes b of the row above its own
// rows, which only tau-steps of two or more stages hold.
#include "host_common.h"
#include "strip_body.h"

namespace rkl {

template <typename T, int S, int R, int WY, bool PER, bool SHY, bool NT>
__global__ __launch_bounds__(64 * WY, (strip_min_waves<T, R, WY>())) void k_tau_strip_rs(LevelView<T> L, const T* __restrict__ u,
                                                          const T* __restrict__ b, T* __restrict__ out,
                                                          T* __restrict__ bc, FCoef<T, S> co, int zc, int gx_tiles,
                                                          int gy_tiles, int nblk, double* __restrict__ part, Batch bt,
                                                          const int* __restrict__ stop) {
  tau_strip_body<T, S, R, WY, PER, false, false, false, SHY, NT, false, false, true>(
      L, u, b, out, co, zc, gx_tiles, gy_tiles, nblk, StripMap{0, 0, 0, 0, 0}, part, bt, stop, nullptr, nullptr,
      nullptr, bc);
}

// target: workgroups the device holds at once; the z chunks are as many as
// fit in one such wave of workgroups, since a partial second wave would cost
// nearly a whole pass
StripGrid strip_grid_rs(int s, int R, int WY, int nx, int ny, int nz, int target) {
  StripGrid g;
  g.ox = 64 - 2 * (s + 1);
  g.map = StripMap{0, 0, 0, 0, 0};
  g.gx = (nx + g.ox - 1) / g.ox;
  g.gy = (ny + R * WY - 3) / (R * WY - 2);
  g.per = g.gx * g.gy;
  const int chunks = std::max(1, target / g.per);
  int zc = std::max(2, std::min(64, (nz + chunks - 1) / chunks));
  zc += zc & 1;
  g.zc = zc;
  g.gz = (nz + zc - 1) / zc;
  g.nblk = g.per * g.gz;
  return g;
}

size_t strip_rs_parts_max(int nx, int ny, int nz) {
  // smallest tile built: 54 output columns (s <= 4), RS_MIN_ROWS rows, 2 planes
  return 2 * (size_t)((nx + 53) / 54) * (size_t)((ny + RS_MIN_ROWS - 1) / RS_MIN_ROWS) * (size_t)((nz + 1) / 2);
}

template <typename T, int S, int R, int WY, bool PER, bool SHY, bool NT>
static int launch_rs_k(const LevelView<T>& L, const T* u, const T* b, T* out, T* bc, const FCoef<T, S>& fc,
                       double* part, const int* stop, const Batch& bt, hipStream_t st) {
  static std::atomic<int> slots[64];
  auto kern = k_tau_strip_rs<T, S, R, WY, PER, SHY, NT>;
  // the grid depends on the level only, not on the batch size, so that a
  // batch member's partial sums (and its answer) are the single solve's
  const StripGrid g = strip_grid_rs(S, R, WY, L.nx, L.ny, L.nz, resident_wgs(kern, 64 * WY, slots));
  hipLaunchKernelGGL(kern, dim3(g.nblk, bt.nb), dim3(64 * WY), 0, st, L, u, b, out, bc, fc, g.zc, g.gx, g.gy, g.nblk,
                     part, bt, stop);
  return g.nblk;
}

template <typename T, int S, int R, int WY, bool SHY>
int launch_strip_rs(const LevelView<T>& L, int target, const T* u, const T* b, T* out, T* bc, const FCoef<T, S>& fc,
                    double* part, const int* stop, const Batch& bt, hipStream_t st) {
  static_assert(R * WY - 2 >= RS_MIN_ROWS, "restriction fusion: workgroups of at least RS_MIN_ROWS output rows");
  (void)target;
  if ((L.nx | L.ny | L.nz) & 1) fail(RKL_EINVAL, "restriction fusion needs even level extents");
  const bool nt = sizeof(T) == 8 && strip_nt<T>(L, bt);
  if (L.periodic) {
    if (nt) return launch_rs_k<T, S, R, WY, true, SHY, true>(L, u, b, out, bc, fc, part, stop, bt, st);
    return launch_rs_k<T, S, R, WY, true, SHY, false>(L, u, b, out, bc, fc, part, stop, bt, st);
  }
  if (nt) return launch_rs_k<T, S, R, WY, false, SHY, true>(L, u, b, out, bc, fc, part, stop, bt, st);
  return launch_rs_k<T, S, R, WY, false, SHY, false>(L, u, b, out, bc, fc, part, stop, bt, st);
}

#define RKL_STRIP_RS_INST(T, S, R, WY, SHY)                                                                        \
  template int launch_strip_rs<T, S, R, WY, SHY>(const LevelView<T>&, int, const T*, const T*, T*, T*,             \
                                                 const FCoef<T, S>&, double*, const int*, const Batch&, hipStream_t);
RKL_STRIP_RS_INST(double, 2, 2, 8, true)
RKL_STRIP_RS_INST(float, 2, 4, 4, false)
RKL_STRIP_RS_INST(float, 3, 4, 4, false)
RKL_STRIP_RS_INST(float, 2, 2, 8, true)
RKL_STRIP_RS_INST(float, 2, 8, 4, true)
#undef RKL_STRIP_RS_INST

}  // namespace rkl
