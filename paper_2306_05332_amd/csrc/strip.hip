// Fused s-stage RKL tau-step kernels in strip form (the body and its design
// notes are in strip_body.h): kernel wrappers, grid geometry, launchers and
// the explicit instantiations.
#include "strip_body.h"

namespace rkl {

template <typename T, int S, int R, int WY, bool PER, bool UZ, bool GS, bool FLAT, bool NT>
__global__ __launch_bounds__(64 * WY) void k_tau_strip(LevelView<T> L, const T* __restrict__ u,
                                                       const T* __restrict__ b, T* __restrict__ out,
                                                       FCoef<T, S> co, int zc, int gx_tiles, int gy_tiles,
                                                       int nblk, StripMap sm, double* __restrict__ part, Batch bt,
                                                       const int* __restrict__ stop) {
  tau_strip_body<T, S, R, WY, PER, UZ, GS, FLAT, false, NT>(L, u, b, out, co, zc, gx_tiles, gy_tiles, nblk, sm,
                                                             part, bt, stop);
}

// the same with the y halo rows shared between the stacked wavefronts
template <typename T, int S, int R, int WY, bool PER, bool UZ, bool GS, bool NT>
__global__ __launch_bounds__(64 * WY) void k_tau_strip_yx(LevelView<T> L, const T* __restrict__ u,
                                                          const T* __restrict__ b, T* __restrict__ out,
                                                          FCoef<T, S> co, int zc, int gx_tiles, int gy_tiles,
                                                          int nblk, StripMap sm, double* __restrict__ part, Batch bt,
                                                          const int* __restrict__ stop) {
  tau_strip_body<T, S, R, WY, PER, UZ, GS, false, true, NT>(L, u, b, out, co, zc, gx_tiles, gy_tiles, nblk, sm,
                                                             part, bt, stop);
}

// flat: (nx, ny, nz) is the transposed view of a 2-D level (ny = 1, nz = the
// 2-D row count); a workgroup then spans WY * R segments of ox columns in x
StripGrid strip_grid(int s, int R, int WY, int nx, int ny, int nz, int target, bool flat, bool pack) {
  StripGrid g;
  g.ox = 64 - 2 * s;
  g.map = StripMap{0, 0, 0, 0, 0};
  if (flat) {
    g.gx = (nx + g.ox * R * WY - 1) / (g.ox * R * WY);
    g.gy = 1;
  } else {
    g.gx = (nx + g.ox - 1) / g.ox;
    g.gy = (ny + R * WY - 1) / (R * WY);
  }
  int per = g.gx * g.gy;  // workgroups per z chunk
  if (!flat && WY == 1 && pack) {
    const int txf = nx / g.ox, rem = nx - txf * g.ox;
    const int pk = rem > 0 ? 64 / (rem + 2 * s) : 0;
    // interior strips: rows ty R - s .. ty R + R + s - 1 all inside 0 .. ny - 1
    const int fi = (s + R - 1) / R;
    const int li = ny - R - s >= 0 ? (ny - R - s) / R : -1;
    const int npk = (pk >= 2 && li >= fi) ? (li - fi + 1) / pk : 0;
    if (npk > 0) {
      g.map = StripMap{txf, pk, npk, fi, txf * g.gy + npk + (g.gy - npk * pk)};
      per = g.map.per;
    }
  }
  const int chunks = std::max(1, (target + per - 1) / per);
  // chunks down to one plane: on small (cache-resident, latency-bound) levels
  // a shorter serial march beats the re-read of the chunk's boundary planes
  g.zc = std::max(1, std::min(64, (nz + chunks - 1) / chunks));
  g.gz = (nz + g.zc - 1) / g.zc;
  g.per = per;
  g.nblk = per * g.gz;
  return g;
}

// The view the FLAT kernel marches: the 2-D level (nz = 1, ihz2 = 0) with y
// moved to the marching axis; the memory layout is unchanged.
template <typename T>
static LevelView<T> flat_view(const LevelView<T>& L) {
  LevelView<T> V = L;
  V.ny = 1;
  V.nz = L.ny;
  V.ihy2 = (T)0;
  V.ihz2 = L.ihy2;
  return V;
}

template <typename T, int S, int R, int WY, bool GS, bool FLAT, bool NT>
static void launch_strip_nt(const LevelView<T>& L, const StripGrid& g, const T* u, const T* b, T* out,
                            const FCoef<T, S>& fc, double* part, const int* stop, const Batch& bt, hipStream_t st) {
  const dim3 grid(g.nblk, bt.nb), block(64 * WY);
  if (L.periodic) {
    if (u == nullptr)
      hipLaunchKernelGGL((k_tau_strip<T, S, R, WY, true, true, GS, FLAT, NT>), grid, block, 0, st, L, u, b, out, fc,
                         g.zc, g.gx, g.gy, g.nblk, g.map, part, bt, stop);
    else
      hipLaunchKernelGGL((k_tau_strip<T, S, R, WY, true, false, GS, FLAT, NT>), grid, block, 0, st, L, u, b, out, fc,
                         g.zc, g.gx, g.gy, g.nblk, g.map, part, bt, stop);
  } else {
    if (u == nullptr)
      hipLaunchKernelGGL((k_tau_strip<T, S, R, WY, false, true, GS, FLAT, NT>), grid, block, 0, st, L, u, b, out, fc,
                         g.zc, g.gx, g.gy, g.nblk, g.map, part, bt, stop);
    else
      hipLaunchKernelGGL((k_tau_strip<T, S, R, WY, false, false, GS, FLAT, NT>), grid, block, 0, st, L, u, b, out,
                         fc, g.zc, g.gx, g.gy, g.nblk, g.map, part, bt, stop);
  }
}

template <typename T, int S, int R, int WY, bool GS, bool FLAT>
static void launch_strip_k(const LevelView<T>& L0, int target, const T* u, const T* b, T* out, const FCoef<T, S>& fc,
                           double* part, const int* stop, const Batch& bt, hipStream_t st) {
  const LevelView<T> L = FLAT ? flat_view(L0) : L0;
  const StripGrid g = strip_grid(S, R, WY, L.nx, L.ny, L.nz, target, FLAT);
  if constexpr (sizeof(T) == 8) {
    if (strip_nt<T>(L, bt)) return launch_strip_nt<T, S, R, WY, GS, FLAT, true>(L, g, u, b, out, fc, part, stop, bt, st);
  }
  launch_strip_nt<T, S, R, WY, GS, FLAT, false>(L, g, u, b, out, fc, part, stop, bt, st);
}

template <typename T, int S, int R, int WY>
void launch_strip(const LevelView<T>& L, int target, const T* u, const T* b, T* out, const FCoef<T, S>& fc,
                  double* part, const int* stop, const Batch& bt, hipStream_t st) {
  launch_strip_k<T, S, R, WY, false, false>(L, target, u, b, out, fc, part, stop, bt, st);
}

// stacked wavefronts with shared y halo rows (3-D levels, WY > 1)
template <typename T, int S, int R, int WY, bool NT>
static void launch_strip_yx_nt(const LevelView<T>& L, const StripGrid& g, const T* u, const T* b, T* out,
                               const FCoef<T, S>& fc, double* part, const int* stop, const Batch& bt, hipStream_t st) {
  const dim3 grid(g.nblk, bt.nb), block(64 * WY);
  if (L.periodic) {
    if (u == nullptr)
      hipLaunchKernelGGL((k_tau_strip_yx<T, S, R, WY, true, true, false, NT>), grid, block, 0, st, L, u, b, out, fc,
                         g.zc, g.gx, g.gy, g.nblk, g.map, part, bt, stop);
    else
      hipLaunchKernelGGL((k_tau_strip_yx<T, S, R, WY, true, false, false, NT>), grid, block, 0, st, L, u, b, out, fc,
                         g.zc, g.gx, g.gy, g.nblk, g.map, part, bt, stop);
  } else {
    if (u == nullptr)
      hipLaunchKernelGGL((k_tau_strip_yx<T, S, R, WY, false, true, false, NT>), grid, block, 0, st, L, u, b, out, fc,
                         g.zc, g.gx, g.gy, g.nblk, g.map, part, bt, stop);
    else
      hipLaunchKernelGGL((k_tau_strip_yx<T, S, R, WY, false, false, false, NT>), grid, block, 0, st, L, u, b, out,
                         fc, g.zc, g.gx, g.gy, g.nblk, g.map, part, bt, stop);
  }
}

template <typename T, int S, int R, int WY>
void launch_strip_yx(const LevelView<T>& L, int target, const T* u, const T* b, T* out, const FCoef<T, S>& fc,
                     double* part, const int* stop, const Batch& bt, hipStream_t st) {
  const StripGrid g = strip_grid(S, R, WY, L.nx, L.ny, L.nz, target, false);
  if constexpr (sizeof(T) == 8) {
    if (strip_nt<T>(L, bt)) return launch_strip_yx_nt<T, S, R, WY, true>(L, g, u, b, out, fc, part, stop, bt, st);
  }
  launch_strip_yx_nt<T, S, R, WY, false>(L, g, u, b, out, fc, part, stop, bt, st);
}

template <typename T, int S, int R, int WY>
void launch_strip2d(const LevelView<T>& L, int target, const T* u, const T* b, T* out, const FCoef<T, S>& fc,
                    double* part, const int* stop, const Batch& bt, hipStream_t st) {
  launch_strip_k<T, S, R, WY, false, true>(L, target, u, b, out, fc, part, stop, bt, st);
}

// one red-black GS / SOR iteration in one pass: the two-stage strip kernel
// with mu = 1, nu = 0, c = omega / D on the cells of each stage's colour
template <typename T, int R, int WY, bool FLAT>
void launch_strip_gsrb(const LevelView<T>& L, int target, const T* u, const T* b, T* out, double omega_over_d,
                       double* part, const int* stop, const Batch& bt, hipStream_t st) {
  FCoef<T, 2> fc;
  for (int j = 0; j < 2; ++j) {
    fc.mu[j] = (T)1;
    fc.nu[j] = (T)0;
    fc.c[j] = (T)omega_over_d;
  }
  launch_strip_k<T, 2, R, WY, true, FLAT>(L, target, u, b, out, fc, part, stop, bt, st);
}

#define RKL_STRIP_INST(T, S, R, WY)                                                                          \
  template void launch_strip<T, S, R, WY>(const LevelView<T>&, int, const T*, const T*, T*, const FCoef<T, S>&, \
                                          double*, const int*, const Batch&, hipStream_t);
RKL_STRIP_INST(double, 1, 8, 4)
RKL_STRIP_INST(double, 2, 8, 4)
RKL_STRIP_INST(double, 1, 8, 1)
RKL_STRIP_INST(double, 2, 8, 1)
RKL_STRIP_INST(float, 1, 8, 4)
RKL_STRIP_INST(float, 2, 8, 4)
RKL_STRIP_INST(float, 3, 8, 4)
RKL_STRIP_INST(float, 1, 8, 1)
RKL_STRIP_INST(float, 2, 8, 1)
RKL_STRIP_INST(float, 3, 8, 1)
RKL_STRIP_INST(double, 1, 4, 4)
RKL_STRIP_INST(double, 2, 4, 4)
RKL_STRIP_INST(float, 1, 4, 4)
RKL_STRIP_INST(float, 2, 4, 4)
RKL_STRIP_INST(float, 3, 4, 4)
RKL_STRIP_INST(double, 1, 5, 1)
RKL_STRIP_INST(double, 2, 5, 1)
RKL_STRIP_INST(float, 1, 5, 1)
RKL_STRIP_INST(float, 2, 5, 1)
RKL_STRIP_INST(float, 3, 5, 1)
#undef RKL_STRIP_INST
#define RKL_STRIPYX_INST(T, S, R, WY)                                                                        \
  template void launch_strip_yx<T, S, R, WY>(const LevelView<T>&, int, const T*, const T*, T*,               \
                                             const FCoef<T, S>&, double*, const int*, const Batch&, hipStream_t);
RKL_STRIPYX_INST(double, 1, 8, 4)
RKL_STRIPYX_INST(double, 2, 8, 4)
RKL_STRIPYX_INST(double, 1, 4, 8)
RKL_STRIPYX_INST(double, 2, 4, 8)
RKL_STRIPYX_INST(double, 3, 4, 8)
RKL_STRIPYX_INST(float, 1, 8, 4)
RKL_STRIPYX_INST(float, 2, 8, 4)
RKL_STRIPYX_INST(float, 3, 8, 4)
RKL_STRIPYX_INST(float, 1, 4, 8)
RKL_STRIPYX_INST(float, 2, 4, 8)
RKL_STRIPYX_INST(float, 3, 4, 8)
RKL_STRIPYX_INST(double, 1, 8, 8)
RKL_STRIPYX_INST(double, 2, 8, 8)
RKL_STRIPYX_INST(float, 1, 8, 8)
RKL_STRIPYX_INST(float, 2, 8, 8)
RKL_STRIPYX_INST(float, 3, 8, 8)
RKL_STRIPYX_INST(double, 1, 2, 8)
RKL_STRIPYX_INST(double, 2, 2, 8)
RKL_STRIPYX_INST(float, 1, 2, 8)
RKL_STRIPYX_INST(float, 2, 2, 8)
RKL_STRIPYX_INST(double, 1, 2, 16)
RKL_STRIPYX_INST(double, 2, 2, 16)
RKL_STRIPYX_INST(float, 1, 2, 16)
RKL_STRIPYX_INST(float, 2, 2, 16)
#undef RKL_STRIPYX_INST
#define RKL_STRIP2D_INST(T, S, R, WY)                                                                          \
  template void launch_strip2d<T, S, R, WY>(const LevelView<T>&, int, const T*, const T*, T*, const FCoef<T, S>&, \
                                            double*, const int*, const Batch&, hipStream_t);
RKL_STRIP2D_INST(double, 1, 8, 1)
RKL_STRIP2D_INST(double, 2, 8, 1)
RKL_STRIP2D_INST(double, 1, 4, 1)
RKL_STRIP2D_INST(double, 2, 4, 1)
RKL_STRIP2D_INST(float, 1, 8, 1)
RKL_STRIP2D_INST(float, 2, 8, 1)
RKL_STRIP2D_INST(float, 3, 8, 1)
RKL_STRIP2D_INST(float, 1, 4, 1)
RKL_STRIP2D_INST(float, 2, 4, 1)
RKL_STRIP2D_INST(float, 3, 4, 1)
RKL_STRIP2D_INST(double, 3, 4, 1)
RKL_STRIP2D_INST(double, 4, 4, 1)
RKL_STRIP2D_INST(float, 4, 8, 1)
RKL_STRIP2D_INST(float, 4, 4, 1)
#undef RKL_STRIP2D_INST
#define RKL_GSRB_INST(T, R, WY, FLAT)                                                                          \
  template void launch_strip_gsrb<T, R, WY, FLAT>(const LevelView<T>&, int, const T*, const T*, T*, double,     \
                                                  double*, const int*, const Batch&, hipStream_t);
RKL_GSRB_INST(double, 8, 4, false)
RKL_GSRB_INST(double, 4, 4, false)
RKL_GSRB_INST(float, 8, 4, false)
RKL_GSRB_INST(float, 4, 4, false)
RKL_GSRB_INST(double, 5, 1, false)
RKL_GSRB_INST(float, 5, 1, false)
RKL_GSRB_INST(double, 8, 1, true)
RKL_GSRB_INST(double, 4, 1, true)
RKL_GSRB_INST(float, 8, 1, true)
RKL_GSRB_INST(float, 4, 1, true)
#undef RKL_GSRB_INST

}  // namespace rkl
