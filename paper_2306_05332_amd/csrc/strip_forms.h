// Two further forms of the strip tau-step, whose body is the plain strip
// kernel's (strip_body.h); their instantiations are split over two
// translation units by precision.
//
// Prolongation fusion (PRO): the first post-smoothing relaxation of a level
// reads u, e (the next coarser level's correction) and b, and writes only
// its result, so the corrected u + P e (Sec. 2.1 steps 4-5, eq.
// prolongation_example_3D) is never stored.
//
// Stage chunks (CH): S consecutive stages j0 .. j0 + S - 1 of a longer
// tau-step (App. A eq. RKL_intermediate_source with the s-stage
// coefficients) in one pass.  The chunk reads Y_{j0-1} (u, with its stencil
// halo), Y_{j0-2} (v, pointwise, for the first stage's nu term) and b, and
// writes Y_{j0+S-1} (out) and Y_{j0+S-2} (out2), the two inputs of the next
// chunk: 5 words per S stages instead of 4 per stage.  The first chunk of a
// tau-step passes v = u with nu_1 = 0, mu_1 = 1.
#pragma once

#include "host_common.h"
#include "strip_body.h"

namespace rkl {

template <typename T, int S, int R, int WY, bool PER, bool SHY, bool NT>
__global__ __launch_bounds__(64 * WY, (strip_min_waves<T, R, WY>())) void k_tau_strip_pro(LevelView<T> L, const T* __restrict__ u,
                                                           const T* __restrict__ e, const T* __restrict__ b,
                                                           T* __restrict__ out, FCoef<T, S> co, int zc, int gx_tiles,
                                                           int gy_tiles, int nblk, Batch bt,
                                                           const int* __restrict__ stop) {
  tau_strip_body<T, S, R, WY, PER, false, false, false, SHY, NT, true>(
      L, u, b, out, co, zc, gx_tiles, gy_tiles, nblk, StripMap{0, 0, 0, 0, 0}, nullptr, bt, stop, e);
}

// target <= 0: as many z chunks as fill one wave of resident workgroups
// (from the kernel's occupancy; the grid depends on the level only)
template <typename T, int S, int R, int WY, bool PER, bool SHY, bool NT>
static void launch_strip_pro_k(const LevelView<T>& L, int target, const T* u, const T* e, const T* b, T* out,
                               const FCoef<T, S>& fc, const int* stop, const Batch& bt, hipStream_t st) {
  auto kern = k_tau_strip_pro<T, S, R, WY, PER, SHY, NT>;
  if (target <= 0) {
    static std::atomic<int> slots[64];
    const int per = strip_grid(S, R, WY, L.nx, L.ny, L.nz, 1, false, false).per;
    target = std::max(1, resident_wgs(kern, 64 * WY, slots) / per) * per;
  }
  const StripGrid g = strip_grid(S, R, WY, L.nx, L.ny, L.nz, target, false, false);
  hipLaunchKernelGGL(kern, dim3(g.nblk, bt.nb), dim3(64 * WY), 0, st, L, u, e, b, out, fc, g.zc, g.gx, g.gy, g.nblk,
                     bt, stop);
}

template <typename T, int S, int R, int WY, bool SHY>
void launch_strip_pro(const LevelView<T>& L, int target, const T* u, const T* e, const T* b, T* out,
                      const FCoef<T, S>& fc, const int* stop, const Batch& bt, hipStream_t st) {
  if ((L.nx | L.ny | L.nz) & 1) fail(RKL_EINVAL, "prolongation fusion needs even level extents");
  const bool nt = sizeof(T) == 8 && strip_nt<T>(L, bt);
  if (L.periodic) {
    if (nt) return launch_strip_pro_k<T, S, R, WY, true, SHY, true>(L, target, u, e, b, out, fc, stop, bt, st);
    return launch_strip_pro_k<T, S, R, WY, true, SHY, false>(L, target, u, e, b, out, fc, stop, bt, st);
  }
  if (nt) return launch_strip_pro_k<T, S, R, WY, false, SHY, true>(L, target, u, e, b, out, fc, stop, bt, st);
  launch_strip_pro_k<T, S, R, WY, false, SHY, false>(L, target, u, e, b, out, fc, stop, bt, st);
}

template <typename T, int S, int R, int WY, bool PER, bool NT>
__global__ __launch_bounds__(64 * WY) void k_tau_strip_ch(LevelView<T> L, const T* __restrict__ u,
                                                          const T* __restrict__ v, const T* __restrict__ b,
                                                          T* __restrict__ out, T* __restrict__ out2, FCoef<T, S> co,
                                                          int zc, int gx_tiles, int gy_tiles, int nblk, Batch bt) {
  tau_strip_body<T, S, R, WY, PER, false, false, false, false, NT, false, true>(
      L, u, b, out, co, zc, gx_tiles, gy_tiles, nblk, StripMap{0, 0, 0, 0, 0}, nullptr, bt, nullptr, nullptr, v, out2);
}

template <typename T, int S, int R, int WY>
void launch_strip_ch(const LevelView<T>& L, int target, const T* u, const T* v, const T* b, T* out, T* out2,
                     const FCoef<T, S>& fc, const Batch& bt, hipStream_t st) {
  const StripGrid g = strip_grid(S, R, WY, L.nx, L.ny, L.nz, target, false, false);
  const dim3 grid(g.nblk, bt.nb), block(64 * WY);
  const bool nt = sizeof(T) == 8 && 4 * (size_t)L.nx * L.ny * L.nz * sizeof(T) * (size_t)bt.nb > STRIP_NT_MIN_BYTES;
#define RKL_CH_LAUNCH(PER, NT)                                                                                    \
  hipLaunchKernelGGL((k_tau_strip_ch<T, S, R, WY, PER, NT>), grid, block, 0, st, L, u, v, b, out, out2, fc, g.zc, \
                     g.gx, g.gy, g.nblk, bt)
  if (L.periodic) {
    if (nt) RKL_CH_LAUNCH(true, true);
    else RKL_CH_LAUNCH(true, false);
  } else {
    if (nt) RKL_CH_LAUNCH(false, true);
    else RKL_CH_LAUNCH(false, false);
  }
#undef RKL_CH_LAUNCH
}

}  // namespace rkl

#define RKL_STRIP_CH_INST(T, S, R, WY)                                                                          \
  template void rkl::launch_strip_ch<T, S, R, WY>(const rkl::LevelView<T>&, int, const T*, const T*, const T*, T*, \
                                                  T*, const rkl::FCoef<T, S>&, const rkl::Batch&, hipStream_t);

#define RKL_STRIP_PRO_INST(T, S, R, WY, SHY)                                                                   \
  template void rkl::launch_strip_pro<T, S, R, WY, SHY>(const rkl::LevelView<T>&, int, const T*, const T*,     \
                                                        const T*, T*, const rkl::FCoef<T, S>&, const int*,     \
                                                        const rkl::Batch&, hipStream_t);
