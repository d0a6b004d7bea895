// Host-side launchers of the gfx950 kernels (see kernels.hip, coarse.hip, fused.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "rkl_device.h"

namespace rkl {

size_t stencil_blocks(int nx, int ny, int nz);  // partial-sum slots used by residual-type kernels
size_t ew_block_count(size_t n);                // partial-sum slots used by k_scale

template <typename T>
void launch_stage(const LevelView<T>& L, const T* yp, const T* ypp, const T* b, T* yout, double mu,
                  double nu, double c, int first, hipStream_t st);
template <typename TU, typename TR>
void launch_residual(const LevelView<TU>& L, const TU* u, const TU* b, TR* r_out, double* part,
                     hipStream_t st);
template <typename T>
void launch_resid_restrict(const LevelView<T>& F, const T* u, const T* b, T* bc, double* part,
                           hipStream_t st);
template <typename T>
void launch_prolong_add(int fnx, int fny, int fnz, int periodic, const T* e, T* fine, hipStream_t st);
template <typename T>
void launch_restrict(int fnx, int fny, int fnz, const T* fine, T* coarse, hipStream_t st);
void launch_reduce(const double* part, int nblk, int stride, int nq, double* out, hipStream_t st);
template <typename T>
void launch_fill(T* a, size_t n, T v, hipStream_t st);
void launch_scale(const double* in, double* out, size_t n, double c, double* part, hipStream_t st);
template <typename T>
void launch_sub_mean(T* a, size_t n, const double* sum, double count, hipStream_t st);
template <typename T>
void launch_sum(const T* a, size_t n, double* part, hipStream_t st);  // ew_block_count(n) partials
template <typename TE>
void launch_add_cast(double* u, const TE* e, size_t n, hipStream_t st);

// Coarsest-grid accelerated RKL solve in one workgroup (coarse.hip).
constexpr int COARSE_MAX_CELLS = 2048;
struct CoarseSchedule {
  const int* sched;     // device: stage count of schedule entry q
  const int* coff;      // device: first coefficient row of entry q
  const double* coef;   // device: rows (mu, nu, c) per stage
  int nsched;
};
template <typename T>
void launch_coarse_solve(const LevelView<T>& L, const T* b, const T* u_in, T* u, CoarseSchedule cs,
                         double tol, double ref_norm, int max_steps, int remove_mean, int* steps_out,
                         double* res_out, hipStream_t st);

// Fused s-stage tau-step, one HBM pass (fused.hip).  Returns false when the
// configuration is not supported (caller falls back to per-stage kernels).
struct StageCoef {
  double mu, nu, c;
};
constexpr int FUSED_MAX_S = 4;
template <typename T>
bool launch_fused_tau(const LevelView<T>& L, const T* u, const T* b, T* out, int s,
                      const StageCoef* co, double* part, hipStream_t st);

}  // namespace rkl
