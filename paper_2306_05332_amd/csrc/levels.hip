// Level building blocks behind the C ABI (mg_vcycle, rkl_smooth,
// rkl_residual, rkl_restrict, rkl_prolong_add, rkl_coarse_solve and their
// float32 twins), the GS-RB passes, the App. B single-level relaxation
// and the Sec. 3 gradient.

#include "solver_core.h"

namespace rkl {

// ------------------------------------------------------------------ level building blocks
// Precision-generic bodies of the single-level entry points.  The float32
// forms are the kernels of the mixed-precision path (the correction equation
// with homogeneous or periodic ghosts); float64 Dirichlet face data is folded
// into a copy of f by the callers before these run.
template <typename T>
Plan& block_plan(const rkl_grid& g, int s, double theta, int min_coarse) {
  return get_plan(g, s, theta, min_coarse, sizeof(T) == 8 ? RKL_FP64 : RKL_MIXED);
}

template <typename T>
T* level0_alt(Plan& P) {
  if constexpr (sizeof(T) == 8) return P.t0;
  else return P.h32.t[0];
}

template <typename T>
void copy_back(T* dst, const T* src, size_t n, hipStream_t st) {
  if (dst != src) HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToDevice, st));
}

// n_steps tau-steps of the plan's smoothing stage count on M phi = b
template <typename T>
void smooth_impl(Plan& P, const T* b, T* phi, int n_steps, hipStream_t st) {
  const LevelView<T> V0 = view<T>(P.lv[0], P.periodic, nullptr);
  T* cur = phi;
  T* alt = level0_alt<T>(P);
  relax_n<T>(P, V0, P.lv[0], n_steps, cur, alt, b, nullptr, st, single_batch(), false);
  copy_back<T>(phi, cur, P.lv[0].n, st);
}

// one V-cycle from phi on M phi = b; relative residual ||M phi - b|| / ||b||
// after it into *rel_out when asked
template <typename T>
void vcycle_impl(Plan& P, const rkl_opts& o, const T* b, T* phi, double* rel_out, hipStream_t st) {
  Hier<T>& H = [&]() -> Hier<T>& {
    if constexpr (sizeof(T) == 8) return P.h64;
    else return P.h32;
  }();
  T* cur = phi;
  T* alt = level0_alt<T>(P);
  vcycle_from<T>(P, H, cur, alt, b, nullptr, 0, o, nullptr, st, VBatch{1, 0, 0, P.dscal});
  copy_back<T>(phi, cur, P.lv[0].n, st);
  if (rel_out) {
    const LevelView<T> V0 = view<T>(P.lv[0], P.periodic, nullptr);
    const double r0 = resid_norm<T>(P, V0, (const T*)nullptr, b, st);
    const double r = resid_norm<T>(P, V0, phi, b, st);
    *rel_out = r0 > 0.0 ? r / r0 : r;
  }
}

// r = b - M u (homogeneous or periodic ghosts, or the level-0 face data in
// V.faces) and ||r||_2
template <typename T>
double residual_impl(Plan& P, const LevelView<T>& V, const T* b, const T* u, T* r_out, hipStream_t st) {
  launch_residual<T, T>(V, u, b, r_out, P.part, nullptr, st);
  launch_reduce(P.part, (int)resid_blocks(V.nx, V.ny, V.nz), 2, 1, P.dscal, nullptr, st);
  check_launch();
  return std::sqrt(readback(P, 1, st)[0]);
}

void check_fine_even(const rkl_grid& g) {
  if (g.nx % 2 || g.ny % 2 || (g.nz % 2 && !flat_grid(g)))
    fail(RKL_EINVAL, "fine sizes must be even (nz = 1 only for a two-dimensional grid)");
}

// coarsest-level solve of M u = b from u = 0; tau-steps taken (-1 when the
// level is too large for the one-workgroup kernel, which keeps no count)
template <typename T>
int coarse_impl(Plan& P, const rkl_opts& o, const T* b, T* u, hipStream_t st) {
  Hier<T> H;
  H.u = {u};
  H.b = {const_cast<T*>(b)};
  H.t = {level0_alt<T>(P)};
  const bool lds = coarse_in_lds(P, P.lv[0]);
  coarse_solve<T>(P, H, 0, o, nullptr, st);
  int steps = -1;
  if (lds) {
    HIPCHK(hipMemcpyAsync(P.hscal, P.dsteps, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::memcpy(&steps, P.hscal, sizeof(int));
  }
  copy_back<T>(u, H.u[0], P.lv[0].n, st);
  HIPCHK(hipStreamSynchronize(st));
  return steps;
}

// stage count and theta checks shared by the smoothing entry points
void check_smooth_args(int s, double tau_frac, int n_steps) {
  rkl_opts o;
  rkl_default_opts(&o);
  o.s = s;
  o.tau_frac = tau_frac;
  (void)resolve_opts(&o);
  if (s < 1) fail(RKL_EINVAL, "s must be in [1, 64]");
  if (n_steps < 0) fail(RKL_EINVAL, "n_steps must be >= 0");
}

template <typename T>
rkl_status restrict_entry(const rkl_grid* grid, const T* fine, T* coarse, void* hip_stream) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, nullptr);
    check_fine_even(*grid);
    if (!fine || !coarse) fail(RKL_EINVAL, "NULL array");
    hipStream_t st = (hipStream_t)hip_stream;
    launch_restrict<T>(grid->nx, grid->ny, grid->nz, fine, coarse, st);
    check_launch();
    HIPCHK(hipStreamSynchronize(st));
    return RKL_OK;
  });
}

template <typename T>
rkl_status prolong_entry(const rkl_grid* grid, const T* coarse, T* fine, void* hip_stream) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, nullptr);
    check_fine_even(*grid);
    if (!fine || !coarse) fail(RKL_EINVAL, "NULL array");
    hipStream_t st = (hipStream_t)hip_stream;
    launch_prolong_add<T>(grid->nx, grid->ny, grid->nz, grid->bc == RKL_BC_PERIODIC ? 1 : 0, coarse, fine,
                          nullptr, st);
    check_launch();
    HIPCHK(hipStreamSynchronize(st));
    return RKL_OK;
  });
}

template <typename T>
rkl_status coarse_entry(const rkl_grid* grid, const rkl_opts* opts, const T* b, T* u, int* steps_out,
                               void* hip_stream) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, nullptr);
    rkl_opts o = resolve_opts(opts);
    o.prec = sizeof(T) == 8 ? RKL_FP64 : RKL_MIXED;
    o = with_s(o, *grid);
    if (!b || !u) fail(RKL_EINVAL, "NULL array");
    Plan& P = block_plan<T>(*grid, o.s, o.tau_frac, INT_MAX);
    std::lock_guard<std::mutex> lk(P.mu);
    const int steps = coarse_impl<T>(P, o, b, u, (hipStream_t)hip_stream);
    if (steps_out) *steps_out = steps;
    return RKL_OK;
  });
}

}  // namespace rkl

using namespace rkl;

extern "C" {

rkl_status mg_vcycle(const rkl_grid* grid, const rkl_opts* opts, const double* f, const double* bc_faces,
                     double* phi, double* rel_res_out, void* hip_stream) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, bc_faces);
    rkl_opts o = resolve_opts(opts);
    o.prec = RKL_FP64;
    o = with_s(o, *grid);
    if (!f || !phi) fail(RKL_EINVAL, "f and phi must be non-NULL");
    Plan& P = block_plan<double>(*grid, o.s, o.tau_frac, o.min_coarse);
    std::lock_guard<std::mutex> lk(P.mu);
    hipStream_t st = (hipStream_t)hip_stream;
    fold_faces(P, bc_faces, f, P.f0, st);
    vcycle_impl<double>(P, o, P.f0, phi, rel_res_out, st);
    HIPCHK(hipStreamSynchronize(st));
    return RKL_OK;
  });
}

rkl_status mg_vcycle_f32(const rkl_grid* grid, const rkl_opts* opts, const float* f, float* phi,
                         double* rel_res_out, void* hip_stream) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, nullptr);
    rkl_opts o = resolve_opts(opts);
    o.prec = RKL_MIXED;
    o = with_s(o, *grid);
    if (!f || !phi) fail(RKL_EINVAL, "f and phi must be non-NULL");
    Plan& P = block_plan<float>(*grid, o.s, o.tau_frac, o.min_coarse);
    std::lock_guard<std::mutex> lk(P.mu);
    hipStream_t st = (hipStream_t)hip_stream;
    vcycle_impl<float>(P, o, f, phi, rel_res_out, st);
    HIPCHK(hipStreamSynchronize(st));
    return RKL_OK;
  });
}

rkl_status rkl_smooth(const rkl_grid* grid, int s, double tau_frac, int n_steps, const double* f,
                      const double* bc_faces, double* phi, void* hip_stream) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, bc_faces);
    check_smooth_args(s, tau_frac, n_steps);
    if (!f || !phi) fail(RKL_EINVAL, "f and phi must be non-NULL");
    Plan& P = block_plan<double>(*grid, s, tau_frac, INT_MAX);
    std::lock_guard<std::mutex> lk(P.mu);
    hipStream_t st = (hipStream_t)hip_stream;
    const double* b = f;  // f is used as given; face data, if any, is folded into a copy
    if (bc_faces != nullptr) {
      fold_faces(P, bc_faces, f, P.f0, st);
      b = P.f0;
    }
    smooth_impl<double>(P, b, phi, n_steps, st);
    HIPCHK(hipStreamSynchronize(st));
    return RKL_OK;
  });
}

rkl_status rkl_smooth_f32(const rkl_grid* grid, int s, double tau_frac, int n_steps, const float* f, float* phi,
                          void* hip_stream) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, nullptr);
    check_smooth_args(s, tau_frac, n_steps);
    if (!f || !phi) fail(RKL_EINVAL, "f and phi must be non-NULL");
    Plan& P = block_plan<float>(*grid, s, tau_frac, INT_MAX);
    std::lock_guard<std::mutex> lk(P.mu);
    hipStream_t st = (hipStream_t)hip_stream;
    smooth_impl<float>(P, f, phi, n_steps, st);
    HIPCHK(hipStreamSynchronize(st));
    return RKL_OK;
  });
}

rkl_status rkl_residual(const rkl_grid* grid, const double* f, const double* bc_faces, const double* phi,
                        double* r_out, double* norm_out, void* hip_stream) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, bc_faces);
    if (!f || !phi) fail(RKL_EINVAL, "f and phi must be non-NULL");
    Plan& P = block_plan<double>(*grid, 2, 0.9, INT_MAX);
    std::lock_guard<std::mutex> lk(P.mu);
    hipStream_t st = (hipStream_t)hip_stream;
    const LevelView<double> V0 = view<double>(P.lv[0], P.periodic, nullptr);
    fold_faces(P, bc_faces, f, P.f0, st);
    const double nrm = residual_impl<double>(P, V0, P.f0, phi, r_out, st);
    if (norm_out) *norm_out = nrm;
    return RKL_OK;
  });
}

rkl_status rkl_residual_f32(const rkl_grid* grid, const float* f, const float* phi, float* r_out, double* norm_out,
                            void* hip_stream) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, nullptr);
    if (!f || !phi) fail(RKL_EINVAL, "f and phi must be non-NULL");
    Plan& P = block_plan<double>(*grid, 2, 0.9, INT_MAX);  // partial sums and scalars only
    std::lock_guard<std::mutex> lk(P.mu);
    hipStream_t st = (hipStream_t)hip_stream;
    const LevelView<float> V0 = view<float>(P.lv[0], P.periodic, nullptr);
    const double nrm = residual_impl<float>(P, V0, f, phi, r_out, st);
    if (norm_out) *norm_out = nrm;
    return RKL_OK;
  });
}

rkl_status rkl_restrict(const rkl_grid* grid, const double* fine, double* coarse, void* hip_stream) {
  return restrict_entry<double>(grid, fine, coarse, hip_stream);
}

rkl_status rkl_restrict_f32(const rkl_grid* grid, const float* fine, float* coarse, void* hip_stream) {
  return restrict_entry<float>(grid, fine, coarse, hip_stream);
}

rkl_status rkl_prolong_add(const rkl_grid* grid, const double* coarse, double* fine, void* hip_stream) {
  return prolong_entry<double>(grid, coarse, fine, hip_stream);
}

rkl_status rkl_prolong_add_f32(const rkl_grid* grid, const float* coarse, float* fine, void* hip_stream) {
  return prolong_entry<float>(grid, coarse, fine, hip_stream);
}

rkl_status rkl_coarse_solve(const rkl_grid* grid, const rkl_opts* opts, const double* b, double* u,
                            int* steps_out, void* hip_stream) {
  return coarse_entry<double>(grid, opts, b, u, steps_out, hip_stream);
}

rkl_status rkl_coarse_solve_f32(const rkl_grid* grid, const rkl_opts* opts, const float* b, float* u,
                                int* steps_out, void* hip_stream) {
  return coarse_entry<float>(grid, opts, b, u, steps_out, hip_stream);
}

rkl_status rkl_gsrb_smooth(const rkl_grid* grid, double omega, int n_iter, const double* f, const double* bc_faces,
                           double* phi, void* hip_stream) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, bc_faces);
    if (!(omega > 0.0 && omega < 2.0)) fail(RKL_EINVAL, "omega must be in (0, 2)");
    if (n_iter < 0) fail(RKL_EINVAL, "n_iter must be >= 0");
    if (!f || !phi) fail(RKL_EINVAL, "f and phi must be non-NULL");
    Plan& P = get_plan(*grid, 2, 0.9, INT_MAX, RKL_FP64);
    std::lock_guard<std::mutex> lk(P.mu);
    hipStream_t st = (hipStream_t)hip_stream;
    const LevelView<double> V0 = view<double>(P.lv[0], P.periodic, nullptr);
    fold_faces(P, bc_faces, f, P.f0, st);
    double* cur = phi;
    double* alt = P.t0;
    for (int q = 0; q < n_iter; ++q) gsrb_iter<double>(V0, cur, alt, P.f0, omega, nullptr, st);
    if (cur != phi) copy_d2d(phi, cur, P.lv[0].n, st);
    HIPCHK(hipStreamSynchronize(st));
    return RKL_OK;
  });
}

rkl_status rkl_gradient(const rkl_grid* grid, const double* phi, const double* bc_faces, double* gx, double* gy,
                        double* gz, void* hip_stream) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, bc_faces);
    if (!phi || !gx || !gy || !gz) fail(RKL_EINVAL, "phi, gx, gy and gz must be non-NULL");
    if (grid->bc == RKL_BC_DIRICHLET && (grid->nx < 2 || grid->ny < 2 || (grid->nz < 2 && !flat_grid(*grid))))
      fail(RKL_EINVAL, "Dirichlet gradients need at least 2 cells along every axis");
    launch_gradient(grid->nx, grid->ny, grid->nz, grid->hx, grid->hy, grid->hz, grid->bc == RKL_BC_PERIODIC ? 1 : 0,
                    bc_faces, phi, gx, gy, gz, (hipStream_t)hip_stream);
    check_launch();
    return RKL_OK;
  });
}

void rkl_default_relax_opts(rkl_relax_opts* o) {
  if (!o) return;
  o->method = RKL_RELAX_RKL;
  o->s = 0;
  o->tau_frac = 0.9;
  o->omega = 0.0;
  o->tol_max = 1e-10;
  o->max_iters = 100000;
  o->check_every = 1;
}

rkl_status rkl_relax_solve(const rkl_grid* grid, const rkl_relax_opts* opts, const double* f, const double* bc_faces,
                           double* phi, rkl_stats* stats, void* hip_stream) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, bc_faces);
    rkl_relax_opts ro;
    rkl_default_relax_opts(&ro);
    if (opts) ro = *opts;
    if (ro.method != RKL_RELAX_RKL && ro.method != RKL_RELAX_GSRB && ro.method != RKL_RELAX_SOR)
      fail(RKL_EINVAL, "unknown relaxation method");
    if (ro.s < -1 || ro.s > 4096) fail(RKL_EINVAL, "s must be in [-1, 4096]");
    if (!(ro.tau_frac > 0.0 && ro.tau_frac < 2.0)) fail(RKL_EINVAL, "tau_frac must be in (0, 2)");
    if (!(ro.omega >= 0.0 && ro.omega < 2.0)) fail(RKL_EINVAL, "omega must be in [0, 2)");
    if (!(ro.tol_max >= 0.0)) fail(RKL_EINVAL, "tol_max must be >= 0");
    if (ro.max_iters < 0 || ro.check_every < 1) fail(RKL_EINVAL, "need max_iters >= 0 and check_every >= 1");
    if (!f || !phi) fail(RKL_EINVAL, "f and phi must be non-NULL");
    if (stats) stats->history_len = 0;
    const bool rkl = ro.method == RKL_RELAX_RKL;
    if (rkl && ro.s == -1) {  // the fixed stage count of App. A.3 for this grid
      const Lev L0 = build_levels(*grid, INT_MAX, 1, ro.tau_frac)[0];
      ro.s = s_opt_rule(L0, grid->bc == RKL_BC_PERIODIC, ro.tau_frac, 6, 2.0, nullptr);
    }
    Plan& P = get_plan(*grid, rkl && ro.s > 0 ? ro.s : 2, ro.tau_frac, INT_MAX, RKL_FP64);
    std::lock_guard<std::mutex> lk(P.mu);
    hipStream_t st = (hipStream_t)hip_stream;
    const Lev& F = P.lv[0];
    const LevelView<double> V0 = view<double>(F, P.periodic, nullptr);
    fold_faces(P, bc_faces, f, P.f0, st);
    f = P.f0;
    double omega = 1.0;
    if (ro.method == RKL_RELAX_SOR) {
      omega = ro.omega;
      if (omega == 0.0) {
        const double ix = 1.0 / (grid->hx * grid->hx), iy = 1.0 / (grid->hy * grid->hy),
                     iz = 1.0 / (grid->hz * grid->hz);
        const double rj = (std::cos(M_PI / grid->nx) * ix + std::cos(M_PI / grid->ny) * iy +
                           std::cos(M_PI / grid->nz) * iz) / (ix + iy + iz);
        omega = 2.0 / (1.0 + std::sqrt(1.0 - rj * rj));
      }
    }
    double* cur = phi;
    double* alt = P.t0;
    double* x3 = P.t0b;  // scratch of the chunked large-s tau-steps
    double* x4 = rkl ? P.t0c() : nullptr;
    int it = 0;
    double res = 0.0;
    rkl_status status = RKL_OK;
    bool first = true;
    while (true) {
      launch_resid_absmax<double>(V0, cur, f, P.part, P.dscal, st);
      check_launch();
      res = readback(P, 1, st)[0];
      record(stats, res);
      if (first && stats) stats->res0 = res;
      first = false;
      if (!std::isfinite(res)) {
        status = RKL_ENONFINITE;
        g_err = "non-finite residual";
        break;
      }
      if (res <= ro.tol_max) break;
      if (it >= ro.max_iters) {
        status = RKL_ENOCONV;
        g_err = "max_iters reached before tol_max";
        break;
      }
      for (int c = 0; c < ro.check_every && it < ro.max_iters; ++c) {
        if (rkl) {
          const std::vector<StageCoef>& co =
              ro.s > 0 ? F.smooth : P.sched_coef[std::min(it, (int)P.sched_coef.size() - 1)];
          if (!tau_chunked<double>(V0, cur, alt, x3, x4, f, co, st)) tau_step<double>(P, V0, cur, alt, f, co, nullptr, st);
        } else {
          gsrb_iter<double>(V0, cur, alt, f, omega, nullptr, st);
        }
        if (P.periodic) remove_mean<double>(P, cur, F.n, nullptr, st);
        ++it;
      }
    }
    if (cur != phi) copy_d2d(phi, cur, F.n, st);
    HIPCHK(hipStreamSynchronize(st));
    if (stats) {
      stats->cycles = it;
      stats->levels = 1;
      stats->rel_res = res;
      stats->status = status;
    }
    return status;
  });
}

}  // extern "C"
