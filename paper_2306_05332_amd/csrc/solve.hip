// Single solves (rkl_poisson_solve): source preparation, the device-side
// convergence loop over float64 V-cycles (Sec. 2.1, Sec. 4.1 stop metric)
// and the mixed-precision defect correction.

#include <limits>

#include "solver_core.h"

namespace rkl {

// dst = src with the Dirichlet face data moved into the right-hand side
// (every kernel then applies the homogeneous ghost -u on every level)
void fold_faces(Plan& P, const double* faces, const double* src, double* dst, hipStream_t st) {
  const Lev& F = P.lv[0];
  if (faces != nullptr) {
    launch_fold_faces(F.nx, F.ny, F.nz, F.hx, F.hy, F.hz, faces, src, dst, st);
    check_launch();
  } else if (src != dst) {
    HIPCHK(hipMemcpyAsync(dst, src, F.n * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
}

// f0 = four_pi_G * rho, mean removed when periodic (f0 = c (rho - mean rho):
// one read-only pass for the sum, one pass writing f0); the scaling pass
// leaves the block partials of f0^2 in P.part (stride 2, offset 1)
void prepare_source(Plan& P, const double* rho, double c, hipStream_t st) {
  const size_t n = P.lv[0].n;
  const double* sum = nullptr;
  if (P.periodic) {
    launch_sum<double>(rho, n, P.part, st);
    launch_reduce(P.part, (int)ew_block_count(n), 1, 1, P.dscal + 8, nullptr, st);
    check_launch();
    sum = P.dscal + 8;
  }
  launch_scale(rho, P.f0, n, c, sum, (double)n, P.part, st);
  check_launch();
}

void copy_d2d(double* dst, const double* src, size_t n, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, st));
}

void record(rkl_stats* stats, double rel) {
  if (stats && stats->history && stats->history_len < stats->history_cap)
    stats->history[stats->history_len++] = rel;
}

// reset the device convergence state with a kernel-free copy from the pinned
// mirror (no memset: the sequence stays capturable)
// zero the device convergence state's header (one small fill kernel, no
// host-to-device copy) and its host mirror, which then describes the state
// the loop starts from without reading it back
void conv_reset(Plan& P, hipStream_t st) {
  static_assert(offsetof(ConvState, hist) % sizeof(double) == 0, "ConvState header is whole doubles");
  launch_fill<double>(reinterpret_cast<double*>(P.dconv), offsetof(ConvState, hist) / sizeof(double), 0.0, nullptr,
                      st);
  check_launch();
  std::memset(P.hconv, 0, sizeof(ConvState));
}

const ConvState& conv_read(Plan& P, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(P.hconv, P.dconv, sizeof(ConvState), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return *P.hconv;
}

// how many more cycles to queue: enough to reach tol at the observed
// contraction (0.12 before any is observed), plus the cycle whose start
// state is tested last
int predict_batch(const ConvState& cs, double tol, int queued, int max_cycles) {
  double rho = 0.12, last = 1.0;
  const int m = cs.m;  // states tested so far
  if (m >= 1 && m - 1 < CONV_HIST) last = cs.hist[m - 1];
  if (m >= 2 && m - 1 < CONV_HIST && cs.hist[m - 2] > 0.0) rho = cs.hist[m - 1] / cs.hist[m - 2];
  rho = std::min(0.9, std::max(0.01, rho));
  // state m (the start of the next cycle to queue) is one cycle past the last
  // tested one, so ceil(log(tol/last)/log(rho)) cycles reach a tested state
  // below tol; before any test, state 0 itself needs a cycle of its own
  int need = 1;
  if (last > tol && tol > 0.0) need = (int)std::ceil(std::log(tol / last) / std::log(rho)) + (m == 0 ? 1 : 0);
  need = std::max(1, std::min(need, 64));
  const int left = max_cycles + 1 - queued;
  return std::max(1, std::min(need, left));
}

void fill_stats(rkl_stats* stats, const ConvState& cs, int result_m) {
  if (!stats) return;
  stats->history_len = 0;
  for (int q = 0; q <= result_m && q < CONV_HIST; ++q) record(stats, cs.hist[q]);
  stats->cycles = result_m;
  stats->rel_res = cs.rel;
}

// ------------------------------------------------------------------ solves
// pinned host slot of the deferred ||f0||^2 (no other read-back writes it)
constexpr int RES0_HOST = 15;

// The mixed path folds its float64 update into the next defect pass when phi
// (8 bytes a cell) and e (4) overflow the 256 MB last-level cache.
// Measured on gfx950: 512^3 defect + update 553 + 550 us per outer iteration
// apart; at 256^3, where they fit, the fold saved nothing.
constexpr size_t MIXED_FOLD_MIN_BYTES = (size_t)256 << 20;

// Common start: f0, ||M 0 - f0||.  Returns false when the solve is already
// decided (zero right-hand side or non-finite data); `status` says how.
// With `defer` the host does not wait for ||f0||: the value is copied into a
// pinned slot in stream order and the caller queues its first cycles at once
// (their device-side check stops at once on a zero or non-finite ||f0||),
// then settles those two cases with solve_start_settle after the loop's first
// synchronisation.
bool solve_start(Plan& P, const rkl_opts& o, const double* rho, const double* faces, double* phi,
                 rkl_stats* stats, hipStream_t st, double& res0, rkl_status& status, bool defer = false) {
  const Lev& F = P.lv[0];
  const LevelView<double> V0 = view<double>(F, P.periodic, nullptr);
  prepare_source(P, rho, o.four_pi_G, st);
  // res0^2 lands in the slot the convergence check reads (Res0Sqrt)
  if (faces != nullptr) {
    fold_faces(P, faces, P.f0, P.f0, st);
    resid_norm2_async<double>(P, V0, nullptr, P.f0, st, RES0SQ_SLOT);
  } else {  // ||M 0 - f0||^2 is the sum of f0^2: the scaling pass's partials
    launch_reduce(P.part + 1, (int)ew_block_count(F.n), 2, 1, P.dscal + RES0SQ_SLOT, nullptr, st);
    check_launch();
  }
  conv_reset(P, st);  // issued before the read-back so that it is done when the loop starts
  status = RKL_OK;
  if (stats) {
    stats->levels = P.L();
    stats->cycles = 0;
    stats->rel_res = 0.0;
  }
  if (defer) {
    HIPCHK(hipMemcpyAsync(P.hscal + RES0_HOST, P.dscal + RES0SQ_SLOT, sizeof(double), hipMemcpyDeviceToHost, st));
    res0 = std::numeric_limits<double>::quiet_NaN();
    return true;
  }
  res0 = std::sqrt(readback(P, 1, st, RES0SQ_SLOT)[0]);
  if (stats) stats->res0 = res0;
  if (res0 == 0.0) {
    launch_fill<double>(phi, F.n, 0.0, nullptr, st);
    check_launch();
    HIPCHK(hipStreamSynchronize(st));
    return false;
  }
  if (!std::isfinite(res0)) {
    g_err = "non-finite source or boundary data";
    status = RKL_ENONFINITE;
    return false;
  }
  return true;
}

// The deferred half of solve_start, after a synchronisation of the stream
// that followed its copy: false when the solve is decided as solve_start
// would have decided it (phi = 0 for a zero right-hand side).
bool solve_start_settle(Plan& P, double* phi, rkl_stats* stats, hipStream_t st, rkl_status& status) {
  const double res0 = std::sqrt(P.hscal[RES0_HOST]);
  if (stats) stats->res0 = res0;
  if (res0 == 0.0) {
    launch_fill<double>(phi, P.lv[0].n, 0.0, nullptr, st);
    check_launch();
    HIPCHK(hipStreamSynchronize(st));
    status = RKL_OK;
    return false;
  }
  if (!std::isfinite(res0)) {
    g_err = "non-finite source or boundary data";
    status = RKL_ENONFINITE;
    return false;
  }
  return true;
}

rkl_status finish_status(const ConvState& cs) {
  switch (cs.status) {
    case 0: return RKL_OK;
    case -3:
      g_err = cs.stalled ? "residual stalled at " + std::to_string(cs.rel) +
                               " above tol (no 10% reduction in 8 cycles: the float64 rounding floor of M phi - f)"
                         : std::string("max_cycles reached before tol");
      return RKL_ENOCONV;
    case -4: g_err = "residual grew in 3 consecutive cycles to over twice its best"; return RKL_EDIVERGED;
    case -5: g_err = "non-finite residual"; return RKL_ENONFINITE;
    default: g_err = "unexpected convergence state"; return RKL_EHIP;
  }
}

rkl_status solve_fp64(Plan& P, const rkl_opts& o, const double* rho, const double* faces, double* phi,
                      rkl_stats* stats, hipStream_t st) {
  const Lev& F = P.lv[0];
  const LevelView<double> V0 = view<double>(F, P.periodic, nullptr);  // face data folded into f0
  double res0;
  rkl_status status;
  if (!solve_start(P, o, rho, faces, phi, stats, st, res0, status, P.L() > 1)) return status;

  if (P.L() == 1) {
    // single level: accelerated RKL iteration (App. A.4, App. B) to tol
    if (o.zero_start) {
      launch_fill<double>(phi, F.n, 0.0, nullptr, st);
      check_launch();
    }
    int cycles = 0;
    double res = 0.0;
    double* cur = phi;
    double* alt = P.t0;
    if (coarse_in_lds(P, F)) {
      launch_coarse_solve<double>(V0, P.f0, phi, P.t0, P.cs(), o.tol, res0, o.max_cycles, 0, P.dsteps,
                                  P.dscal, nullptr, st);
      check_launch();
      copy_d2d(phi, P.t0, F.n, st);
      HIPCHK(hipMemcpyAsync(P.hscal, P.dsteps, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(P.hscal + 1, P.dscal, sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      int steps;
      std::memcpy(&steps, P.hscal, sizeof(int));
      cycles = steps;
      res = P.hscal[1];
    } else {
      cycles = accel_multi<double>(P, V0, cur, alt, P.f0, o.tol, res0, o.max_cycles, false, st, &res, P.t0b,
                                   P.t0c());
      if (cur != phi) copy_d2d(phi, cur, F.n, st);
    }
    const double rel = res / res0;
    record(stats, rel);
    if (!std::isfinite(rel)) status = RKL_ENONFINITE;
    else if (rel > o.tol) {
      status = RKL_ENOCONV;
      g_err = "max_cycles reached before tol";
    }
    if (P.periodic) remove_mean<double>(P, phi, F.n, nullptr, st);
    HIPCHK(hipStreamSynchronize(st));
    if (stats) {
      stats->cycles = cycles;
      stats->rel_res = rel;
    }
    return status;
  }

  // V-cycles with the convergence test on the device.  Cycle m starts from
  // buffer bufs[start[m]] and writes only the other two, so when the test at
  // the start of cycle m stops the loop, that buffer is the answer.
  double* bufs[3] = {phi, P.t0, P.t0b};
  std::vector<int> start(1, 0);
  const int* stop = &P.dconv->stop;  // the state was reset by solve_start
  const bool gs = o.smoother == RKL_SMOOTH_GSRB;
  const bool fused0 = fused_tau_supported<double>(V0, gs ? 2 : o.s) && o.n_pre > 0;
  const bool pair0 = fused0 && o.n_pre >= 2 && pair_ok<double>(V0, o.s, gs);
  // zero_start: cycle 0 relaxes from the zero iterate without reading phi
  // (the fused tau-step's zero-input form: 16 bytes a cell instead of 24);
  // other paths start from phi filled with zeros
  const bool cold0 = o.zero_start && fused0 && !gs;
  if (o.zero_start && !cold0) {
    launch_fill<double>(phi, F.n, 0.0, nullptr, st);
    check_launch();
  }
  int queued = 0;
  ConvState cs = *P.hconv;  // as reset
  while (true) {
    const int batch = predict_batch(cs, o.tol, queued, o.max_cycles);
    for (int q = 0; q < batch; ++q) {
      const int m = queued;
      const int ia = start[m], ib = (ia + 1) % 3, ic = (ia + 2) % 3;
      double* a = bufs[ia];
      double *cur, *alt;
      int pre_done;
      int nblk, stride;
      if (fused0) {
        // first relaxation, fused with the residual norm of the start state
        tau_keep<double>(P, V0, (cold0 && m == 0) ? nullptr : a, bufs[ib], bufs[ic], cur, alt, P.f0,
                         pair0 ? F.smooth2 : F.smooth, P.part, stop, st, gs);
        nblk = (int)(gs ? gsrb_blocks<double>(V0) : fused_tau_blocks<double>(V0, pair0 ? 2 * o.s : o.s));
        stride = 1;
        launch_check(P.part, nblk, stride, Res0Sqrt::ptr(P), o.tol, o.max_cycles, 1.0, P.dconv, st);
        check_launch();
        pre_done = pair0 ? 2 : 1;
      } else {
        launch_residual<double, double>(V0, a, P.f0, (double*)nullptr, P.part, stop, st);
        nblk = (int)resid_blocks(F.nx, F.ny, F.nz);
        stride = 2;
        launch_check(P.part, nblk, stride, Res0Sqrt::ptr(P), o.tol, o.max_cycles, 1.0, P.dconv, st);
        check_launch();
        if (o.n_pre > 0) {
          tau_keep<double>(P, V0, a, bufs[ib], bufs[ic], cur, alt, P.f0, F.smooth, nullptr, stop, st, gs);
          pre_done = 1;
        } else {
          // the copy respects the stop flag like every kernel of the cycle: a
          // cycle queued past the stopping one must leave bufs[ia] intact
          launch_copy<double>(bufs[ib], a, F.n, stop, st);
          check_launch();
          cur = bufs[ib];
          alt = bufs[ic];
          pre_done = 0;
        }
      }
      vcycle_from<double>(P, P.h64, cur, alt, P.f0, nullptr, pre_done, o, stop, st, VBatch{1, 0, 0, P.dscal});
      int ie = 0;
      for (int k = 0; k < 3; ++k)
        if (bufs[k] == cur) ie = k;
      start.push_back(ie);
      ++queued;
    }
    cs = conv_read(P, st);
    if (cs.stop) break;
    if (queued > o.max_cycles) fail(RKL_EHIP, "convergence loop ended without a decision");
  }
  if (!solve_start_settle(P, phi, stats, st, status)) return status;
  const int rm = cs.result_m;
  double* res = bufs[start[rm]];
  if (cold0 && rm == 0) {  // the answer is the zero start state, which phi never held
    launch_fill<double>(phi, F.n, 0.0, nullptr, st);
    check_launch();
  } else if (P.periodic && res != phi) {  // phi = res - mean(res): the copy carries the mean removal
    launch_sum<double>(res, F.n, P.part, st);
    launch_reduce(P.part, (int)ew_block_count(F.n), 1, 1, P.dscal + 8, nullptr, st);
    launch_copy_sub_mean(phi, res, F.n, P.dscal + 8, (double)F.n, st);
    check_launch();
  } else {
    if (res != phi) copy_d2d(phi, res, F.n, st);
    if (P.periodic) remove_mean<double>(P, phi, F.n, nullptr, st);
  }
  HIPCHK(hipStreamSynchronize(st));
  fill_stats(stats, cs, rm);
  return finish_status(cs);
}

rkl_status solve_mixed(Plan& P, const rkl_opts& o, const double* rho, const double* faces, double* phi,
                       rkl_stats* stats, hipStream_t st) {
  const Lev& F = P.lv[0];
  const LevelView<double> V0 = view<double>(F, P.periodic, nullptr);  // face data folded into f0
  const LevelView<float> V32 = view<float>(F, P.periodic, nullptr);
  double res0;
  rkl_status status;
  if (!solve_start(P, o, rho, faces, phi, stats, st, res0, status, true)) return status;
  if (o.zero_start) {
    launch_fill<double>(phi, F.n, 0.0, nullptr, st);
    check_launch();
  }
  const int* stop = &P.dconv->stop;  // the state was reset by solve_start
  const int nblk = (int)resid_blocks(F.nx, F.ny, F.nz);
  // When phi and e together overflow the last-level cache, the update
  // phi += e of an iteration is folded into the next iteration's defect pass
  // (launch_residual_add), which writes the updated phi into the other one
  // of ph[]: state k lives in ph[k & 1].  Below that size the separate update
  // re-reads phi and e from the cache and the fold saves nothing.
  const bool fold = F.nz > 1 && 12.0 * (double)F.n > (double)MIXED_FOLD_MIN_BYTES;
  double* ph[2] = {phi, P.t0};
  const float* eprev = nullptr;  // the last queued iteration's correction (fold)
  int queued = 0;
  ConvState cs = *P.hconv;  // as reset
  while (true) {
    const int batch = predict_batch(cs, o.tol, queued, o.max_cycles);
    for (int q = 0; q < batch; ++q) {
      // float64 defect r = f - M phi, stored as the float32 right-hand side
      if (fold && queued > 0)
        launch_residual_add(V0, ph[(queued - 1) & 1], eprev, P.f0, ph[queued & 1], P.h32.b[0], P.part, stop, st);
      else  // zero_start: the first defect is f itself (phi = 0 is not read)
        launch_residual<double, float>(V0, (o.zero_start && queued == 0) ? nullptr : phi, P.f0, P.h32.b[0], P.part,
                                       stop, st);
      launch_check(P.part, nblk, 2, Res0Sqrt::ptr(P), o.tol, o.max_cycles, (double)F.n, P.dconv, st);
      check_launch();
      // periodic: the defect of the mean-free f sums to zero up to rounding
      // (the periodic M sums to zero); the rounding-level mean that the
      // restriction carries is dropped on level 1, so level 0 needs no pass
      // one float32 V-cycle on M e = r from e = 0 (homogeneous level-0 ghosts)
      float* cur = P.h32.u[0];
      float* alt = P.h32.t[0];
      int pre_done = 0;
      if (o.n_pre > 0) {
        pre_done = relax_from_zero<float>(P, V32, F, o.n_pre, cur, alt, P.h32.b[0], stop, st, single_batch(),
                                          o.smoother == RKL_SMOOTH_GSRB);
      } else {
        launch_fill<float>(cur, F.n, 0.0f, stop, st);
      }
      vcycle_from<float>(P, P.h32, cur, alt, P.h32.b[0], nullptr, pre_done, o, stop, st, VBatch{1, 0, 0, P.dscal});
      if (fold) eprev = cur;  // read by the next iteration's defect pass, before its V-cycle runs
      else launch_add_cast<float>(phi, cur, F.n, stop, st);
      check_launch();
      ++queued;
    }
    cs = conv_read(P, st);
    if (cs.stop) break;
    if (queued > o.max_cycles) fail(RKL_EHIP, "refinement loop ended without a decision");
  }
  if (!solve_start_settle(P, phi, stats, st, status)) return status;
  double* ans = fold ? ph[cs.result_m & 1] : phi;  // the tested state
  if (P.periodic && ans != phi) {  // phi = ans - mean(ans): the copy carries the mean removal
    launch_sum<double>(ans, F.n, P.part, st);
    launch_reduce(P.part, (int)ew_block_count(F.n), 1, 1, P.dscal + 8, nullptr, st);
    launch_copy_sub_mean(phi, ans, F.n, P.dscal + 8, (double)F.n, st);
    check_launch();
  } else if (ans != phi) {
    copy_d2d(phi, ans, F.n, st);
  } else if (P.periodic) {
    remove_mean<double>(P, phi, F.n, nullptr, st);
  }
  HIPCHK(hipStreamSynchronize(st));
  fill_stats(stats, cs, cs.result_m);
  return finish_status(cs);
}

// One full solve.  A single-level grid runs the float64 accelerated RKL
// iteration whatever the precision asks: with no coarse grid there is no
// float32 V-cycle to refine.
rkl_status solve_one(const rkl_grid& g, const rkl_opts& o, const double* rho, const double* faces, double* phi,
                     rkl_stats* stats, hipStream_t st) {
  Plan* P = &get_plan(g, o.s, o.tau_frac, o.min_coarse, o.prec);
  const bool mixed = o.prec == RKL_MIXED && P->L() > 1;
  if (o.prec == RKL_MIXED && !mixed) P = &get_plan(g, o.s, o.tau_frac, o.min_coarse, RKL_FP64);
  std::lock_guard<std::mutex> lk(P->mu);
  const rkl_status r = mixed ? solve_mixed(*P, o, rho, faces, phi, stats, st) : solve_fp64(*P, o, rho, faces, phi, stats, st);
  if (stats) stats->status = r;
  return r;
}

}  // namespace rkl

using namespace rkl;

extern "C" {

rkl_status rkl_poisson_solve(const rkl_grid* grid, const rkl_opts* opts, const double* rho,
                             const double* bc_faces, double* phi, rkl_stats* stats, void* hip_stream) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, bc_faces);
    const rkl_opts o = with_s(resolve_opts(opts), *grid);
    if (!rho || !phi) fail(RKL_EINVAL, "rho and phi must be non-NULL");
    if (stats) stats->history_len = 0;
    return solve_one(*grid, o, rho, bc_faces, phi, stats, (hipStream_t)hip_stream);
  });
}

}  // extern "C"
