// Internals of the solver's host side shared by its translation units
// (plan.hip, solve.hip, batch.hip, tune.hip, levels.hip): the level
// hierarchy and plan cache, the tau-step and V-cycle drivers (templates,
// instantiated where they are used) and the helpers of the solves.
//
// Method (Mandal, Mukherjee & Mignone 2023):
//  * correction-scheme V-cycle, Sec. 2.1, with every level written as
//    M_l u_l = b_l, b_0 = f, b_{l+1} = -R(M_l u_l - b_l) (the listing's coarse
//    signs made consistent), N_pre = 2, N_post = 1 (Sec. 4.1);
//  * relaxation: one s-stage RKL1 tau-step (App. A eq. RKL_intermediate_source)
//    with tau = theta * tau_max(s), tau_max from eq. tau_max and
//    |lambda_max| = 4 sum_d h_d^-2;
//  * coarsest level: accelerated RKL schedule (App. A.4, eq. sk_optimal
//    generalised to 3-D through x_k = 1 - theta Delta t_par |lambda_k|);
//  * periodic compatibility: f -= mean(f) and coarse right-hand sides made
//    mean-free (Sec. 2.3);
//  * stop metric: ||M u - f||_2 / ||M 0 - f||_2 (Sec. 4.1).
#pragma once

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "host_common.h"
#include "kernels.h"

namespace rkl {

// ------------------------------------------------------------------ levels
struct Lev {
  int nx, ny, nz;
  double hx, hy, hz;
  bool flat;                       // two-dimensional: nz = 1, hz = inf (no z coupling)
  size_t n;
  double lam, dtpar;               // Lambda_l = 4 sum h^-2, Delta t_par = 2 / Lambda_l
  std::vector<StageCoef> smooth;   // coefficients of the smoothing tau-step
  std::vector<StageCoef> smooth2;  // two smoothing tau-steps as one 2s-stage recurrence
};
std::vector<StageCoef> stage_coefs(int s, double theta, double dtpar);
std::vector<int> accel_schedule(const Lev& L, bool periodic, double theta);
int s_opt_rule(const Lev& L, bool periodic, double theta, int kmax, double digits, double* m_out);

// ------------------------------------------------------------------ plan
template <typename T>
struct Hier {
  std::vector<T*> u, b, t;
};

struct PlanKey {
  int dev, nx, ny, nz, bc, s, min_coarse, prec;
  double hx, hy, hz, theta;
  bool operator<(const PlanKey& o) const {
    return std::tie(dev, nx, ny, nz, bc, s, min_coarse, prec, hx, hy, hz, theta) <
           std::tie(o.dev, o.nx, o.ny, o.nz, o.bc, o.s, o.min_coarse, o.prec, o.hx, o.hy, o.hz,
                    o.theta);
  }
};

struct Plan {
  PlanKey key;
  bool periodic = false;
  std::vector<Lev> lv;
  Hier<double> h64;
  Hier<float> h32;
  double* f0 = nullptr;   // level-0 source (float64)
  double* t0 = nullptr;   // level-0 alternate iterates (float64): with phi they form the
  double* t0b = nullptr;  // three buffers that keep a cycle's start state intact
  double* t0c_ = nullptr;  // fourth level-0 array (chunked large-s tau-steps), allocated on first use
  double* t0c() {
    if (!t0c_) t0c_ = alloc<double>(lv[0].n);
    return t0c_;
  }
  ConvState* dconv = nullptr;  // device convergence state
  ConvState* hconv = nullptr;  // pinned host mirror
  double* part = nullptr;
  size_t part_cap = 0;
  double* dscal = nullptr;  // device scalars
  double* hscal = nullptr;  // pinned host mirror
  int* dsteps = nullptr;
  // coarsest-level schedule
  std::vector<int> sched;
  std::vector<std::vector<StageCoef>> sched_coef;
  int* d_sched = nullptr;
  int* d_coff = nullptr;
  double* d_coef = nullptr;
  int tail64 = -1, tail32 = -1;  // first level run by the one-workgroup tail (-1: none)
  std::vector<void*> allocs;
  std::mutex mu;

  int L() const { return (int)lv.size(); }
  CoarseSchedule cs() const { return {d_sched, d_coff, d_coef, (int)sched.size()}; }

  template <typename U>
  U* alloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    if (hipMalloc(&p, n * sizeof(U)) != hipSuccess) {
      (void)hipGetLastError();
      fail(RKL_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(U)) + " bytes failed");
    }
    allocs.push_back(p);
    return (U*)p;
  }
  ~Plan() {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(key.dev);
    for (void* p : allocs) (void)hipFree(p);
    if (hscal) (void)hipHostFree(hscal);
    if (hconv) (void)hipHostFree(hconv);
    (void)hipSetDevice(cur);
  }
};

// P.dscal slots: 0 reductions in passing, 5 res0^2 of the running solve
// (read by the convergence check), 8 periodic sums
constexpr int RES0SQ_SLOT = 5;
std::vector<Lev> build_levels(const rkl_grid& g, int min_coarse, int s, double theta);

bool coarse_in_lds(const Plan& P, const Lev& C);
TailShape tail_shape(const Plan& P, int lt);
Plan& get_plan(const rkl_grid& g, int s, double theta, int min_coarse, int prec);

template <typename T>
LevelView<T> view(const Lev& L, bool periodic, const double* faces) {
  LevelView<T> v;
  v.nx = L.nx;
  v.ny = L.ny;
  v.nz = L.nz;
  v.ihx2 = (T)(1.0 / (L.hx * L.hx));
  v.ihy2 = (T)(1.0 / (L.hy * L.hy));
  v.ihz2 = (T)(1.0 / (L.hz * L.hz));
  v.periodic = periodic ? 1 : 0;
  v.faces = faces;
  return v;
}
bool coarse_in_lds(const Plan& P, const Lev& C);
const double* readback(Plan& P, int nq, hipStream_t st, int at = 0);

// ||b - M u||^2 into P.dscal[at] (u may be nullptr), not synchronising
template <typename T>
void resid_norm2_async(Plan& P, const LevelView<T>& V, const T* u, const T* b, hipStream_t st, int at = 0) {
  launch_residual<T, T>(V, u, b, (T*)nullptr, P.part, nullptr, st);
  check_launch();
  launch_reduce(P.part, (int)resid_blocks(V.nx, V.ny, V.nz), 2, 1, P.dscal + at, nullptr, st);
  check_launch();
}

// ||b - M u||_2, synchronising
template <typename T>
double resid_norm(Plan& P, const LevelView<T>& V, const T* u, const T* b, hipStream_t st) {
  resid_norm2_async<T>(P, V, u, b, st);
  return std::sqrt(readback(P, 1, st)[0]);
}

template <typename T>
void remove_mean(Plan& P, T* a, size_t n, const int* stop, hipStream_t st) {
  launch_sum<T>(a, n, P.part, st);
  launch_reduce(P.part, (int)ew_block_count(n), 1, 1, P.dscal + 8, stop, st);
  launch_sub_mean<T>(a, n, P.dscal + 8, (double)n, stop, st);
  check_launch();
}

// ------------------------------------------------------------------ tau-steps
// One tau-step on M u = b from `cur`; the result ends in `cur` (the buffers
// are swapped when it lands in `alt`).  Fused single-pass kernel when the
// level supports it, otherwise one kernel per stage with Y_j written over
// Y_{j-2}.
// One red-black Gauss-Seidel / SOR iteration (Sec. 2.2.4) from `cur`; the
// result ends in `cur`.  One pass when the level takes the strip kernel,
// else two one-colour passes.
template <typename T>
void gsrb_iter(const LevelView<T>& V, T*& cur, T*& alt, const T* b, double omega, const int* stop, hipStream_t st,
               const Batch& bt = single_batch()) {
  if (launch_gsrb_fused<T>(V, cur, b, alt, omega, nullptr, stop, st, bt)) {
    check_launch();
    std::swap(cur, alt);
    return;
  }
  if (bt.nb > 1) fail(RKL_EINVAL, "batched solves need the fused smoother on every level above the tail");
  launch_gsrb_half<T>(V, cur, alt, b, 0, omega, stop, st);
  launch_gsrb_half<T>(V, alt, cur, b, 1, omega, stop, st);
  check_launch();
}

template <typename T>
void tau_step(Plan& P, const LevelView<T>& V, T*& cur, T*& alt, const T* b,
              const std::vector<StageCoef>& co, const int* stop, hipStream_t st,
              const Batch& bt = single_batch(), bool gs = false) {
  if (gs) return gsrb_iter<T>(V, cur, alt, b, 1.0, stop, st, bt);
  const int s = (int)co.size();
  if (launch_fused_tau<T>(V, cur, b, alt, s, co.data(), nullptr, stop, st, bt)) {
    check_launch();
    std::swap(cur, alt);
    return;
  }
  if (bt.nb > 1) fail(RKL_EINVAL, "batched solves need the fused tau-step on every level above the tail");
  launch_stage<T>(V, cur, nullptr, b, alt, co[0].mu, co[0].nu, co[0].c, 1, stop, st);
  for (int j = 2; j <= s; ++j) {
    // Y_{j-1} is in `alt` for even j (odd index), in `cur` for odd j; Y_j
    // overwrites Y_{j-2} in the other buffer
    T* yp = (j & 1) ? cur : alt;
    T* yw = (j & 1) ? alt : cur;
    launch_stage<T>(V, yp, yw, b, yw, co[j - 1].mu, co[j - 1].nu, co[j - 1].c, 0, stop, st);
  }
  check_launch();
  if (s & 1) std::swap(cur, alt);
}

// A tau-step of more stages than the fused kernel takes, as chunks of up to
// tau_chunk_max stages (App. A eq. RKL_intermediate_source; each chunk reads
// Y_{j-1}, Y_{j-2} and b and writes its last two stages).  Needs two
// scratch arrays x3, x4 besides cur and alt; on return cur holds the result
// and alt, x3, x4 the other three arrays (the same set of four).  False: the
// level has no chunk form (the caller runs stage by stage).
template <typename T>
bool tau_chunked(const LevelView<T>& V, T*& cur, T*& alt, T*& x3, T*& x4, const T* b,
                 const std::vector<StageCoef>& co, hipStream_t st) {
  const int K = tau_chunk_max<T>(V);
  const int s = (int)co.size();
  if (K < 2 || x3 == nullptr || x4 == nullptr || s <= FUSED_MAX_S) return false;
  T* bufs[4] = {cur, alt, x3, x4};
  T* a = cur;   // Y_{j-1}
  T* ap = cur;  // Y_{j-2} (the first stage's nu_1 = 0 term reads Y_0 itself)
  for (int j = 1; j <= s;) {
    const int S = std::min(K, s - j + 1);
    T* out = nullptr;
    T* out2 = nullptr;
    for (T* q : bufs) {
      if (q == a || q == ap) continue;
      if (!out) out = q;
      else if (!out2) out2 = q;
    }
    launch_tau_chunk<T>(V, a, ap, b, out, S >= 2 ? out2 : nullptr, S, co.data() + (j - 1), st);
    if (S >= 2) {
      a = out;
      ap = out2;
    } else {
      ap = a;
      a = out;
    }
    j += S;
  }
  check_launch();
  T* rest[3];
  int k = 0;
  for (T* q : bufs)
    if (q != a) rest[k++] = q;
  cur = a;
  alt = rest[0];
  x3 = rest[1];
  x4 = rest[2];
  return true;
}

// Two relaxations in one pass: on a two-dimensional level the strip kernel
// runs the 2s-stage recurrence of two tau-steps reading u and b once (there
// are no y-halo rows, so the extra stages cost little); 3-D levels keep one
// pass per tau-step, where the 2s-stage pass's halo rows make it slower.
template <typename T>
bool pair_ok(const LevelView<T>& V, int s, bool gs) {
  return !gs && level_is_2d(V) && fused_tau_supported<T>(V, 2 * s);
}

// n relaxations, paired where pair_ok allows
template <typename T>
void relax_n(Plan& P, const LevelView<T>& V, const Lev& Lv, int n, T*& cur, T*& alt, const T* b, const int* stop,
             hipStream_t st, const Batch& bt, bool gs);

// A tau-step whose input is the zero iterate (first relaxation of a coarse
// correction); the result lands in `cur` (its previous contents are ignored).
template <typename T>
void tau_from_zero(Plan& P, const LevelView<T>& V, T*& cur, T*& alt, const T* b,
                   const std::vector<StageCoef>& co, const int* stop, hipStream_t st,
                   const Batch& bt = single_batch(), bool gs = false) {
  const int s = (int)co.size();
  const bool fused = gs ? launch_gsrb_fused<T>(V, (const T*)nullptr, b, cur, 1.0, nullptr, stop, st, bt)
                        : launch_fused_tau<T>(V, (const T*)nullptr, b, cur, s, co.data(), nullptr, stop, st, bt);
  if (fused) {
    check_launch();
    return;
  }
  if (bt.nb > 1) fail(RKL_EINVAL, "batched solves need the fused smoother on every level above the tail");
  launch_fill<T>(cur, (size_t)V.nx * V.ny * V.nz, (T)0, stop, st);
  check_launch();
  tau_step<T>(P, V, cur, alt, b, co, stop, st, single_batch(), gs);
}

template <typename T>
void relax_n(Plan& P, const LevelView<T>& V, const Lev& Lv, int n, T*& cur, T*& alt, const T* b, const int* stop,
             hipStream_t st, const Batch& bt, bool gs) {
  const int s = (int)Lv.smooth.size();
  for (int q = 0; q < n;) {
    if (n - q >= 2 && pair_ok<T>(V, s, gs)) {
      tau_step<T>(P, V, cur, alt, b, Lv.smooth2, stop, st, bt, gs);
      q += 2;
    } else {
      tau_step<T>(P, V, cur, alt, b, Lv.smooth, stop, st, bt, gs);
      ++q;
    }
  }
}

// The first n_pre >= 1 relaxations of a coarse correction from the zero
// iterate (one or two of them fused into the first pass); returns how many ran
template <typename T>
int relax_from_zero(Plan& P, const LevelView<T>& V, const Lev& Lv, int n_pre, T*& cur, T*& alt, const T* b,
                    const int* stop, hipStream_t st, const Batch& bt, bool gs) {
  const bool pair = n_pre >= 2 && pair_ok<T>(V, (int)Lv.smooth.size(), gs);
  tau_from_zero<T>(P, V, cur, alt, b, pair ? Lv.smooth2 : Lv.smooth, stop, st, bt, gs);
  return pair ? 2 : 1;
}

// n >= 0 relaxations of a level before its residual is restricted to the
// next one: with `fuse` the last of them also writes that level's right-hand
// side bc = R(b - M u) and its partial pairs (Sec. 2.1 steps 1-2b in one
// pass over the level) where the level's strip kernel has the form.
// Returns the pairs written, 0 when the caller restricts separately.
template <typename T>
int relax_restrict(Plan& P, const LevelView<T>& V, const Lev& Lv, int n, T*& cur, T*& alt, const T* b, T* bc,
                   double* part, const int* stop, hipStream_t st, const Batch& b1, const Batch& b2, bool gs,
                   bool fuse) {
  if (n >= 1 && fuse && !gs && !level_is_2d(V)) {
    relax_n<T>(P, V, Lv, n - 1, cur, alt, b, stop, st, b1, gs);
    const int nb = launch_fused_tau_rs<T>(V, cur, b, alt, bc, (int)Lv.smooth.size(), Lv.smooth.data(), part, stop, st,
                                          b2);
    if (nb > 0) {
      check_launch();
      std::swap(cur, alt);
      return nb;
    }
    relax_n<T>(P, V, Lv, 1, cur, alt, b, stop, st, b1, gs);
    return 0;
  }
  relax_n<T>(P, V, Lv, n, cur, alt, b, stop, st, b1, gs);
  return 0;
}

// A tau-step from `a` that never writes `a`: the result lands in x or y and
// is returned in `cur`, the other in `alt`.  With `part` the fused kernel
// also writes the partial sums of (M a - b)^2.
template <typename T>
bool tau_keep(Plan& P, const LevelView<T>& V, T* a, T* x, T* y, T*& cur, T*& alt, const T* b,
              const std::vector<StageCoef>& co, double* part, const int* stop, hipStream_t st, bool gs = false,
              const Batch& bt = single_batch()) {
  if (gs) {
    if (launch_gsrb_fused<T>(V, a, b, x, 1.0, part, stop, st, bt)) {
      check_launch();
      cur = x;
      alt = y;
      return true;
    }
    if (bt.nb > 1) fail(RKL_EINVAL, "batched solves need the fused smoother on level 0");
    launch_gsrb_half<T>(V, a, x, b, 0, 1.0, stop, st);
    launch_gsrb_half<T>(V, x, y, b, 1, 1.0, stop, st);
    check_launch();
    cur = y;
    alt = x;
    return false;
  }
  const int s = (int)co.size();
  if (launch_fused_tau<T>(V, a, b, x, s, co.data(), part, stop, st, bt)) {
    check_launch();
    cur = x;
    alt = y;
    return true;
  }
  if (bt.nb > 1) fail(RKL_EINVAL, "batched solves need the fused smoother on level 0");
  if (a == nullptr) fail(RKL_EHIP, "a relaxation from the zero iterate needs the fused tau-step");
  // stage 1: a -> x; stage j >= 2 writes over Y_{j-2}, except that Y_0 = a
  // is never overwritten (stage 2 writes y)
  launch_stage<T>(V, a, nullptr, b, x, co[0].mu, co[0].nu, co[0].c, 1, stop, st);
  T* yjm1 = x;  // Y_{j-1}
  T* yjm2 = a;  // Y_{j-2}
  for (int j = 2; j <= s; ++j) {
    T* w = (j == 2) ? y : yjm2;
    launch_stage<T>(V, yjm1, yjm2, b, w, co[j - 1].mu, co[j - 1].nu, co[j - 1].c, 0, stop, st);
    yjm2 = yjm1;
    yjm1 = w;
  }
  check_launch();
  cur = yjm1;
  alt = (cur == x) ? y : x;
  return false;
}

// Accelerated RKL iteration driven from the host (levels too large for the
// one-workgroup kernel): residual read back before every tau-step.
template <typename T>
int accel_multi(Plan& P, const LevelView<T>& V, T*& cur, T*& alt, const T* b, double tol, double ref,
                int max_steps, bool rm_mean, hipStream_t st, double* res_out, T* x3 = nullptr, T* x4 = nullptr) {
  int step = 0;
  double res = 0.0;
  const size_t n = (size_t)V.nx * V.ny * V.nz;
  while (true) {
    res = resid_norm<T>(P, V, cur, b, st);
    if (res <= tol * ref || step >= max_steps) break;
    const int q = std::min(step, (int)P.sched.size() - 1);
    if (!(x3 && x4 && tau_chunked<T>(V, cur, alt, x3, x4, b, P.sched_coef[q], st)))
      tau_step<T>(P, V, cur, alt, b, P.sched_coef[q], nullptr, st);
    if (rm_mean) remove_mean<T>(P, cur, n, nullptr, st);
    ++step;
  }
  if (res_out) *res_out = res;
  return step;
}

template <typename T>
double coarse_tol_for(const rkl_opts& o) {
  if (o.coarse_tol > 0.0) return o.coarse_tol;
  return sizeof(T) == 8 ? 1e-13 : 1e-6;
}

// coarsest level l: M u_l = b_l from u_l = 0
template <typename T>
void coarse_solve(Plan& P, Hier<T>& H, int l, const rkl_opts& o, const int* stop, hipStream_t st) {
  const Lev& C = P.lv[l];
  const LevelView<T> V = view<T>(C, P.periodic, nullptr);
  const double tol = coarse_tol_for<T>(o);
  if (coarse_in_lds(P, C)) {
    launch_coarse_solve<T>(V, H.b[l], nullptr, H.u[l], P.cs(), tol, 0.0, o.coarse_max_steps,
                           P.periodic ? 1 : 0, P.dsteps, nullptr, stop, st);
    check_launch();
    return;
  }
  if (stop != nullptr) {
    // inside the device-side loop: skip once it has decided to stop
    int flag = 0;
    HIPCHK(hipMemcpyAsync(P.hscal, stop, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::memcpy(&flag, P.hscal, sizeof(int));
    if (flag) return;
  }
  launch_fill<T>(H.u[l], C.n, (T)0, nullptr, st);
  const double bn = resid_norm<T>(P, V, (const T*)nullptr, H.b[l], st);
  if (bn == 0.0) return;
  accel_multi<T>(P, V, H.u[l], H.t[l], H.b[l], tol, bn, o.coarse_max_steps, P.periodic, st, nullptr);
}

// The V-cycle of Sec. 2.1 on M_0 u = b0 below the first level-0 relaxation.
// On entry cur0 holds the iterate after `pre_done` level-0 relaxations
// (alt0 is its alternate buffer); on exit cur0 holds the cycle's result.
// faces0: level-0 Dirichlet data (float64 path only) or nullptr.
template <typename T>
int tail_level(const Plan& P) {
  return sizeof(T) == 8 ? P.tail64 : P.tail32;
}

// Batch geometry of the V-cycle: nb members whose level-l arrays are nb
// contiguous blocks of n_l cells; stop flags and partial sums strided per
// member; dsum: two doubles per member of scratch for periodic means.
struct VBatch {
  int nb = 1;
  int stop_stride = 0;
  int part_stride = 0;
  double* dsum = nullptr;
  double* part = nullptr;  // nullptr: the plan's own buffer
};

template <typename T>
void vcycle_from(Plan& P, Hier<T>& H, T*& cur0, T*& alt0, const T* b0, const double* faces0, int pre_done,
                 const rkl_opts& o, const int* stop, hipStream_t st, const VBatch& vb) {
  const int L = P.L();
  double* part = vb.part ? vb.part : P.part;
  auto V = [&](int l) { return view<T>(P.lv[l], P.periodic, l == 0 ? faces0 : nullptr); };
  auto B1 = [&](int l) { return Batch{vb.nb, (long long)P.lv[l].n, 0, vb.stop_stride, vb.part_stride}; };
  auto B2 = [&](int l, int l2) {
    return Batch{vb.nb, (long long)P.lv[l].n, (long long)P.lv[l2].n, vb.stop_stride, vb.part_stride};
  };
  const bool gs = o.smoother == RKL_SMOOTH_GSRB;
  if (L == 1) {
    if (vb.nb > 1) fail(RKL_EINVAL, "batched solves need at least two levels");
    for (int q = pre_done; q < o.n_pre + o.n_post; ++q)
      tau_step<T>(P, V(0), cur0, alt0, b0, P.lv[0].smooth, stop, st, single_batch(), gs);
    return;
  }
  // levels lt.. run in the one-workgroup tail when they fit
  const int lt = tail_level<T>(P);
  if (vb.nb > 1 && lt <= 0) fail(RKL_EINVAL, "batched solves need the one-workgroup coarse tail");
  const int lbot = lt > 0 ? lt : L - 1;
  const bool fuse_rs = (o.fuse & 2) != 0;
  // pairs of partial sums the fused restriction into the next level wrote (0: restrict separately)
  int rs_pairs = relax_restrict<T>(P, V(0), P.lv[0], std::max(0, o.n_pre - pre_done), cur0, alt0, b0, H.b[1], part,
                                   stop, st, B1(0), B2(0, 1), gs, fuse_rs);
  for (int l = 1; l <= lbot; ++l) {
    T* fu = (l == 1) ? cur0 : H.u[l - 1];
    const T* fb = (l == 1) ? b0 : H.b[l - 1];
    const Lev& Fl = P.lv[l - 1];
    int pairs = rs_pairs;
    if (pairs == 0) {
      launch_resid_restrict<T>(V(l - 1), fu, fb, H.b[l], part, stop, st, B2(l - 1, l));
      check_launch();
      pairs = (int)resid_blocks(Fl.nx, Fl.ny, Fl.nz);
    }
    rs_pairs = 0;
    const Lev& C = P.lv[l];
    if (l == lt) {
      const TailShape ts = tail_shape(P, lt);
      const StageCoef* sm[TAIL_MAX_LEVELS];
      for (int k = 0; k < ts.nlev; ++k) sm[k] = P.lv[lt + k].smooth.data();
      launch_tail<T>(ts, sm, o.s, o.n_pre, o.n_post, P.periodic ? 1 : 0, P.cs(), coarse_tol_for<T>(o),
                     o.coarse_max_steps, H.b[lt], H.u[lt], stop, st, B1(lt), gs ? 1 : 0);
      check_launch();
      break;
    }
    if (P.periodic) {  // coarse right-hand side made mean-free (its sum: the restriction's partials)
      Batch bs{vb.nb, (long long)C.n, 0, vb.stop_stride, vb.part_stride};
      launch_sub_mean_part<T>(H.b[l], C.n, part, pairs, 2, 1, (double)C.n, stop, st, bs);
      check_launch();
    }
    if (l < L - 1) {  // then l + 1 <= lbot: the loop restricts this level next
      if (o.n_pre > 0) {
        const int done = relax_from_zero<T>(P, V(l), C, o.n_pre, H.u[l], H.t[l], H.b[l], stop, st, B1(l), gs);
        rs_pairs = relax_restrict<T>(P, V(l), C, o.n_pre - done, H.u[l], H.t[l], H.b[l], H.b[l + 1], part, stop, st,
                                     B1(l), B2(l, l + 1), gs, fuse_rs);
      } else {
        launch_fill<T>(H.u[l], C.n, (T)0, stop, st, B1(l));
      }
    } else {
      if (vb.nb > 1) fail(RKL_EINVAL, "batched solves need the one-workgroup coarse tail");
      coarse_solve<T>(P, H, l, o, stop, st);
    }
  }
  for (int l = lbot - 1; l >= 0; --l) {
    T*& cu = (l == 0) ? cur0 : H.u[l];
    T*& ca = (l == 0) ? alt0 : H.t[l];
    const T* bl = (l == 0) ? b0 : H.b[l];
    const Lev& F = P.lv[l];
    // prolongation + correction (Sec. 2.1 steps 4-5) fused into the first
    // post-smoothing tau-step where the level's strip kernel allows it
    if (o.n_post > 0 && !gs && (o.fuse & 1) &&
        launch_fused_tau_pro<T>(V(l), cu, H.u[l + 1], bl, ca, (int)F.smooth.size(), F.smooth.data(), stop, st,
                                B2(l, l + 1))) {
      check_launch();
      std::swap(cu, ca);
      if (o.n_post > 1) relax_n<T>(P, V(l), F, o.n_post - 1, cu, ca, bl, stop, st, B1(l), gs);
      continue;
    }
    launch_prolong_add<T>(F.nx, F.ny, F.nz, P.periodic ? 1 : 0, H.u[l + 1], cu, stop, st, B2(l, l + 1));
    check_launch();
    if (o.n_post > 0) relax_n<T>(P, V(l), F, o.n_post, cu, ca, bl, stop, st, B1(l), gs);
  }
}
void fold_faces(Plan& P, const double* faces, const double* src, double* dst, hipStream_t st);
void prepare_source(Plan& P, const double* rho, double c, hipStream_t st);
void copy_d2d(double* dst, const double* src, size_t n, hipStream_t st);
void record(rkl_stats* stats, double rel);
void conv_reset(Plan& P, hipStream_t st);
const ConvState& conv_read(Plan& P, hipStream_t st);
int predict_batch(const ConvState& cs, double tol, int queued, int max_cycles);
void fill_stats(rkl_stats* stats, const ConvState& cs, int result_m);

rkl_opts resolve_opts(const rkl_opts* in);
bool solve_start(Plan& P, const rkl_opts& o, const double* rho, const double* faces, double* phi,
                 rkl_stats* stats, hipStream_t st, double& res0, rkl_status& status);

// res0^2 kept on the device for the convergence test; the check kernel takes sqrt
struct Res0Sqrt {
  static const double* ptr(Plan& P) { return P.dscal + RES0SQ_SLOT; }
};
rkl_status finish_status(const ConvState& cs);
rkl_status solve_fp64(Plan& P, const rkl_opts& o, const double* rho, const double* faces, double* phi,
                      rkl_stats* stats, hipStream_t st);
rkl_status solve_mixed(Plan& P, const rkl_opts& o, const double* rho, const double* faces, double* phi,
                       rkl_stats* stats, hipStream_t st);
int auto_s(const rkl_grid& g, int prec);
rkl_opts with_s(rkl_opts o, const rkl_grid& g);
rkl_status solve_one(const rkl_grid& g, const rkl_opts& o, const double* rho, const double* faces, double* phi,
                     rkl_stats* stats, hipStream_t st);

// drop the batched-solve classes and the captured graph (rkl_release_all)
void release_batched();

// guards the plan cache and the batched-solve classes (plan.hip)
extern std::mutex g_plans_mu;
// stage counts recorded per grid for Options.s = 0 (plan.hip): (nx, ny, nz, bc, prec) -> s
extern std::mutex g_s_mu;
extern std::map<std::tuple<int, int, int, int, int>, int> g_auto_s;

}  // namespace rkl
