// Host side of the RKL-multigrid Poisson solver: plan cache, level hierarchy,
// V-cycle driver, convergence loop, mixed-precision defect correction and the
// C ABI declared in include/rkl_poisson.h.
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

#include "../../include/rkl_poisson.h"
#include "host_common.h"
#include "kernels.h"

namespace rkl {

thread_local std::string g_err = "no error";

[[noreturn]] void fail(rkl_status st, const std::string& msg) {
  g_err = msg;
  throw Fail{st};
}

bool flat_grid(const rkl_grid& g) { return g.nz == 1 && std::isinf(g.hz) && g.hz > 0.0; }

void validate_grid(const rkl_grid* g, const double* bc_faces) {
  if (!g) fail(RKL_EINVAL, "grid is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) fail(RKL_EINVAL, "cell counts must be >= 1");
  if ((double)g->nx * g->ny * g->nz > 4.0e10) fail(RKL_EINVAL, "grid too large");
  if (!(g->hx > 0.0 && g->hy > 0.0 && g->hz > 0.0) || !std::isfinite(g->hx) || !std::isfinite(g->hy))
    fail(RKL_EINVAL, "spacings must be positive and finite");
  if (!std::isfinite(g->hz) && g->nz != 1)
    fail(RKL_EINVAL, "hz = inf (a two-dimensional grid) needs nz = 1");
  if (g->bc != RKL_BC_DIRICHLET && g->bc != RKL_BC_PERIODIC) fail(RKL_EINVAL, "unknown boundary type");
  if (g->bc == RKL_BC_PERIODIC && bc_faces) fail(RKL_EINVAL, "bc_faces must be NULL for periodic grids");
}

namespace {

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

// Stage coefficients of one s-stage tau-step: mu_j = (2j-1)/j, nu_j = (1-j)/j,
// c_j = mu~_j tau = (mu_j w1) tau, w1 = 2/(s^2+s), tau = theta tau_max(s).
std::vector<StageCoef> stage_coefs(int s, double theta, double dtpar) {
  const double w1 = 2.0 / (double)(s * s + s);
  const double tau = theta * dtpar * (double)(s * s + s) / 2.0;
  std::vector<StageCoef> out;
  for (int j = 1; j <= s; ++j) {
    const double mu = (2.0 * j - 1.0) / j;
    const double nu = (1.0 - j) / j;
    out.push_back({mu, nu, (mu * w1) * tau});
  }
  return out;
}

// Accelerated schedule on a level: k from n/2 down to 1 (n = smallest cell
// count), s_k = Round(2.4048 / arccos(x_k) - 1/2), x_k = 1 - theta dt_par
// |lambda_k|, repeats skipped.  |lambda_k|: Dirichlet diagonal mode
// sum_d 4 sin^2(k pi / 2 n_d) / h_d^2; periodic axis mode min_d 4 sin^2(k pi / n_d) / h_d^2.
// A two-dimensional level has no z modes: d runs over x and y only.
std::vector<int> accel_schedule(const Lev& L, bool periodic, double theta) {
  const int ns[3] = {L.nx, L.ny, L.nz};
  const double hs[3] = {L.hx, L.hy, L.hz};
  const int nd = L.flat ? 2 : 3;
  const int n = L.flat ? std::min(L.nx, L.ny) : std::min(L.nx, std::min(L.ny, L.nz));
  int k = std::max(1, n / 2);
  int s_old = 0;
  std::vector<int> out;
  while (true) {
    double lk = periodic ? 1e300 : 0.0;
    for (int d = 0; d < nd; ++d) {
      if (periodic) {
        const double sv = std::sin(k * M_PI / ns[d]);
        lk = std::min(lk, 4.0 * sv * sv / (hs[d] * hs[d]));
      } else {
        const double sv = std::sin(k * M_PI / (2.0 * ns[d]));
        lk += 4.0 * sv * sv / (hs[d] * hs[d]);
      }
    }
    double x = 1.0 - theta * L.dtpar * lk;
    x = std::max(-1.0, std::min(1.0, x));
    const double th = std::acos(x);
    int s;
    if (th <= 0.0) s = 1 << 20;
    else s = std::max(1, (int)std::floor(2.4048 / th - 0.5 + 0.5));
    if (s > 4096) s = 4096;  // a flat mode (x = 1) cannot be damped; keep tables bounded
    if (s != s_old) {
      out.push_back(s);
      s_old = s;
    }
    if (k == 1) break;
    --k;
  }
  return out;
}

// Best fixed stage count of App. A.3 (eq. sopt_theory) on a level at
// tau = theta tau_max: mode k of the smoothest family (as in accel_schedule)
// enters the stage polynomial at x_k = 1 - theta dt_par |lambda_k|; the
// spectral radius over the first kmax modes is rho(s) = max_k |P_s(x_k)|
// (eq. spectral_rad_RKL), the iteration count for d digits m = d / -log10
// rho (eq. iteration), and s_opt minimises m_eff = s m over 1 <= s <= the
// largest cell count.  P_s by the three-term recursion (eq. LP_recursion),
// advanced one s at a time for every mode.
int s_opt_rule(const Lev& L, bool periodic, double theta, int kmax, double digits, double* m_out) {
  const int ns[3] = {L.nx, L.ny, L.nz};
  const double hs[3] = {L.hx, L.hy, L.hz};
  const int nd = L.flat ? 2 : 3;
  int nmin = ns[0], nmax = ns[0];
  for (int d = 1; d < nd; ++d) {
    nmin = std::min(nmin, ns[d]);
    nmax = std::max(nmax, ns[d]);
  }
  const int K = std::max(1, std::min(kmax, nmin / 2));
  std::vector<double> x(K), p0(K, 1.0), p1(K);
  for (int k = 1; k <= K; ++k) {
    double lk = periodic ? 1e300 : 0.0;
    for (int d = 0; d < nd; ++d) {
      if (periodic) {
        const double sv = std::sin(k * M_PI / ns[d]);
        lk = std::min(lk, 4.0 * sv * sv / (hs[d] * hs[d]));
      } else {
        const double sv = std::sin(k * M_PI / (2.0 * ns[d]));
        lk += 4.0 * sv * sv / (hs[d] * hs[d]);
      }
    }
    x[k - 1] = 1.0 - theta * L.dtpar * lk;
    p1[k - 1] = x[k - 1];  // P_1
  }
  int best_s = 1;
  double best = HUGE_VAL;
  for (int s = 1; s <= nmax; ++s) {
    if (s >= 2) {  // P_s = ((2s-1) x P_{s-1} - (s-1) P_{s-2}) / s
      for (int k = 0; k < K; ++k) {
        const double pn = ((2.0 * s - 1.0) / s) * x[k] * p1[k] - ((s - 1.0) / s) * p0[k];
        p0[k] = p1[k];
        p1[k] = pn;
      }
    }
    double rho = 0.0;
    for (int k = 0; k < K; ++k) rho = std::max(rho, std::fabs(p1[k]));
    double m;
    if (rho <= 0.0) m = 0.0;
    else if (rho >= 1.0) m = HUGE_VAL;
    else m = s * digits / -std::log10(rho);
    if (m < best) {
      best = m;
      best_s = s;
    }
  }
  if (m_out) *m_out = best;
  return best_s;
}

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

std::mutex g_plans_mu;
std::map<PlanKey, std::unique_ptr<Plan>> g_plans;

// Levels from finest to coarsest: halve every axis (x and y only for a
// two-dimensional grid) while each halved count is even and >= min_coarse.
std::vector<Lev> build_levels(const rkl_grid& g, int min_coarse, int s, double theta) {
  std::vector<Lev> lv;
  int n[3] = {g.nx, g.ny, g.nz};
  double h[3] = {g.hx, g.hy, g.hz};
  const bool flat = flat_grid(g);
  const int nd = flat ? 2 : 3;
  while (true) {
    Lev L;
    L.nx = n[0];
    L.ny = n[1];
    L.nz = n[2];
    L.hx = h[0];
    L.hy = h[1];
    L.hz = h[2];
    L.flat = flat;
    L.n = (size_t)n[0] * n[1] * n[2];
    L.lam = 4.0 * (1.0 / (h[0] * h[0]) + 1.0 / (h[1] * h[1]) + 1.0 / (h[2] * h[2]));
    L.dtpar = 2.0 / L.lam;
    L.smooth = stage_coefs(s, theta, L.dtpar);
    // the second tau-step's first stage is the recurrence with mu = 1, nu = 0,
    // and its second stage's Y_{j-2} is the first step's result: two steps
    // are the 2s-stage recurrence with the coefficient list repeated
    L.smooth2 = L.smooth;
    L.smooth2.insert(L.smooth2.end(), L.smooth.begin(), L.smooth.end());
    lv.push_back(L);
    bool ok = true;
    for (int d = 0; d < nd; ++d)
      ok = ok && (n[d] % 2 == 0) && ((n[d] / 2) % 2 == 0) && (n[d] / 2 >= min_coarse);
    if (!ok) break;
    for (int d = 0; d < nd; ++d) {
      n[d] /= 2;
      h[d] *= 2.0;
    }
  }
  return lv;
}

bool coarse_in_lds(const Plan& P, const Lev& C);

TailShape tail_shape(const Plan& P, int lt) {
  TailShape ts;
  std::memset(&ts, 0, sizeof(ts));
  ts.nlev = P.L() - lt;
  if (ts.nlev > TAIL_MAX_LEVELS) {
    ts.nlev = TAIL_MAX_LEVELS + 1;  // too deep: tail_fits rejects it
    return ts;
  }
  for (int l = lt; l < P.L(); ++l) {
    const Lev& V = P.lv[l];
    ts.nx[l - lt] = V.nx;
    ts.ny[l - lt] = V.ny;
    ts.nz[l - lt] = V.nz;
    ts.ihx2[l - lt] = 1.0 / (V.hx * V.hx);
    ts.ihy2[l - lt] = 1.0 / (V.hy * V.hy);
    ts.ihz2[l - lt] = 1.0 / (V.hz * V.hz);
  }
  return ts;
}

Plan& get_plan(const rkl_grid& g, int s, double theta, int min_coarse, int prec) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  PlanKey key{dev, g.nx, g.ny, g.nz, g.bc, s, min_coarse, prec, g.hx, g.hy, g.hz, theta};
  std::lock_guard<std::mutex> lk(g_plans_mu);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) return *it->second;
  auto P = std::make_unique<Plan>();
  P->key = key;
  P->periodic = g.bc == RKL_BC_PERIODIC;
  P->lv = build_levels(g, min_coarse, s, theta);
  const int L = P->L();
  P->f0 = P->alloc<double>(P->lv[0].n);
  P->t0 = P->alloc<double>(P->lv[0].n);
  P->t0b = P->alloc<double>(P->lv[0].n);
  P->h64.u.assign(L, nullptr);
  P->h64.b.assign(L, nullptr);
  P->h64.t.assign(L, nullptr);
  for (int l = 1; l < L; ++l) {
    P->h64.u[l] = P->alloc<double>(P->lv[l].n);
    P->h64.b[l] = P->alloc<double>(P->lv[l].n);
    P->h64.t[l] = P->alloc<double>(P->lv[l].n);
  }
  if (prec == RKL_MIXED) {
    P->h32.u.assign(L, nullptr);
    P->h32.b.assign(L, nullptr);
    P->h32.t.assign(L, nullptr);
    for (int l = 0; l < L; ++l) {
      P->h32.u[l] = P->alloc<float>(P->lv[l].n);
      P->h32.b[l] = P->alloc<float>(P->lv[l].n);
      P->h32.t[l] = P->alloc<float>(P->lv[l].n);
    }
  }
  // partial sums: residual kernels (pairs), fused tau-step (one per block), elementwise
  // sums (pairs for the source scaling)
  size_t cap = 2 * resid_blocks(g.nx, g.ny, g.nz);
  cap = std::max(cap, 2 * ew_block_count(P->lv[0].n));
  cap = std::max(cap, fused_tau_blocks_max(P->lv[0].nx, P->lv[0].ny, P->lv[0].nz));
  cap = std::max(cap, (size_t)1024);
  P->part = P->alloc<double>(cap);
  P->part_cap = cap;
  P->dscal = P->alloc<double>(16);
  P->dsteps = P->alloc<int>(4);
  P->dconv = P->alloc<ConvState>(1);
  HIPCHK(hipHostMalloc((void**)&P->hscal, 16 * sizeof(double), hipHostMallocDefault));
  HIPCHK(hipHostMalloc((void**)&P->hconv, sizeof(ConvState), hipHostMallocDefault));
  // coarsest schedule tables
  const Lev& C = P->lv[L - 1];
  P->sched = accel_schedule(C, P->periodic, theta);
  std::vector<int> coff;
  std::vector<double> coef;
  for (int s_q : P->sched) {
    coff.push_back((int)(coef.size() / 3));
    auto co = stage_coefs(s_q, theta, C.dtpar);
    P->sched_coef.push_back(co);
    for (auto& c : co) {
      coef.push_back(c.mu);
      coef.push_back(c.nu);
      coef.push_back(c.c);
    }
  }
  P->d_sched = P->alloc<int>(P->sched.size());
  P->d_coff = P->alloc<int>(coff.size());
  P->d_coef = P->alloc<double>(coef.size());
  HIPCHK(hipMemcpy(P->d_sched, P->sched.data(), P->sched.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(P->d_coff, coff.data(), coff.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(P->d_coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice));
  if (coarse_in_lds(*P, C) && L >= 3) {
    for (int lt = 1; lt < L - 1; ++lt) {
      const TailShape ts = tail_shape(*P, lt);
      if (P->tail64 < 0 && tail_fits<double>(ts, s)) P->tail64 = lt;
      if (P->tail32 < 0 && tail_fits<float>(ts, s)) P->tail32 = lt;
    }
  }
  Plan& ref = *P;
  g_plans[key] = std::move(P);
  return ref;
}

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

// the coarsest level fits the one-workgroup LDS solver
bool coarse_in_lds(const Plan& P, const Lev& C) {
  size_t rows = 0;
  for (int s : P.sched) rows += (size_t)s;
  return C.n <= (size_t)COARSE_MAX_CELLS && P.sched.size() <= (size_t)COARSE_MAX_SCHED &&
         rows <= (size_t)COARSE_MAX_COEF;
}

// read `nq` device scalars (synchronises the stream)
const double* readback(Plan& P, int nq, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(P.hscal, P.dscal, nq * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return P.hscal;
}

// ||b - M u||^2 into P.dscal[0] (u may be nullptr), not synchronising
template <typename T>
void resid_norm2_async(Plan& P, const LevelView<T>& V, const T* u, const T* b, hipStream_t st) {
  launch_residual<T, T>(V, u, b, (T*)nullptr, P.part, nullptr, st);
  check_launch();
  launch_reduce(P.part, (int)resid_blocks(V.nx, V.ny, V.nz), 2, 1, P.dscal, nullptr, st);
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
  if (pre_done < o.n_pre) relax_n<T>(P, V(0), P.lv[0], o.n_pre - pre_done, cur0, alt0, b0, stop, st, B1(0), gs);
  for (int l = 1; l <= lbot; ++l) {
    T* fu = (l == 1) ? cur0 : H.u[l - 1];
    const T* fb = (l == 1) ? b0 : H.b[l - 1];
    launch_resid_restrict<T>(V(l - 1), fu, fb, H.b[l], part, stop, st, B2(l - 1, l));
    check_launch();
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
      const Lev& Fl = P.lv[l - 1];
      Batch bs{vb.nb, (long long)C.n, 0, vb.stop_stride, vb.part_stride};
      launch_sub_mean_part<T>(H.b[l], C.n, part, (int)resid_blocks(Fl.nx, Fl.ny, Fl.nz), 2, 1, (double)C.n, stop, st,
                              bs);
      check_launch();
    }
    if (l < L - 1) {
      if (o.n_pre > 0) {
        const int done = relax_from_zero<T>(P, V(l), C, o.n_pre, H.u[l], H.t[l], H.b[l], stop, st, B1(l), gs);
        if (done < o.n_pre) relax_n<T>(P, V(l), C, o.n_pre - done, H.u[l], H.t[l], H.b[l], stop, st, B1(l), gs);
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
    if (o.n_post > 0 && !gs && o.fuse &&
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
void conv_reset(Plan& P, hipStream_t st) {
  std::memset(P.hconv, 0, sizeof(ConvState));
  HIPCHK(hipMemcpyAsync(P.dconv, P.hconv, offsetof(ConvState, hist), hipMemcpyHostToDevice, st));
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

// ------------------------------------------------------------------ validation
rkl_opts resolve_opts(const rkl_opts* in) {
  rkl_opts o;
  rkl_default_opts(&o);
  if (in) o = *in;
  if (o.s < 0 || o.s > 64) fail(RKL_EINVAL, "s must be in [0, 64] (0: tuned or default)");
  if (!(o.tau_frac > 0.0 && o.tau_frac < 2.0)) fail(RKL_EINVAL, "tau_frac must be in (0, 2)");
  if (o.n_pre < 0 || o.n_post < 0 || o.n_pre + o.n_post < 1) fail(RKL_EINVAL, "need n_pre + n_post >= 1");
  if (o.min_coarse < 2) fail(RKL_EINVAL, "min_coarse must be >= 2");
  if (!(o.tol >= 0.0) || !std::isfinite(o.tol)) fail(RKL_EINVAL, "tol must be finite and >= 0");
  if (o.max_cycles < 0) fail(RKL_EINVAL, "max_cycles must be >= 0");
  if (o.prec != RKL_FP64 && o.prec != RKL_MIXED) fail(RKL_EINVAL, "unknown precision");
  if (!std::isfinite(o.four_pi_G)) fail(RKL_EINVAL, "four_pi_G must be finite");
  if (!(o.coarse_tol >= 0.0)) fail(RKL_EINVAL, "coarse_tol must be >= 0");
  if (o.coarse_max_steps < 0) fail(RKL_EINVAL, "coarse_max_steps must be >= 0");
  if (o.smoother != RKL_SMOOTH_RKL && o.smoother != RKL_SMOOTH_GSRB) fail(RKL_EINVAL, "unknown smoother");
  if (o.fuse != 0 && o.fuse != 1) fail(RKL_EINVAL, "fuse must be 0 or 1");
  return o;
}

// ------------------------------------------------------------------ solves
// Common start: f0, ||M 0 - f0||.  Returns false when the solve is already
// decided (zero right-hand side or non-finite data); `status` says how.
bool solve_start(Plan& P, const rkl_opts& o, const double* rho, const double* faces, double* phi,
                 rkl_stats* stats, hipStream_t st, double& res0, rkl_status& status) {
  const Lev& F = P.lv[0];
  const LevelView<double> V0 = view<double>(F, P.periodic, nullptr);
  prepare_source(P, rho, o.four_pi_G, st);
  if (faces != nullptr) {
    fold_faces(P, faces, P.f0, P.f0, st);
    resid_norm2_async<double>(P, V0, nullptr, P.f0, st);
  } else {  // ||M 0 - f0||^2 is the sum of f0^2: the scaling pass's partials
    launch_reduce(P.part + 1, (int)ew_block_count(F.n), 2, 1, P.dscal, nullptr, st);
    check_launch();
  }
  HIPCHK(hipMemcpyAsync(P.dscal + 4, P.dscal, sizeof(double), hipMemcpyDeviceToDevice, st));  // res0^2
  res0 = std::sqrt(readback(P, 1, st)[0]);
  if (stats) {
    stats->res0 = res0;
    stats->levels = P.L();
    stats->cycles = 0;
    stats->rel_res = 0.0;
  }
  status = RKL_OK;
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

// res0^2 kept on the device for the convergence test; the check kernel takes sqrt
struct Res0Sqrt {
  static const double* ptr(Plan& P) { return P.dscal + 5; }
};

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
  if (!solve_start(P, o, rho, faces, phi, stats, st, res0, status)) return status;

  if (P.L() == 1) {
    // single level: accelerated RKL iteration (App. A.4, App. B) to tol
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
  HIPCHK(hipMemcpyAsync(P.dscal + 5, P.dscal + 4, sizeof(double), hipMemcpyDeviceToDevice, st));
  conv_reset(P, st);
  const int* stop = &P.dconv->stop;
  const bool gs = o.smoother == RKL_SMOOTH_GSRB;
  const bool fused0 = fused_tau_supported<double>(V0, gs ? 2 : o.s) && o.n_pre > 0;
  const bool pair0 = fused0 && o.n_pre >= 2 && pair_ok<double>(V0, o.s, gs);
  int queued = 0;
  ConvState cs = conv_read(P, st);
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
        tau_keep<double>(P, V0, a, bufs[ib], bufs[ic], cur, alt, P.f0, pair0 ? F.smooth2 : F.smooth, P.part, stop,
                         st, gs);
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
  const int rm = cs.result_m;
  double* res = bufs[start[rm]];
  if (P.periodic && res != phi) {  // phi = res - mean(res): the copy carries the mean removal
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
  if (!solve_start(P, o, rho, faces, phi, stats, st, res0, status)) return status;
  HIPCHK(hipMemcpyAsync(P.dscal + 5, P.dscal + 4, sizeof(double), hipMemcpyDeviceToDevice, st));
  conv_reset(P, st);
  const int* stop = &P.dconv->stop;
  const int nblk = (int)resid_blocks(F.nx, F.ny, F.nz);
  int queued = 0;
  ConvState cs = conv_read(P, st);
  while (true) {
    const int batch = predict_batch(cs, o.tol, queued, o.max_cycles);
    for (int q = 0; q < batch; ++q) {
      // float64 defect r = f - M phi, stored as the float32 right-hand side
      launch_residual<double, float>(V0, phi, P.f0, P.h32.b[0], P.part, stop, st);
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
      launch_add_cast<float>(phi, cur, F.n, stop, st);
      check_launch();
      ++queued;
    }
    cs = conv_read(P, st);
    if (cs.stop) break;
    if (queued > o.max_cycles) fail(RKL_EHIP, "refinement loop ended without a decision");
  }
  if (P.periodic) remove_mean<double>(P, phi, F.n, nullptr, st);
  HIPCHK(hipStreamSynchronize(st));
  fill_stats(stats, cs, cs.result_m);
  return finish_status(cs);
}


// s = 0 in the options asks for the stage count recorded for the grid (a
// timed choice made by the tuner), else the default s = 2.
std::mutex g_s_mu;
std::map<std::tuple<int, int, int, int, int>, int> g_auto_s;  // (nx, ny, nz, bc, prec) -> s

int auto_s(const rkl_grid& g, int prec) {
  std::lock_guard<std::mutex> lk(g_s_mu);
  auto it = g_auto_s.find(std::make_tuple(g.nx, g.ny, g.nz, (int)g.bc, prec));
  return it == g_auto_s.end() ? 2 : it->second;
}

rkl_opts with_s(rkl_opts o, const rkl_grid& g) {
  if (o.s == 0) o.s = auto_s(g, o.prec);
  return o;
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

// ------------------------------------------------------------------ batched solves
// Members with identical grids form a class.  A class owns contiguous
// buffers (member m at m * n_l on level l) and every kernel of its V-cycle
// covers all members in one launch; each member has its own convergence state
// and stop flag, so converged members idle (their workgroups return at once)
// while the others go on.  The defect-correction form of the loop (float64
// residual, a V-cycle on the correction equation from zero at the inner
// precision, float64 update) serves both precisions.
struct ClassKey {
  int dev, nx, ny, nz, bc, s, min_coarse, prec, nb;
  int direct;  // float64 with n_pre > 0: iterate on phi itself (ClassPlan::direct)
  int fuse;    // transfer fusion (rkl_opts.fuse): which kernels the captured graph holds
  double hx, hy, hz, theta;
  bool operator<(const ClassKey& o) const {
    return std::tie(dev, nx, ny, nz, bc, s, min_coarse, prec, nb, direct, fuse, hx, hy, hz, theta) <
           std::tie(o.dev, o.nx, o.ny, o.nz, o.bc, o.s, o.min_coarse, o.prec, o.nb, o.direct, o.fuse, o.hx, o.hy,
                    o.hz, o.theta);
  }
};

struct ClassPlan {
  Plan* base = nullptr;  // level descriptors, schedule tables and tail choice of one member
  int nb = 0;
  int s = 2;             // stages per tau-step of this class
  int part_stride = 0;
  double *f0 = nullptr, *phi = nullptr, *res0sq = nullptr, *dsum = nullptr, *part = nullptr;
  double** tab_in = nullptr;
  double** tab_out = nullptr;
  ConvState* conv = nullptr;
  ConvState* hconv = nullptr;
  Hier<float> h32;
  Hier<double> h64;
  // float64 classes iterate on phi directly over the rotating level-0 buffers
  // {phi, h64.u[0], h64.t[0]}: cycle m starts from buffer rot[m % nrot]
  bool direct = false;
  int rot[3] = {0, 0, 0};
  int nrot = 1;
  std::vector<void*> allocs;
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
  ~ClassPlan() {
    for (void* p : allocs) (void)hipFree(p);
    if (hconv) (void)hipHostFree(hconv);
  }
};

std::map<ClassKey, std::unique_ptr<ClassPlan>> g_classes;

ClassPlan& get_class(const rkl_grid& g, const rkl_opts& o, int nb) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  const int direct = (o.prec == RKL_FP64 && o.n_pre > 0) ? 1 : 0;
  ClassKey key{dev, g.nx, g.ny, g.nz, g.bc, o.s, o.min_coarse, o.prec, nb, direct, o.fuse, g.hx, g.hy, g.hz, o.tau_frac};
  Plan& base = get_plan(g, o.s, o.tau_frac, o.min_coarse, o.prec);
  std::lock_guard<std::mutex> lk(g_plans_mu);
  auto it = g_classes.find(key);
  if (it != g_classes.end()) return *it->second;
  if (nb > 65535) fail(RKL_EINVAL, "at most 65535 members per grid class");
  auto C = std::make_unique<ClassPlan>();
  C->base = &base;
  C->nb = nb;
  const Lev& F = base.lv[0];
  const int L = base.L();
  size_t ps = 2 * resid_blocks(F.nx, F.ny, F.nz);
  ps = std::max(ps, 2 * ew_block_count(F.n));
  ps = std::max(ps, fused_tau_blocks_max(F.nx, F.ny, F.nz));
  C->part_stride = (int)ps;
  C->f0 = C->alloc<double>((size_t)nb * F.n);
  C->phi = C->alloc<double>((size_t)nb * F.n);
  C->res0sq = C->alloc<double>(nb);
  C->dsum = C->alloc<double>(2 * (size_t)nb);
  C->part = C->alloc<double>((size_t)nb * ps);
  C->tab_in = C->alloc<double*>(nb);
  C->tab_out = C->alloc<double*>(nb);
  C->conv = C->alloc<ConvState>(nb);
  HIPCHK(hipHostMalloc((void**)&C->hconv, (size_t)nb * sizeof(ConvState), hipHostMallocDefault));
  auto make = [&](auto& H, auto tag) {
    using U = decltype(tag);
    H.u.assign(L, nullptr);
    H.b.assign(L, nullptr);
    H.t.assign(L, nullptr);
    for (int l = 0; l < L; ++l) {
      H.u[l] = C->template alloc<U>((size_t)nb * base.lv[l].n);
      H.b[l] = C->template alloc<U>((size_t)nb * base.lv[l].n);
      H.t[l] = C->template alloc<U>((size_t)nb * base.lv[l].n);
    }
  };
  if (o.prec == RKL_MIXED) make(C->h32, 0.0f);
  else make(C->h64, 0.0);
  C->s = o.s;
  C->direct = direct != 0;
  ClassPlan& ref = *C;
  g_classes[key] = std::move(C);
  return ref;
}

constexpr int CONV_INTS = (int)(sizeof(ConvState) / sizeof(int));

// one outer iteration for every member of the class (stream-ordered, no sync)
template <typename T>
void class_iteration(ClassPlan& C, Hier<T>& H, const rkl_opts& o, hipStream_t st) {
  Plan& P = *C.base;
  const Lev& F = P.lv[0];
  const int nb = C.nb, ps = C.part_stride;
  const int* stop = &C.conv->stop;
  const LevelView<double> V0 = view<double>(F, P.periodic, nullptr);
  const LevelView<T> VT = view<T>(F, P.periodic, nullptr);
  launch_residual<double, T>(V0, C.phi, C.f0, H.b[0], C.part, stop, st, Batch{nb, (long long)F.n, 0, CONV_INTS, ps});
  launch_check(C.part, (int)resid_blocks(F.nx, F.ny, F.nz), 2, C.res0sq, o.tol, o.max_cycles, (double)F.n, C.conv,
               st, Batch{nb, 0, 0, 0, ps});
  check_launch();  // periodic: no level-0 mean pass (the defect is mean-free up to rounding; see solve_mixed)
  T* cur = H.u[0];
  T* alt = H.t[0];
  const Batch b0{nb, (long long)F.n, 0, CONV_INTS, ps};
  int pre_done = 0;
  if (o.n_pre > 0) {
    pre_done = relax_from_zero<T>(P, VT, F, o.n_pre, cur, alt, H.b[0], stop, st, b0, o.smoother == RKL_SMOOTH_GSRB);
  } else {
    launch_fill<T>(cur, F.n, (T)0, stop, st, b0);
  }
  vcycle_from<T>(P, H, cur, alt, H.b[0], nullptr, pre_done, o, stop, st, VBatch{nb, CONV_INTS, ps, C.dsum, C.part});
  launch_add_cast<T>(C.phi, cur, F.n, stop, st, Batch{nb, (long long)F.n, (long long)F.n, CONV_INTS, 0});
  check_launch();
}

// One float64 V-cycle on phi itself for every member, as in the single solve:
// the first relaxation from bufs[ia] (never written) carries the residual
// partials of its start state for the convergence test; ia becomes the buffer
// the cycle ends in.
void class_iteration_direct(ClassPlan& C, const rkl_opts& o, hipStream_t st, int& ia) {
  Plan& P = *C.base;
  Hier<double>& H = C.h64;
  const Lev& F = P.lv[0];
  const int nb = C.nb, ps = C.part_stride;
  const int* stop = &C.conv->stop;
  const LevelView<double> V0 = view<double>(F, P.periodic, nullptr);
  double* bufs[3] = {C.phi, H.u[0], H.t[0]};
  const bool gs = o.smoother == RKL_SMOOTH_GSRB;
  const bool pair0 = o.n_pre >= 2 && pair_ok<double>(V0, o.s, gs);
  const Batch b0{nb, (long long)F.n, 0, CONV_INTS, ps};
  double *cur = nullptr, *alt = nullptr;
  tau_keep<double>(P, V0, bufs[ia], bufs[(ia + 1) % 3], bufs[(ia + 2) % 3], cur, alt, C.f0,
                   pair0 ? F.smooth2 : F.smooth, C.part, stop, st, gs, b0);
  const int nblk = (int)(gs ? gsrb_blocks<double>(V0) : fused_tau_blocks<double>(V0, pair0 ? 2 * o.s : o.s));
  launch_check(C.part, nblk, 1, C.res0sq, o.tol, o.max_cycles, 1.0, C.conv, st, Batch{nb, 0, 0, 0, ps});
  check_launch();
  vcycle_from<double>(P, H, cur, alt, C.f0, nullptr, pair0 ? 2 : 1, o, stop, st,
                      VBatch{nb, CONV_INTS, ps, C.dsum, C.part});
  for (int k = 0; k < 3; ++k)
    if (bufs[k] == cur) ia = k;
}

// k outer iterations of a class; a direct (float64) class captures more if
// needed so that the buffer rotation ends where it started (graph replays
// then continue it), and records the rotation.  Returns the count captured.
int class_iterations(ClassPlan& C, rkl_opts o, int k, hipStream_t st) {
  o.s = C.s;
  if (C.direct) {
    std::vector<int> seq;
    int ia = 0;
    for (int q = 0; q < k || ia != 0; ++q) {
      if (q >= k + 3) fail(RKL_EHIP, "level-0 buffer rotation does not close");
      seq.push_back(ia);
      class_iteration_direct(C, o, st, ia);
    }
    int per = 1;  // period of the rotation within the captured sequence
    while (per < (int)seq.size() && seq[per] != 0) ++per;
    if (per > 3) fail(RKL_EHIP, "unexpected level-0 buffer rotation");
    C.nrot = per;
    for (int q = 0; q < 3; ++q) C.rot[q] = seq[q % per];
    return (int)seq.size();
  }
  for (int q = 0; q < k; ++q) {
    if (o.prec == RKL_MIXED) class_iteration<float>(C, C.h32, o, st);
    else class_iteration<double>(C, C.h64, o, st);
  }
  return k;
}

// Start of a class: f0 = 4 pi G rho (mean-free when periodic), phi = 0,
// ||M 0 - f0||^2 and a reset convergence state for every member.
// Enqueued part: the host arrays rho, phi and r0sq (nb doubles, receives
// ||M 0 - f0||^2 per member) must stay alive until the stream is synchronised.
void class_start_enqueue(ClassPlan& C, const rkl_opts& o, const double* const* rho, double* const* phi,
                         double* r0sq, hipStream_t st) {
  Plan& P = *C.base;
  const Lev& F = P.lv[0];
  const int nb = C.nb, ps = C.part_stride;
  HIPCHK(hipMemcpyAsync(C.tab_in, rho, nb * sizeof(double*), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(C.tab_out, phi, nb * sizeof(double*), hipMemcpyHostToDevice, st));
  // the single solve's arithmetic (prepare_source, solve_start), member by member
  const int nblk = (int)ew_block_count(F.n);
  const double* sum = nullptr;
  if (P.periodic) {
    launch_sum_tab(C.tab_in, F.n, C.part, st, Batch{nb, 0, 0, 0, ps});
    launch_reduce(C.part, nblk, 1, 1, C.dsum, nullptr, st, Batch{nb, 2, 0, 0, ps});
    sum = C.dsum;
  }
  launch_scale_tab(C.tab_in, C.f0, F.n, o.four_pi_G, sum, (double)F.n, C.part, st,
                   Batch{nb, (long long)F.n, 2, 0, ps});
  check_launch();
  // ||M 0 - f0||^2 = sum of f0^2 (no face data in batched solves)
  launch_reduce(C.part + 1, nblk, 2, 1, C.res0sq, nullptr, st, Batch{nb, 1, 0, 0, ps});
  launch_fill<double>(C.phi, F.n, 0.0, nullptr, st, Batch{nb, (long long)F.n, 0, 0, 0});
  check_launch();
  HIPCHK(hipMemcpyAsync(r0sq, C.res0sq, nb * sizeof(double), hipMemcpyDeviceToHost, st));
}

// After the synchronisation: ||M 0 - f0|| per member, and a reset convergence
// state.  A zero right-hand side is tested against 1 instead, which stops it
// at once with phi = 0.
std::vector<double> class_start_finish(ClassPlan& C, std::vector<double>& r0, hipStream_t st) {
  const int nb = C.nb;
  std::vector<double> res0(nb);
  bool fix = false;
  for (int m = 0; m < nb; ++m) {
    res0[m] = std::sqrt(r0[m]);
    if (r0[m] == 0.0) {
      r0[m] = 1.0;
      fix = true;
    }
  }
  if (fix) {
    HIPCHK(hipMemcpyAsync(C.res0sq, r0.data(), nb * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  std::memset(C.hconv, 0, (size_t)nb * sizeof(ConvState));
  HIPCHK(hipMemcpyAsync(C.conv, C.hconv, (size_t)nb * sizeof(ConvState), hipMemcpyHostToDevice, st));
  return res0;
}

// Member mb of a direct class: its answer is the start state of cycle
// result_m, rotation buffer rot[result_m % nrot]; when that is not phi, copy it
// into phi.
__global__ __launch_bounds__(256) void k_take_answer(double* __restrict__ phi, const double* __restrict__ b1,
                                                     const double* __restrict__ b2, size_t n,
                                                     const ConvState* __restrict__ conv, int r0, int r1, int r2,
                                                     int nrot, long long stride) {
  const long long mb = blockIdx.y;
  const int q = conv[mb].result_m % nrot;
  const int k = q == 0 ? r0 : (q == 1 ? r1 : r2);
  if (k == 0) return;
  const double* __restrict__ src = (k == 1 ? b1 : b2) + mb * stride;
  double* __restrict__ dst = phi + mb * stride;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

// answer into phi (direct classes), final mean removal (periodic) and
// copy-out to the caller's arrays
void class_finish(ClassPlan& C, hipStream_t st) {
  Plan& P = *C.base;
  const Lev& F = P.lv[0];
  const int nb = C.nb, ps = C.part_stride;
  if (C.direct) {
    const unsigned blocks = (unsigned)std::min<size_t>((F.n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_take_answer, dim3(blocks, nb), dim3(256), 0, st, C.phi, C.h64.u[0], C.h64.t[0], F.n,
                       C.conv, C.rot[0], C.rot[1], C.rot[2], C.nrot, (long long)F.n);
    check_launch();
  }
  if (P.periodic) {
    launch_sum<double>(C.phi, F.n, C.part, st, Batch{nb, (long long)F.n, 0, 0, ps});
    launch_reduce(C.part, (int)ew_block_count(F.n), 1, 1, C.dsum, nullptr, st, Batch{nb, 2, 0, 0, ps});
    launch_sub_mean<double>(C.phi, F.n, C.dsum, (double)F.n, nullptr, st, Batch{nb, (long long)F.n, 2, 0, 0});
  }
  launch_copy_tab(C.tab_out, C.phi, F.n, st, Batch{nb, (long long)F.n, 0, 0, 0});
  check_launch();
}

// options that the captured kernels take as arguments
struct LoopSig {
  std::vector<std::pair<ClassPlan*, int>> cls;  // classes and iterations captured
  double tol, coarse_tol;
  int max_cycles, n_pre, n_post, coarse_max_steps;
  int tune_gen;  // kernel variants are chosen at capture time
  int smoother, fuse;
  bool operator==(const LoopSig& o) const {
    return cls == o.cls && tol == o.tol && coarse_tol == o.coarse_tol && max_cycles == o.max_cycles &&
           n_pre == o.n_pre && n_post == o.n_post && coarse_max_steps == o.coarse_max_steps &&
           tune_gen == o.tune_gen && smoother == o.smoother && fuse == o.fuse;
  }
};

struct GraphCache {
  LoopSig sig;
  hipGraphExec_t exec = nullptr;
  hipStream_t stream = nullptr;
  std::vector<hipStream_t> branch;  // capture streams of classes 1.. (default priority)
  std::vector<hipEvent_t> events;   // fork event, then one join event per branch
  ~GraphCache() {
    if (exec) (void)hipGraphExecDestroy(exec);
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    for (hipStream_t b : branch) (void)hipStreamDestroy(b);
    if (stream) (void)hipStreamDestroy(stream);
  }
};
std::unique_ptr<GraphCache> g_graph;

// Capture `iters` outer iterations of every class into one graph (cached).
// Classes share no buffer, so each is a branch of its own (forked from and
// joined back into the capture stream by events): the latency-bound small
// levels and tails of one class overlap the other classes' sweeps.
hipGraphExec_t batch_graph(std::vector<ClassPlan*>& cls, const rkl_opts& o, int iters) {
  LoopSig sig{{}, o.tol, o.coarse_tol, o.max_cycles, o.n_pre, o.n_post, o.coarse_max_steps, tune_generation(),
              o.smoother, o.fuse};
  for (auto* c : cls) sig.cls.push_back({c, iters});
  if (g_graph && g_graph->sig == sig) return g_graph->exec;
  tail_prepare();
  auto G = std::make_unique<GraphCache>();
  G->sig = sig;
  HIPCHK(hipStreamCreateWithFlags(&G->stream, hipStreamNonBlocking));
  const size_t nc = cls.size();
  for (size_t c = 1; c < nc; ++c) {
    hipStream_t b = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&b, hipStreamNonBlocking));
    G->branch.push_back(b);
  }
  for (size_t e = 0; e < nc; ++e) {
    hipEvent_t ev = nullptr;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    G->events.push_back(ev);
  }
  HIPCHK(hipStreamBeginCapture(G->stream, hipStreamCaptureModeThreadLocal));
  HIPCHK(hipEventRecord(G->events[0], G->stream));  // fork
  for (size_t c = 1; c < nc; ++c) {
    HIPCHK(hipStreamWaitEvent(G->branch[c - 1], G->events[0], 0));
    class_iterations(*cls[c], o, iters, G->branch[c - 1]);
    HIPCHK(hipEventRecord(G->events[c], G->branch[c - 1]));
  }
  class_iterations(*cls[0], o, iters, G->stream);
  for (size_t c = 1; c < nc; ++c) HIPCHK(hipStreamWaitEvent(G->stream, G->events[c], 0));  // join
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamEndCapture(G->stream, &graph));
  HIPCHK(hipGraphInstantiate(&G->exec, graph, nullptr, nullptr, 0));
  (void)hipGraphDestroy(graph);
  g_graph = std::move(G);
  return g_graph->exec;
}

// A class runs batched when its hierarchy ends in the one-workgroup tail and
// every level above the tail takes the fused tau-step.
template <typename T>
bool class_ok(Plan& P, const rkl_opts& o) {
  const int lt = tail_level<T>(P);
  if (P.L() < 2 || lt <= 0) return false;
  const int sf = o.smoother == RKL_SMOOTH_GSRB ? 2 : o.s;
  for (int l = 0; l < lt; ++l)
    if (!fused_tau_supported<T>(view<T>(P.lv[l], P.periodic, nullptr), sf)) return false;
  return true;
}

rkl_status solve_batched(const rkl_grid* grids, int nbatch, const rkl_opts& o, const double* const* rho,
                         double* const* phi, rkl_stats* stats, hipStream_t st) {
  // group members by grid
  std::map<std::tuple<int, int, int, double, double, double, int>, std::vector<int>> groups;
  for (int q = 0; q < nbatch; ++q) {
    const rkl_grid& g = grids[q];
    groups[std::make_tuple(g.nx, g.ny, g.nz, g.hx, g.hy, g.hz, g.bc)].push_back(q);
  }
  std::vector<ClassPlan*> cls;
  std::vector<std::vector<int>> members;
  std::vector<int> single;  // members solved one by one
  for (auto& kv : groups) {
    const rkl_grid& g = grids[kv.second[0]];
    const rkl_opts og = with_s(o, g);
    Plan& P = get_plan(g, og.s, og.tau_frac, og.min_coarse, og.prec);
    const bool ok = og.prec == RKL_MIXED ? class_ok<float>(P, og) : class_ok<double>(P, og);
    if (!ok) {
      single.insert(single.end(), kv.second.begin(), kv.second.end());
      continue;
    }
    cls.push_back(&get_class(g, og, (int)kv.second.size()));
    members.push_back(kv.second);
  }
  rkl_status worst = RKL_OK;
  for (int q : single) {
    const rkl_status s =
        solve_one(grids[q], with_s(o, grids[q]), rho[q], nullptr, phi[q], stats ? &stats[q] : nullptr, st);
    if (s != RKL_OK && worst == RKL_OK) worst = s;
  }
  if (cls.empty()) return worst;
  std::vector<std::vector<double>> res0(cls.size());
  // every class's start enqueued, then one synchronisation for all of them
  std::vector<std::vector<const double*>> rp(cls.size());
  std::vector<std::vector<double*>> pp(cls.size());
  std::vector<std::vector<double>> r0(cls.size());
  for (size_t c = 0; c < cls.size(); ++c) {
    for (int q : members[c]) {
      rp[c].push_back(rho[q]);
      pp[c].push_back(phi[q]);
    }
    r0[c].assign(cls[c]->nb, 0.0);
    class_start_enqueue(*cls[c], o, rp[c].data(), pp[c].data(), r0[c].data(), st);
  }
  HIPCHK(hipStreamSynchronize(st));
  // (the state resets read the pinned mirrors in stream order; the host touches
  // those again only after the loop's synchronisation)
  for (size_t c = 0; c < cls.size(); ++c) res0[c] = class_start_finish(*cls[c], r0[c], st);
  // iterations per graph launch: enough for the predicted contraction
  const int iters = std::max(1, std::min(o.max_cycles + 1, (int)std::ceil(std::log(std::max(o.tol, 1e-300)) /
                                                                             std::log(0.12)) + 1));
  hipGraphExec_t ex = batch_graph(cls, o, iters);
  int launched = 0;
  while (true) {
    HIPCHK(hipGraphLaunch(ex, st));
    launched += iters;
    bool all = true;
    for (auto* c : cls) {
      HIPCHK(hipMemcpyAsync(c->hconv, c->conv, (size_t)c->nb * sizeof(ConvState), hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    for (auto* c : cls)
      for (int m = 0; m < c->nb; ++m) all = all && c->hconv[m].stop;
    if (all) break;
    if (launched > o.max_cycles + 1) fail(RKL_EHIP, "batched loop ended without a decision");
  }
  for (size_t c = 0; c < cls.size(); ++c) {
    class_finish(*cls[c], st);
    for (int m = 0; m < cls[c]->nb; ++m) {
      const ConvState& cs = cls[c]->hconv[m];
      const rkl_status s = finish_status(cs);
      if (s != RKL_OK && worst == RKL_OK) worst = s;
      if (stats) {
        rkl_stats& S = stats[members[c][m]];
        S.levels = cls[c]->base->L();
        S.res0 = res0[c][m];
        S.status = s;
        fill_stats(&S, cs, cs.result_m);
      }
    }
  }
  HIPCHK(hipStreamSynchronize(st));
  return worst;
}

// ------------------------------------------------------------------ tuning
// scratch device memory owned by one tuning call
struct DevScratch {
  std::vector<void*> p;
  void* get(size_t bytes) {
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(bytes, 8)) != hipSuccess) {
      (void)hipGetLastError();
      fail(RKL_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    p.push_back(q);
    return q;
  }
  ~DevScratch() {
    for (void* q : p) (void)hipFree(q);
  }
};

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Time every fused tau-step variant and workgroup target on one level shape
// (reps launches each, HIP events on the caller's stream) and install the
// fastest in the tuning table.
template <typename T>
int autotune_level(const rkl_grid& g, int s, int prec, int reps, rkl_tune_entry* res, int cap, hipStream_t st) {
  const Lev Lv = build_levels(g, INT_MAX, s, 0.9)[0];
  const bool per = g.bc == RKL_BC_PERIODIC;
  const LevelView<T> V = view<T>(Lv, per, nullptr);
  if (!fused_tau_supported<T>(V, s))
    fail(RKL_EINVAL, "no fused tau-step for this shape and s (needs nx >= 16, ny >= 8, nz >= 8, s <= " +
                         std::to_string(sizeof(T) == 8 ? 3 : 4) + "; two-dimensional: nz = 1, s <= " +
                         std::to_string(sizeof(T) == 8 ? 2 : 3) + ")");
  DevScratch mem;
  T* u = (T*)mem.get(Lv.n * sizeof(T));
  T* o = (T*)mem.get(Lv.n * sizeof(T));
  T* b = (T*)mem.get(Lv.n * sizeof(T));
  double* part = (double*)mem.get(fused_tau_blocks_max(Lv.nx, Lv.ny, Lv.nz) * sizeof(double));
  launch_fill<T>(u, Lv.n, (T)1, nullptr, st);
  launch_fill<T>(b, Lv.n, (T)0, nullptr, st);
  check_launch();
  EventPair ev;
  std::vector<rkl_tune_entry> all;
  const int targets[] = {64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096};
  for (int v = 1; v < FV_COUNT; ++v) {
    if (!fused_variant_ok<T>(v, s) || variant_is_2d(v) != level_is_2d(V)) continue;
    std::vector<int> tgs(std::begin(targets), std::end(targets));
    // strip variants: every distinct chunk length (1 .. 64 planes), since the
    // time depends on how evenly the workgroups fill the chip's SIMDs
    const int per = fused_chunk_blocks<T>(V, v, s);
    if (per > 0) {  // (the fixed targets stay, for the built-in choice's time)
      const int nmarch = level_is_2d(V) ? V.ny : V.nz;  // planes (2-D: rows) a chunk splits
      int last = -1;
      for (int zc = std::min(64, nmarch); zc >= 1; --zc) {
        const int chunks = (nmarch + zc - 1) / zc;
        if (chunks == last) continue;
        last = chunks;
        if ((long long)per * chunks > (1 << 22)) break;
        tgs.push_back(per * chunks);
      }
    }
    for (int tg : tgs) {
      const FusedChoice c{v, tg};
      for (int w = 0; w < 2; ++w) {
        launch_fused_tau_as<T>(V, c, u, b, o, s, Lv.smooth.data(), part, nullptr, st);
        std::swap(u, o);
      }
      HIPCHK(hipEventRecord(ev.a, st));
      for (int r = 0; r < reps; ++r) {
        launch_fused_tau_as<T>(V, c, u, b, o, s, Lv.smooth.data(), part, nullptr, st);
        std::swap(u, o);
      }
      HIPCHK(hipEventRecord(ev.b, st));
      HIPCHK(hipEventSynchronize(ev.b));
      check_launch();
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, ev.a, ev.b));
      rkl_tune_entry e;
      e.nx = g.nx;
      e.ny = g.ny;
      e.nz = g.nz;
      e.bc = g.bc;
      e.prec = prec;
      e.s = s;
      e.variant = v;
      e.target = tg;
      e.us = 1000.0 * (double)ms / reps;
      all.push_back(e);
    }
  }
  std::sort(all.begin(), all.end(), [](const rkl_tune_entry& a, const rkl_tune_entry& b) { return a.us < b.us; });
  tune_install(g.nx, g.ny, g.nz, per ? 1 : 0, sizeof(T) == 8 ? 1 : 0, s, FusedChoice{all[0].variant, all[0].target});
  for (int q = 0; q < (int)all.size() && q < cap; ++q) res[q] = all[q];
  return (int)all.size();
}

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

}  // namespace
}  // namespace rkl

using namespace rkl;

extern "C" {

void rkl_default_opts(rkl_opts* o) {
  if (!o) return;
  o->s = 2;
  o->tau_frac = 0.9;
  o->n_pre = 2;
  o->n_post = 1;
  o->min_coarse = 4;
  o->tol = 1e-10;
  o->max_cycles = 100;
  o->prec = RKL_FP64;
  o->four_pi_G = 4.0 * M_PI;
  o->coarse_tol = 0.0;
  o->coarse_max_steps = 200;
  o->smoother = RKL_SMOOTH_RKL;
  o->fuse = 1;
}

const char* rkl_last_error(void) { return g_err.c_str(); }

void rkl_release_all(void) {
  std::lock_guard<std::mutex> lk(g_plans_mu);
  g_graph.reset();
  g_classes.clear();
  g_plans.clear();
}

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

int rkl_tau_step_launches(const rkl_grid* grid, int s, int prec) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, nullptr);
    if (s < 1 || s > 64) fail(RKL_EINVAL, "s must be in [1, 64]");
    Lev L = build_levels(*grid, INT_MAX, s, 0.9)[0];
    const bool per = grid->bc == RKL_BC_PERIODIC;
    bool fused;
    if (prec == RKL_MIXED) fused = fused_tau_supported<float>(view<float>(L, per, nullptr), s);
    else if (prec == RKL_FP64) fused = fused_tau_supported<double>(view<double>(L, per, nullptr), s);
    else fail(RKL_EINVAL, "unknown precision");
    return (rkl_status)(fused ? 1 : s);
  });
}

rkl_status rkl_poisson_solve_batched(const rkl_grid* grids, int nbatch, const rkl_opts* opts,
                                     const double* const* rho, double* const* phi, rkl_stats* stats,
                                     void* hip_stream) {
  return guarded([&]() -> rkl_status {
    if (nbatch < 0) fail(RKL_EINVAL, "nbatch must be >= 0");
    if (nbatch == 0) return RKL_OK;
    if (!grids || !rho || !phi) fail(RKL_EINVAL, "grids, rho and phi must be non-NULL");
    for (int q = 0; q < nbatch; ++q) {
      validate_grid(&grids[q], nullptr);
      if (!rho[q] || !phi[q]) fail(RKL_EINVAL, "NULL member array");
      if (stats) {
        stats[q].history_len = 0;
        stats[q].status = RKL_OK;
      }
    }
    const rkl_opts o = resolve_opts(opts);
    static std::mutex batch_mu;
    std::lock_guard<std::mutex> lk(batch_mu);
    return solve_batched(grids, nbatch, o, rho, phi, stats, (hipStream_t)hip_stream);
  });
}

rkl_status rkl_tune_set(const rkl_tune_entry* entries, int n) {
  return guarded([&]() -> rkl_status {
    if (n < 0 || (n > 0 && !entries)) fail(RKL_EINVAL, "entries must hold n >= 0 items");
    for (int q = 0; q < n; ++q) {
      const rkl_tune_entry& e = entries[q];
      if (e.nx < 1 || e.ny < 1 || e.nz < 1 || (e.bc != RKL_BC_DIRICHLET && e.bc != RKL_BC_PERIODIC) ||
          (e.prec != RKL_FP64 && e.prec != RKL_MIXED) || e.variant < 0 || e.variant >= FV_COUNT ||
          (e.variant != FV_HEUR && e.target < 1))
        fail(RKL_EINVAL, "malformed tuning entry " + std::to_string(q));
      const bool ok = e.prec == RKL_FP64 ? fused_variant_ok<double>(e.variant, e.s) : fused_variant_ok<float>(e.variant, e.s);
      if (e.variant != FV_HEUR && !ok) fail(RKL_EINVAL, "variant not available for this s and precision in entry " + std::to_string(q));
      if (e.variant != FV_HEUR && variant_is_2d(e.variant) != (e.nz == 1))
        fail(RKL_EINVAL, "entry " + std::to_string(q) + ": strip2d variants are for two-dimensional levels (nz = 1) only");
    }
    for (int q = 0; q < n; ++q) {
      const rkl_tune_entry& e = entries[q];
      tune_install(e.nx, e.ny, e.nz, e.bc == RKL_BC_PERIODIC, e.prec == RKL_FP64, e.s, FusedChoice{e.variant, e.target});
    }
    return RKL_OK;
  });
}

rkl_status rkl_tune_clear(void) {
  return guarded([&]() -> rkl_status {
    tune_clear();
    std::lock_guard<std::mutex> lk(g_s_mu);
    g_auto_s.clear();
    return RKL_OK;
  });
}

rkl_status rkl_tune_get(const rkl_grid* level, int s, int prec, rkl_tune_entry* out) {
  return guarded([&]() -> rkl_status {
    validate_grid(level, nullptr);
    if (!out) fail(RKL_EINVAL, "out must be non-NULL");
    if (s < 1 || s > 64) fail(RKL_EINVAL, "s must be in [1, 64]");
    const Lev Lv = build_levels(*level, INT_MAX, s, 0.9)[0];
    const bool per = level->bc == RKL_BC_PERIODIC;
    FusedChoice c{FV_HEUR, 0};
    if (prec == RKL_FP64) {
      const LevelView<double> V = view<double>(Lv, per, nullptr);
      if (fused_tau_supported<double>(V, s)) c = fused_choice<double>(V, s);
    } else if (prec == RKL_MIXED) {
      const LevelView<float> V = view<float>(Lv, per, nullptr);
      if (fused_tau_supported<float>(V, s)) c = fused_choice<float>(V, s);
    } else {
      fail(RKL_EINVAL, "unknown precision");
    }
    *out = rkl_tune_entry{level->nx, level->ny, level->nz, (int)level->bc, prec, s, c.variant, c.target, 0.0};
    return RKL_OK;
  });
}

rkl_status rkl_autotune(const rkl_grid* level, int s, int prec, int reps, rkl_tune_entry* results, int cap,
                        int* n_results, void* hip_stream) {
  return guarded([&]() -> rkl_status {
    validate_grid(level, nullptr);
    if (reps < 1 || reps > 100000) fail(RKL_EINVAL, "reps must be in [1, 100000]");
    if (cap < 0 || (cap > 0 && !results)) fail(RKL_EINVAL, "results must hold cap >= 0 entries");
    int n;
    if (prec == RKL_FP64) n = autotune_level<double>(*level, s, prec, reps, results, cap, (hipStream_t)hip_stream);
    else if (prec == RKL_MIXED) n = autotune_level<float>(*level, s, prec, reps, results, cap, (hipStream_t)hip_stream);
    else fail(RKL_EINVAL, "unknown precision");
    if (n_results) *n_results = n;
    return RKL_OK;
  });
}

rkl_status rkl_tune_set_s(const rkl_grid* grid, int prec, int s) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, nullptr);
    if (prec != RKL_FP64 && prec != RKL_MIXED) fail(RKL_EINVAL, "unknown precision");
    if (s < 0 || s > 64) fail(RKL_EINVAL, "s must be in [0, 64] (0 erases the entry)");
    std::lock_guard<std::mutex> lk(g_s_mu);
    const auto k = std::make_tuple(grid->nx, grid->ny, grid->nz, (int)grid->bc, prec);
    if (s == 0) g_auto_s.erase(k);
    else g_auto_s[k] = s;
    return RKL_OK;
  });
}

int rkl_level_shapes(const rkl_grid* grid, int min_coarse, int* nxyz, int cap) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, nullptr);
    if (min_coarse < 2) fail(RKL_EINVAL, "min_coarse must be >= 2");
    if (cap < 0 || (cap > 0 && !nxyz)) fail(RKL_EINVAL, "nxyz must hold 3 * cap ints");
    const std::vector<Lev> lv = build_levels(*grid, min_coarse, 2, 0.9);
    for (int l = 0; l < (int)lv.size() && l < cap; ++l) {
      nxyz[3 * l] = lv[l].nx;
      nxyz[3 * l + 1] = lv[l].ny;
      nxyz[3 * l + 2] = lv[l].nz;
    }
    return (rkl_status)lv.size();
  });
}

const char* rkl_variant_name(int variant) { return fused_variant_name(variant); }

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

int rkl_s_opt(const rkl_grid* grid, double tau_frac, int kmax, double digits, double* m_eff_out) {
  return guarded([&]() -> rkl_status {
    validate_grid(grid, nullptr);
    if (!(tau_frac > 0.0 && tau_frac < 2.0)) fail(RKL_EINVAL, "tau_frac must be in (0, 2)");
    if (kmax < 1) fail(RKL_EINVAL, "kmax must be >= 1");
    if (!(digits > 0.0) || !std::isfinite(digits)) fail(RKL_EINVAL, "digits must be positive and finite");
    const Lev L = build_levels(*grid, INT_MAX, 1, tau_frac)[0];
    return (rkl_status)s_opt_rule(L, grid->bc == RKL_BC_PERIODIC, tau_frac, kmax, digits, m_eff_out);
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
