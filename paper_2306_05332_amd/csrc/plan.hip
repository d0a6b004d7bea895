// Plan cache and level hierarchy of the solver (Sec. 2.1 levels, App. A
// stage coefficients, App. A.3 / A.4 stage counts), option checks, error
// state, and the C-ABI entry points that configure rather than compute.

#include "solver_core.h"

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
  cap = std::max(cap, strip_rs_parts_max(P->lv[0].nx, P->lv[0].ny, P->lv[0].nz));
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

// the coarsest level fits the one-workgroup LDS solver
bool coarse_in_lds(const Plan& P, const Lev& C) {
  size_t rows = 0;
  for (int s : P.sched) rows += (size_t)s;
  return C.n <= (size_t)COARSE_MAX_CELLS && P.sched.size() <= (size_t)COARSE_MAX_SCHED &&
         rows <= (size_t)COARSE_MAX_COEF;
}

// read `nq` device scalars from P.dscal + at (synchronises the stream)
const double* readback(Plan& P, int nq, hipStream_t st, int at) {
  HIPCHK(hipMemcpyAsync(P.hscal, P.dscal + at, nq * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return P.hscal;
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
  if (o.fuse < 0 || o.fuse > 3) fail(RKL_EINVAL, "fuse must be 0 .. 3 (bit 0: prolongation, bit 1: restriction)");
  if (o.zero_start != 0 && o.zero_start != 1) fail(RKL_EINVAL, "zero_start must be 0 or 1");
  return o;
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
  o->fuse = 3;
  o->zero_start = 0;
}

const char* rkl_last_error(void) { return g_err.c_str(); }

void rkl_release_all(void) {
  std::lock_guard<std::mutex> lk(g_plans_mu);
  release_batched();
  g_plans.clear();
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

}  // extern "C"
