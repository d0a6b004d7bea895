// Batched solves (rkl_poisson_solve_batched): classes of identical grids
// iterated together, their refinement iterations captured in one HIP graph.

#include "solver_core.h"

namespace rkl {

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
  ps = std::max(ps, strip_rs_parts_max(F.nx, F.ny, F.nz));
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

void release_batched() {
  g_graph.reset();
  g_classes.clear();
}

}  // namespace rkl

using namespace rkl;

extern "C" {

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

}  // extern "C"
