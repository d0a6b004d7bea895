// Tile autotuner of the fused tau-step (rkl_autotune) and the tuning-table
// entry points.

#include "solver_core.h"

namespace rkl {

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

}  // namespace rkl

using namespace rkl;

extern "C" {

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

const char* rkl_variant_name(int variant) { return fused_variant_name(variant); }

}  // extern "C"
