// Coarse tail of the V-cycle in one workgroup.
//
// Below a few thousand cells a level is far too small to fill the GPU, and
// every kernel launch costs several microseconds, so the part of the V-cycle
// (Sec. 2.1) from the first level of at most TAIL_MAX_CELLS cells down to the
// coarsest one runs inside a single 512-thread workgroup with all of its
// arrays in LDS:
//   b of the top tail level (as restricted, its mean removed when periodic,
//   Sec. 2.3) -> N_pre RKL tau-steps from zero -> residual + 8-point
//   restriction -> ... -> accelerated RKL coarsest solve (App. A.4, on one
//   wavefront) -> prolongation + correction -> N_post tau-steps -> ... ->
//   the top level's correction u, written back to HBM.
// The arithmetic is that of the per-level kernels (stage recurrence of App. A
// eq. RKL_intermediate_source; ghosts of Sec. 2.3 for the error equation:
// homogeneous Dirichlet -c or periodic wrap).  Two-dimensional hierarchies
// (nz = 1 and ihz2 = 0 on every level) restrict with the 4-child average of
// eq. restriction_example_2D and prolong with the parent plane as its own z
// neighbour, i.e. the (9, 3, 3, 1)/16 weights of eq. prolongation_example_2D.
#include <cstring>

#include "kernels.h"

namespace rkl {

template <typename T>
struct TailLevel {
  int nx, ny, nz, off;  // off: first of this level's three LDS arrays (u, alt, b)
  T ihx2, ihy2, ihz2;
  T mu[TAIL_MAX_S], nu[TAIL_MAX_S], c[TAIL_MAX_S];
  T gsc;                // red-black Gauss-Seidel smoother: 1 / D, D = 2 sum h^-2 (interior cells)
};

template <typename T>
struct TailArgs {
  int nlev, s, n_pre, n_post, periodic, cmax;
  int gs;               // smoother: 0 RKL tau-step, 1 red-black Gauss-Seidel pass
  int flat;             // 1: two-dimensional levels
  double ctol;
  CoarseSchedule cs;
  TailLevel<T> lv[TAIL_MAX_LEVELS];
};

constexpr int TNT = 512;

// Cell walk of one thread over a level: q = tid, tid + TNT, ... with its
// (i, j, k) advanced by carries (one division per level and phase, not per cell).
struct CellWalk {
  int q, i, j, k, di, dj, dk, n, nx, ny;
  __device__ CellWalk(int tid, int stride, int nx_, int ny_, int nz_) : nx(nx_), ny(ny_) {
    n = nx_ * ny_ * nz_;
    q = tid;
    i = tid % nx;
    j = (tid / nx) % ny;
    k = tid / (nx * ny);
    di = stride % nx;
    dj = (stride / nx) % ny;
    dk = stride / (nx * ny);
  }
  __device__ bool ok() const { return q < n; }
  __device__ void next(int stride) {
    q += stride;
    i += di;
    int cj = 0;
    if (i >= nx) {
      i -= nx;
      cj = 1;
    }
    j += dj + cj;
    int ck = 0;
    if (j >= ny) {
      j -= ny;
      ck = 1;
    }
    k += dk + ck;
  }
};

// 7-point M at cell q = (i, j, k) of a level held in LDS.  Every neighbour is
// read unconditionally: a periodic neighbour wraps, a missing Dirichlet
// neighbour reads the centre with sign -1 (the error-equation ghost -c), so
// the six reads can be in flight together.
template <typename T>
__device__ __forceinline__ T tail_lap(const TailLevel<T>& V, const T* Y, int q, int i, int j, int k, int per) {
  const int nx = V.nx, ny = V.ny, nz = V.nz;
  const int sy = nx, sz = nx * ny;
  const int qxm = i > 0 ? q - 1 : (per ? q + nx - 1 : q);
  const int qxp = i < nx - 1 ? q + 1 : (per ? q - (nx - 1) : q);
  const int qym = j > 0 ? q - sy : (per ? q + (ny - 1) * sy : q);
  const int qyp = j < ny - 1 ? q + sy : (per ? q - (ny - 1) * sy : q);
  const int qzm = k > 0 ? q - sz : (per ? q + (nz - 1) * sz : q);
  const int qzp = k < nz - 1 ? q + sz : (per ? q - (nz - 1) * sz : q);
  const T c = Y[q];
  T xm = Y[qxm], xp = Y[qxp], ym = Y[qym], yp = Y[qyp], zm = Y[qzm], zp = Y[qzp];
  if (!per) {
    xm = i > 0 ? xm : -xm;
    xp = i < nx - 1 ? xp : -xp;
    ym = j > 0 ? ym : -ym;
    yp = j < ny - 1 ? yp : -yp;
    zm = k > 0 ? zm : -zm;
    zp = k < nz - 1 ? zp : -zp;
  }
  return ((xm + xp) - (T)2 * c) * V.ihx2 + ((ym + yp) - (T)2 * c) * V.ihy2 + ((zm + zp) - (T)2 * c) * V.ihz2;
}

// Value of `v` in lane `src` (ds_bpermute: the LDS crossbar, no LDS memory).
__device__ __forceinline__ double lane_get(double v, int src) {
  const int a = src << 2;
  const int lo = __builtin_amdgcn_ds_bpermute(a, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(a, __double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_get(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

// Accelerated RKL on a coarsest level of at most 64 cells held one cell per
// lane of wavefront 0, in registers: the six neighbours come from their
// lanes by lane exchanges (a Dirichlet ghost reads the lane itself and flips
// the sign), so a stage touches no LDS memory.  Same schedule, stop test
// (before every tau-step) and periodic mean removal as the LDS form.
template <typename T>
__device__ void coarse_regs(const TailLevel<T>& V, const int* ssched, const int* scoff, const double* scoef,
                            int nsched, int per, double ctol, int cmax, T* B, T* U) {
  const int lane = threadIdx.x;
  const int nx = V.nx, ny = V.ny, nz = V.nz, n = nx * ny * nz;
  const bool has = lane < n;
  const int q = has ? lane : 0;
  const int i = q % nx, j = (q / nx) % ny, k = q / (nx * ny);
  const int sy = nx, sz = nx * ny;
  int nb[6];
  nb[0] = i > 0 ? q - 1 : (per ? q + nx - 1 : q);
  nb[1] = i < nx - 1 ? q + 1 : (per ? q - (nx - 1) : q);
  nb[2] = j > 0 ? q - sy : (per ? q + (ny - 1) * sy : q);
  nb[3] = j < ny - 1 ? q + sy : (per ? q - (ny - 1) * sy : q);
  nb[4] = k > 0 ? q - sz : (per ? q + (nz - 1) * sz : q);
  nb[5] = k < nz - 1 ? q + sz : (per ? q - (nz - 1) * sz : q);
  T sg[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) sg[d] = (T)1;
  if (!per) {
    if (i == 0) sg[0] = (T)-1;
    if (i == nx - 1) sg[1] = (T)-1;
    if (j == 0) sg[2] = (T)-1;
    if (j == ny - 1) sg[3] = (T)-1;
    if (k == 0) sg[4] = (T)-1;
    if (k == nz - 1) sg[5] = (T)-1;
  }
  if (!has) {
#pragma unroll
    for (int d = 0; d < 6; ++d) nb[d] = lane;  // idle lanes hold 0 and read themselves
  }
  const T bl = has ? B[q] : (T)0;
  auto mres = [&](T y) -> T {  // (M y - b) at this lane's cell; every lane takes part in the exchanges
    T v[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) v[d] = sg[d] * lane_get(y, nb[d]);
    return ((v[0] + v[1]) - (T)2 * y) * V.ihx2 + ((v[2] + v[3]) - (T)2 * y) * V.ihy2 +
           ((v[4] + v[5]) - (T)2 * y) * V.ihz2 - bl;
  };
  // Stop test ||M u - b|| <= ctol ||b|| before every tau-step, on squared
  // norms.  On a periodic level M annihilates constants, so the residual of
  // a tau-step's result is taken before its mean is removed: the two
  // wavefront sums are independent (they overlap), and the residual is also
  // the next tau-step's first-stage M u - b.
  const double b2 = wave_sum_dpp((double)bl * (double)bl);
  const double lim2 = ctol * ctol * b2;
  const double inv_n = 1.0 / (double)n;
  T u = (T)0;
  int step = 0;
  if (b2 > 0.0) {
    T r = mres(u);
    while (true) {
      const double res2 = wave_sum_dpp(has ? (double)r * (double)r : 0.0);
      if (per && step > 0) u -= (T)(wave_sum_dpp(has ? (double)u : 0.0) * inv_n);
      if (!has) u = (T)0;
      if (res2 <= lim2 || step >= cmax) break;
      const int qs = step < nsched ? step : nsched - 1;
      const int s = ssched[qs];
      const double* co = scoef + 3 * scoff[qs];
      T y1 = u, y2 = u;  // Y_{j-1}, Y_{j-2}
      for (int jj = 1; jj <= s; ++jj) {
        const T mu = (T)co[3 * (jj - 1)], nu = (T)co[3 * (jj - 1) + 1], c = (T)co[3 * (jj - 1) + 2];
        const T rr = jj == 1 ? r : mres(y1);  // stage 1: the stop test's M u - b
        T y = (jj == 1) ? y1 + c * rr : mu * y1 + nu * y2 + c * rr;
        if (!has) y = (T)0;
        y2 = y1;
        y1 = y;
      }
      u = y1;
      r = mres(u);
      ++step;
    }
  }
  if (has) U[q] = u;
}

template <typename T>
__global__ __launch_bounds__(TNT) void k_tail(TailArgs<T> A, const T* __restrict__ b_top, T* __restrict__ u_top,
                                              Batch bt, const int* __restrict__ stop) {
  {
    const long long mb = blockIdx.x;  // one workgroup per member
    b_top += mb * bt.s0;
    u_top += mb * bt.s0;
    if (stop != nullptr) stop += mb * bt.stop_stride;
  }
  extern __shared__ __align__(16) unsigned char pool_raw[];
  __shared__ double red[TNT / WAVE];
  __shared__ double bc;
  __shared__ int ssched[COARSE_MAX_SCHED];
  __shared__ int scoff[COARSE_MAX_SCHED];
  __shared__ double scoef[3 * COARSE_MAX_COEF];
  {
    int cells = 0;  // the pool holds three arrays per level
    for (int l = 0; l < A.nlev; ++l) cells += 3 * A.lv[l].nx * A.lv[l].ny * A.lv[l].nz;
    lds_poison(reinterpret_cast<T*>(pool_raw), cells);
    lds_poison(red, TNT / WAVE);
    lds_poison(scoef, 3 * COARSE_MAX_COEF);
    lds_poison_sync();
  }
  if (stop != nullptr && *stop) return;
  T* pool = reinterpret_cast<T*>(pool_raw);
  const int tid = threadIdx.x;
  const int per = A.periodic;
  const int nl = A.nlev;
  // which of a level's two iterate arrays is current: bit l set -> the second
  unsigned swapped = 0u;
  const int nsched = min(A.cs.nsched, COARSE_MAX_SCHED);
  for (int q = tid; q < nsched; q += TNT) {
    ssched[q] = A.cs.sched[q];
    scoff[q] = A.cs.coff[q];
  }
  const int ncoef = nsched > 0 ? min(A.cs.coff[nsched - 1] + A.cs.sched[nsched - 1], COARSE_MAX_COEF) : 0;
  for (int q = tid; q < 3 * ncoef; q += TNT) scoef[q] = A.cs.coef[q];

  auto nof = [&](int l) { return A.lv[l].nx * A.lv[l].ny * A.lv[l].nz; };
  auto bptr = [&](int l) { return pool + A.lv[l].off + 2 * nof(l); };
  auto curp = [&](int l) { return pool + A.lv[l].off + (((swapped >> l) & 1u) ? nof(l) : 0); };
  auto altp = [&](int l) { return pool + A.lv[l].off + (((swapped >> l) & 1u) ? 0 : nof(l)); };
  // block-wide: subtract the mean of level l's right-hand side (periodic)
  auto remove_b_mean = [&](int l) {
    T* B = bptr(l);
    const int n = nof(l);
    double sm = 0.0;
    for (int q = tid; q < n; q += TNT) sm += (double)B[q];
    const double t = block_sum<TNT>(sm, red);
    if (tid == 0) bc = t;
    __syncthreads();
    const T m = (T)(bc / (double)n);
    for (int q = tid; q < n; q += TNT) B[q] -= m;
    __syncthreads();
  };
  // One sweep over level l calling fn(q, (M Y)[q], Y[q]) for every cell.  When
  // the walk stride TNT is a multiple of nx * ny, a thread's cells share
  // (i, j): its x and y neighbour offsets are computed once and it walks k;
  // other levels take the generic cell walk.  Ghosts as in tail_lap.
  auto lap_sweep = [&](int l, const T* Y, auto&& fn) {
    const TailLevel<T>& V = A.lv[l];
    const int nx = V.nx, ny = V.ny, nz = V.nz, nxy = nx * ny, n = nxy * nz;
    if (TNT % nxy == 0) {
      const int i = tid % nx, j = (tid / nx) % ny, kstep = TNT / nxy;
      const int dxm = i > 0 ? -1 : (per ? nx - 1 : 0);
      const int dxp = i < nx - 1 ? 1 : (per ? -(nx - 1) : 0);
      const int dym = j > 0 ? -nx : (per ? (ny - 1) * nx : 0);
      const int dyp = j < ny - 1 ? nx : (per ? -(ny - 1) * nx : 0);
      const bool gxm = !per && i == 0, gxp = !per && i == nx - 1;
      const bool gym = !per && j == 0, gyp = !per && j == ny - 1;
      for (int q = tid, k = tid / nxy; q < n; q += TNT, k += kstep) {
        const int dzm = k > 0 ? -nxy : (per ? (nz - 1) * nxy : 0);
        const int dzp = k < nz - 1 ? nxy : (per ? -(nz - 1) * nxy : 0);
        const T c = Y[q];
        T xm = Y[q + dxm], xp = Y[q + dxp], ym = Y[q + dym], yp = Y[q + dyp], zm = Y[q + dzm], zp = Y[q + dzp];
        if (!per) {
          xm = gxm ? -xm : xm;
          xp = gxp ? -xp : xp;
          ym = gym ? -ym : ym;
          yp = gyp ? -yp : yp;
          zm = k > 0 ? zm : -zm;
          zp = k < nz - 1 ? zp : -zp;
        }
        fn(q, ((xm + xp) - (T)2 * c) * V.ihx2 + ((ym + yp) - (T)2 * c) * V.ihy2 + ((zm + zp) - (T)2 * c) * V.ihz2,
           c);
      }
    } else {
      for (CellWalk w(tid, TNT, nx, ny, nz); w.ok(); w.next(TNT))
        fn(w.q, tail_lap(V, Y, w.q, w.i, w.j, w.k, per), Y[w.q]);
    }
  };
  // one relaxation on level l: an RKL tau-step (stage by stage, Y_j over
  // Y_{j-2}) or a red-black Gauss-Seidel pass (in place: a cell's neighbours
  // all have the other colour on these even-sized levels); from_zero: u = 0
  auto tau = [&](int l, bool from_zero) {
    const TailLevel<T>& V = A.lv[l];
    const int n = nof(l);
    T* B = bptr(l);
    T* cur = curp(l);
    T* alt = altp(l);
    if (from_zero) {
      for (int q = tid; q < n; q += TNT) cur[q] = (T)0;
      __syncthreads();
    }
    if (A.gs) {
      for (int colour = 0; colour < 2; ++colour) {
        for (CellWalk w(tid, TNT, V.nx, V.ny, V.nz); w.ok(); w.next(TNT)) {
          if (((w.i + w.j + w.k) & 1) != colour) continue;
          const int q = w.q;
          T cf = V.gsc;
          if (!per) {  // the operator's diagonal: + h_d^-2 per Dirichlet face of the cell
            T extra = (T)0;
            if (w.i == 0) extra += V.ihx2;
            if (w.i == V.nx - 1) extra += V.ihx2;
            if (w.j == 0) extra += V.ihy2;
            if (w.j == V.ny - 1) extra += V.ihy2;
            if (w.k == 0) extra += V.ihz2;
            if (w.k == V.nz - 1) extra += V.ihz2;
            if (extra != (T)0) cf = (T)1 / ((T)1 / V.gsc + extra);
          }
          cur[q] += cf * (tail_lap(V, cur, q, w.i, w.j, w.k, per) - B[q]);
        }
        __syncthreads();
      }
      return;
    }
    for (int j = 1; j <= A.s; ++j) {
      const T* yp = (j & 1) ? cur : alt;
      T* yw = (j & 1) ? alt : cur;
      const T mu = V.mu[j - 1], nu = V.nu[j - 1], c = V.c[j - 1];
      if (j == 1)
        lap_sweep(l, yp, [&](int q, T mv, T cv) { yw[q] = cv + c * (mv - B[q]); });
      else
        lap_sweep(l, yp, [&](int q, T mv, T cv) { yw[q] = mu * cv + nu * yw[q] + c * (mv - B[q]); });
      __syncthreads();
    }
    if (A.s & 1) swapped ^= 1u << l;
  };

  // top level right-hand side: eight loads in flight per thread before the
  // stores (one at a time, each would wait out the memory latency)
  {
    const int n = nof(0);
    T* B = bptr(0);
    for (int q0 = 0; q0 < n; q0 += 8 * TNT) {
      T v[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int q = q0 + m * TNT + tid;
        v[m] = q < n ? b_top[q] : (T)0;
      }
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int q = q0 + m * TNT + tid;
        if (q < n) B[q] = v[m];
      }
    }
    __syncthreads();
    if (per) remove_b_mean(0);
  }
  // downstroke
  for (int l = 0; l < nl - 1; ++l) {
    if (A.n_pre > 0) {
      tau(l, true);
      for (int q = 1; q < A.n_pre; ++q) tau(l, false);
    } else {
      T* cur = curp(l);
      for (int q = tid; q < nof(l); q += TNT) cur[q] = (T)0;
      __syncthreads();
    }
    // b_{l+1} = R(b_l - M u_l): the fine residual into the level's free
    // second array, then the average of each coarse cell's children (periodic:
    // the coarse sum taken on the way, its mean removed after)
    const TailLevel<T>& F = A.lv[l];
    const TailLevel<T>& C = A.lv[l + 1];
    const T* U = curp(l);
    const T* B = bptr(l);
    T* RF = altp(l);
    T* BC = bptr(l + 1);
    lap_sweep(l, U, [&](int q, T mv, T) { RF[q] = B[q] - mv; });
    __syncthreads();
    const int ndz = A.flat ? 1 : 2;
    const T rw = A.flat ? (T)0.25 : (T)0.125;
    const int fnxy = F.nx * F.ny;
    double csum = 0.0;
    for (CellWalk w(tid, TNT, C.nx, C.ny, C.nz); w.ok(); w.next(TNT)) {
      const int f0 = ((2 * w.k) * F.ny + 2 * w.j) * F.nx + 2 * w.i;
      T acc = (RF[f0] + RF[f0 + 1]) + (RF[f0 + F.nx] + RF[f0 + F.nx + 1]);
      if (ndz == 2) acc += (RF[f0 + fnxy] + RF[f0 + fnxy + 1]) + (RF[f0 + fnxy + F.nx] + RF[f0 + fnxy + F.nx + 1]);
      const T v = acc * rw;
      BC[w.q] = v;
      csum += (double)v;
    }
    if (per) {
      const double t = block_sum<TNT>(csum, red);
      if (tid == 0) bc = t;
      __syncthreads();
      const T m = (T)(bc / (double)nof(l + 1));
      for (int q = tid; q < nof(l + 1); q += TNT) BC[q] -= m;
    }
    __syncthreads();
  }
  // coarsest level: accelerated RKL on wavefront 0 (up to 4 cells per lane),
  // neighbour offsets precomputed once; ghosts: periodic wrap or -c.  Only
  // this wavefront touches the level's arrays, and the LDS operations of one
  // wavefront complete in issue order, so wavefront-scope fences (compiler
  // ordering) separate the stages.
  if (nof(nl - 1) <= WAVE) {
    if (tid < WAVE)
      coarse_regs<T>(A.lv[nl - 1], ssched, scoff, scoef, nsched, per, A.ctol, A.cmax, bptr(nl - 1), curp(nl - 1));
    __syncthreads();
  } else {
    const int l = nl - 1;
    const TailLevel<T>& V = A.lv[l];
    const int n = nof(l);
    if (tid < WAVE) {
      T* B = bptr(l);
      T* cur = curp(l);
      T* alt = altp(l);
      int nb[4][6];   // neighbour index (the cell itself for a Dirichlet ghost)
      unsigned gh[4]; // bit d: neighbour d is a Dirichlet ghost (-c)
      bool has[4];
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const int q = tid + WAVE * cc;
        has[cc] = q < n;
        const int qq = has[cc] ? q : 0;
        const int i = qq % V.nx, j = (qq / V.nx) % V.ny, k = qq / (V.nx * V.ny);
        const int sy = V.nx, sz = V.nx * V.ny;
        nb[cc][0] = i > 0 ? qq - 1 : (per ? qq + V.nx - 1 : qq);
        nb[cc][1] = i < V.nx - 1 ? qq + 1 : (per ? qq - (V.nx - 1) : qq);
        nb[cc][2] = j > 0 ? qq - sy : (per ? qq + (V.ny - 1) * sy : qq);
        nb[cc][3] = j < V.ny - 1 ? qq + sy : (per ? qq - (V.ny - 1) * sy : qq);
        nb[cc][4] = k > 0 ? qq - sz : (per ? qq + (V.nz - 1) * sz : qq);
        nb[cc][5] = k < V.nz - 1 ? qq + sz : (per ? qq - (V.nz - 1) * sz : qq);
        gh[cc] = 0u;
        if (!per) {
          if (i == 0) gh[cc] |= 1u;
          if (i == V.nx - 1) gh[cc] |= 2u;
          if (j == 0) gh[cc] |= 4u;
          if (j == V.ny - 1) gh[cc] |= 8u;
          if (k == 0) gh[cc] |= 16u;
          if (k == V.nz - 1) gh[cc] |= 32u;
        }
      }
      auto lapc = [&](const T* Y, int cc) -> T {
        const int q = tid + WAVE * cc;
        const T c = Y[q];
        T v[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) v[d] = Y[nb[cc][d]];
#pragma unroll
        for (int d = 0; d < 6; ++d) v[d] = ((gh[cc] >> d) & 1u) ? -v[d] : v[d];
        return ((v[0] + v[1]) - (T)2 * c) * V.ihx2 + ((v[2] + v[3]) - (T)2 * c) * V.ihy2 +
               ((v[4] + v[5]) - (T)2 * c) * V.ihz2;
      };
      T bl[4];
      double b2 = 0.0;
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const int q = tid + WAVE * cc;
        bl[cc] = has[cc] ? B[q] : (T)0;
        if (has[cc]) cur[q] = (T)0;
        b2 += (double)bl[cc] * (double)bl[cc];
      }
      const double bnorm = sqrt(wave_sum_dpp(b2));
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      int step = 0;
      if (bnorm > 0.0) {
        T rchk[4];  // the stop test's M u - b, which is also the first stage's
        while (true) {
          double r2 = 0.0;
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            rchk[cc] = (T)0;
            if (has[cc]) {
              const T r = lapc(cur, cc) - bl[cc];
              rchk[cc] = r;
              r2 += (double)r * (double)r;
            }
          }
          const double res = sqrt(wave_sum_dpp(r2));
          if (res <= A.ctol * bnorm || step >= A.cmax) break;
          const int qs = step < nsched ? step : nsched - 1;
          const int s = ssched[qs];
          const double* co = scoef + 3 * scoff[qs];
          for (int j = 1; j <= s; ++j) {
            const T mu = (T)co[3 * (j - 1)], nu = (T)co[3 * (j - 1) + 1], c = (T)co[3 * (j - 1) + 2];
            const T* yp = (j & 1) ? cur : alt;
            T* yw = (j & 1) ? alt : cur;
            T outv[4];
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
              const int q = tid + WAVE * cc;
              outv[cc] = (T)0;
              if (has[cc]) {
                const T r = j == 1 ? rchk[cc] : lapc(yp, cc) - bl[cc];
                outv[cc] = (j == 1) ? yp[q] + c * r : mu * yp[q] + nu * yw[q] + c * r;
              }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
              const int q = tid + WAVE * cc;
              if (has[cc]) yw[q] = outv[cc];
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          }
          if (s & 1) {
            T* t = cur;
            cur = alt;
            alt = t;
          }
          if (per) {
            double sm = 0.0;
#pragma unroll
            for (int cc = 0; cc < 4; ++cc)
              if (has[cc]) sm += (double)cur[tid + WAVE * cc];
            const T m = (T)(wave_sum_dpp(sm) / (double)n);
#pragma unroll
            for (int cc = 0; cc < 4; ++cc)
              if (has[cc]) cur[tid + WAVE * cc] -= m;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          }
          ++step;
        }
      }
      // leave the result in the level's first array
      if (cur != curp(l)) {
        T* dst = curp(l);
        for (int q = tid; q < n; q += WAVE) dst[q] = cur[q];
      }
    }
    __syncthreads();
  }
  // upstroke
  for (int l = nl - 2; l >= 0; --l) {
    const TailLevel<T>& F = A.lv[l];
    const TailLevel<T>& C = A.lv[l + 1];
    const T* E = curp(l + 1);
    T* U = curp(l);
    // per axis: the parent and the neighbour on the fine cell's side
    // (wrapped, or clamped with sign -1 for a homogeneous Dirichlet ghost);
    // the eight coarse values then weigh (3,1) x (3,1) x (3,1) / 64.  A 2-D
    // hierarchy takes the parent plane as its own z neighbour.
    const int cnxy = C.nx * C.ny;
    const int fnxy = F.nx * F.ny;
    if (!A.flat && TNT % fnxy == 0) {
      // a thread's cells share (i, j) and step k by TNT / (nx ny) (one parity
      // of k when that step is even): the x-y parents and neighbours are set
      // once, and a coarse plane's x-y interpolation serves the two fine
      // planes around it
      const int i = tid % F.nx, j = (tid / F.nx) % F.ny, kstep = TNT / fnxy;
      int ox0 = i >> 1, ox1 = ox0 + ((i & 1) ? 1 : -1);
      T gx = (T)1, gy = (T)1;
      if (per) ox1 = ox1 < 0 ? ox1 + C.nx : (ox1 >= C.nx ? ox1 - C.nx : ox1);
      else if (ox1 < 0 || ox1 >= C.nx) { ox1 = ox0; gx = (T)-1; }
      const int J = j >> 1;
      int jn = J + ((j & 1) ? 1 : -1);
      if (per) jn = jn < 0 ? jn + C.ny : (jn >= C.ny ? jn - C.ny : jn);
      else if (jn < 0 || jn >= C.ny) { jn = J; gy = (T)-1; }
      const int oy0 = J * C.nx, oy1 = jn * C.nx;
      auto exy = [&](int Kw) -> T {  // 16 x (x, then y interpolation of coarse plane Kw)
        const int o = Kw * cnxy;
        return (T)3 * ((T)3 * E[o + oy0 + ox0] + gx * E[o + oy0 + ox1]) +
               gy * ((T)3 * E[o + oy1 + ox0] + gx * E[o + oy1 + ox1]);
      };
      int pa = -1, pb = -1;  // wrapped indices of the previous cell's two planes
      T va = (T)0, vb = (T)0;
      for (int k = tid / fnxy; k < F.nz; k += kstep) {
        const int K = k >> 1;
        int kn = K + ((k & 1) ? 1 : -1);
        T gz = (T)1;
        if (per) kn = kn < 0 ? kn + C.nz : (kn >= C.nz ? kn - C.nz : kn);
        else if (kn < 0 || kn >= C.nz) { kn = K; gz = (T)-1; }
        const T p0 = K == pa ? va : (K == pb ? vb : exy(K));
        const T p1 = kn == pa ? va : (kn == pb ? vb : exy(kn));
        pa = K;
        va = p0;
        pb = kn;
        vb = p1;
        U[k * fnxy + j * F.nx + i] += ((T)3 * p0 + gz * p1) * (T)(1.0 / 64.0);
      }
    } else
    for (CellWalk w(tid, TNT, F.nx, F.ny, F.nz); w.ok(); w.next(TNT)) {
      const int q = w.q;
      int ox[2], oy[2], oz[2];
      T gx = (T)1, gy = (T)1, gz = (T)1;
      {
        const int I = w.i >> 1, n1 = I + ((w.i & 1) ? 1 : -1);
        ox[0] = I;
        if (per) ox[1] = n1 < 0 ? n1 + C.nx : (n1 >= C.nx ? n1 - C.nx : n1);
        else if (n1 < 0 || n1 >= C.nx) { ox[1] = I; gx = (T)-1; }
        else ox[1] = n1;
      }
      {
        const int J = w.j >> 1, n1 = J + ((w.j & 1) ? 1 : -1);
        oy[0] = J * C.nx;
        int jn;
        if (per) jn = n1 < 0 ? n1 + C.ny : (n1 >= C.ny ? n1 - C.ny : n1);
        else if (n1 < 0 || n1 >= C.ny) { jn = J; gy = (T)-1; }
        else jn = n1;
        oy[1] = jn * C.nx;
      }
      {
        const int K = w.k >> 1, n1 = K + ((w.k & 1) ? 1 : -1);
        oz[0] = K * cnxy;
        int kn;
        if (A.flat) kn = K;
        else if (per) kn = n1 < 0 ? n1 + C.nz : (n1 >= C.nz ? n1 - C.nz : n1);
        else if (n1 < 0 || n1 >= C.nz) { kn = K; gz = (T)-1; }
        else kn = n1;
        oz[1] = kn * cnxy;
      }
      const T e000 = E[oz[0] + oy[0] + ox[0]], e001 = E[oz[0] + oy[0] + ox[1]];
      const T e010 = E[oz[0] + oy[1] + ox[0]], e011 = E[oz[0] + oy[1] + ox[1]];
      const T e100 = E[oz[1] + oy[0] + ox[0]], e101 = E[oz[1] + oy[0] + ox[1]];
      const T e110 = E[oz[1] + oy[1] + ox[0]], e111 = E[oz[1] + oy[1] + ox[1]];
      // x first (3 e0 + gx e1), then y, then z
      const T p00 = (T)3 * e000 + gx * e001, p01 = (T)3 * e010 + gx * e011;
      const T p10 = (T)3 * e100 + gx * e101, p11 = (T)3 * e110 + gx * e111;
      const T p0 = (T)3 * p00 + gy * p01, p1 = (T)3 * p10 + gy * p11;
      U[q] += ((T)3 * p0 + gz * p1) * (T)(1.0 / 64.0);
    }
    __syncthreads();
    for (int q = 0; q < A.n_post; ++q) tau(l, false);
  }
  // correction of the top tail level back to HBM
  {
    const T* U = curp(0);
    for (int q = tid; q < nof(0); q += TNT) u_top[q] = U[q];
  }
}

template <typename T>
size_t tail_lds_bytes(const TailShape& ts) {
  size_t cells = 0;
  for (int l = 0; l < ts.nlev; ++l) cells += 3 * (size_t)ts.nx[l] * ts.ny[l] * ts.nz[l];
  return cells * sizeof(T);
}

template <typename T>
bool tail_fits(const TailShape& ts, int s) {
  if (ts.nlev < 2 || ts.nlev > TAIL_MAX_LEVELS || s > TAIL_MAX_S) return false;
  const size_t top = (size_t)ts.nx[0] * ts.ny[0] * ts.nz[0];
  const size_t bottom = (size_t)ts.nx[ts.nlev - 1] * ts.ny[ts.nlev - 1] * ts.nz[ts.nlev - 1];
  if (top > (size_t)TAIL_MAX_CELLS || bottom > (size_t)(4 * WAVE)) return false;
  return tail_lds_bytes<T>(ts) <= TAIL_MAX_LDS;
}

// Raise the dynamic LDS limit of both tail kernels (once per process; a
// stream capture must not be the first caller).
void tail_prepare() {
  static bool done = false;
  if (done) return;
  (void)hipFuncSetAttribute((const void*)k_tail<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)TAIL_MAX_LDS);
  (void)hipFuncSetAttribute((const void*)k_tail<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)TAIL_MAX_LDS);
  done = true;
}

template <typename T>
void launch_tail(const TailShape& ts, const StageCoef* const* smooth, int s, int n_pre, int n_post, int periodic,
                 CoarseSchedule cs, double ctol, int cmax, const T* b_top, T* u_top, const int* stop,
                 hipStream_t st, const Batch& bt, int gs) {
  TailArgs<T> A;
  std::memset(&A, 0, sizeof(A));
  A.gs = gs;
  A.flat = ts.nz[0] == 1 && ts.ihz2[0] == 0.0 ? 1 : 0;
  A.nlev = ts.nlev;
  A.s = s;
  A.n_pre = n_pre;
  A.n_post = n_post;
  A.periodic = periodic;
  A.cmax = cmax;
  A.ctol = ctol;
  A.cs = cs;
  int off = 0;
  for (int l = 0; l < ts.nlev; ++l) {
    TailLevel<T>& V = A.lv[l];
    V.nx = ts.nx[l];
    V.ny = ts.ny[l];
    V.nz = ts.nz[l];
    V.off = off;
    off += 3 * V.nx * V.ny * V.nz;
    V.ihx2 = (T)ts.ihx2[l];
    V.ihy2 = (T)ts.ihy2[l];
    V.ihz2 = (T)ts.ihz2[l];
    V.gsc = (T)(1.0 / (2.0 * (ts.ihx2[l] + ts.ihy2[l] + ts.ihz2[l])));
    for (int j = 0; j < s; ++j) {
      V.mu[j] = (T)smooth[l][j].mu;
      V.nu[j] = (T)smooth[l][j].nu;
      V.c[j] = (T)smooth[l][j].c;
    }
  }
  const size_t shm = tail_lds_bytes<T>(ts);
  tail_prepare();
  hipLaunchKernelGGL(k_tail<T>, dim3(bt.nb), dim3(TNT), shm, st, A, b_top, u_top, bt, stop);
}

template bool tail_fits<double>(const TailShape&, int);
template bool tail_fits<float>(const TailShape&, int);
template void launch_tail<double>(const TailShape&, const StageCoef* const*, int, int, int, int, CoarseSchedule,
                                  double, int, const double*, double*, const int*, hipStream_t, const Batch&, int);
template void launch_tail<float>(const TailShape&, const StageCoef* const*, int, int, int, int, CoarseSchedule,
                                 double, int, const float*, float*, const int*, hipStream_t, const Batch&, int);

}  // namespace rkl
