// Coarsest-grid solver: the accelerated RKL iteration (App. A.4) on a level
// small enough to live in one workgroup's LDS.
//
// Stage counts follow the schedule built on the host (per-mode optimal s from
// the first zero of J0, eq. sk_optimal, walking k = n/2 .. 1 and skipping
// repeats; the last entry repeats).  The iterate starts from u_in (or zero).  Before every tau-step the residual
// ||M u - b|| is compared with tol * ref (ref = ||b|| unless given), as in the
// paper's "while (res > tol)" loop.  Periodic levels drop the mean of u after
// each step.  All sums are float64 and fixed-order.
#include "kernels.h"

namespace rkl {


template <typename T>
__device__ __forceinline__ void cell_ijk(int q, int nx, int ny, int& i, int& j, int& k) {
  i = q % nx;
  const int t = q / nx;
  j = t % ny;
  k = t / ny;
}

// CNT threads: one wavefront for levels of up to 256 cells (barriers and
// reductions stay inside the wave), four wavefronts above.
template <typename T, int CNT>
__global__ __launch_bounds__(CNT) void k_coarse_solve(LevelView<T> L, const T* __restrict__ b,
                                                      const T* __restrict__ u_in,
                                                      T* __restrict__ u_out, CoarseSchedule cs,
                                                      double tol, double ref_norm, int max_steps,
                                                      int remove_mean, int* steps_out,
                                                      double* res_out, const int* __restrict__ stop) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[CNT / WAVE];
  __shared__ double bcast;
  // schedule and stage coefficients cached in LDS (read once per stage)
  __shared__ int ssched[COARSE_MAX_SCHED];
  __shared__ int scoff[COARSE_MAX_SCHED];
  __shared__ double scoef[3 * COARSE_MAX_COEF];
  lds_poison(reinterpret_cast<T*>(smem_raw), 3 * L.nx * L.ny * L.nz);
  lds_poison(red, CNT / WAVE);
  lds_poison(scoef, 3 * COARSE_MAX_COEF);
  lds_poison_sync();
  if (stop != nullptr && *stop) return;
  const int nsched = min(cs.nsched, COARSE_MAX_SCHED);
  for (int q = threadIdx.x; q < nsched; q += CNT) {
    ssched[q] = cs.sched[q];
    scoff[q] = cs.coff[q];
  }
  const int ncoef = nsched > 0 ? min(cs.coff[nsched - 1] + cs.sched[nsched - 1], COARSE_MAX_COEF) : 0;
  for (int q = threadIdx.x; q < 3 * ncoef; q += CNT) scoef[q] = cs.coef[q];
  const int N = L.nx * L.ny * L.nz;
  T* A = reinterpret_cast<T*>(smem_raw);
  T* B = A + N;
  T* Bv = B + N;
  const int tid = threadIdx.x;

  double s2 = 0.0;
  for (int q = tid; q < N; q += CNT) {
    const T v = b[q];
    Bv[q] = v;
    A[q] = u_in ? u_in[q] : (T)0;
    s2 += (double)v * (double)v;
  }
  double t = block_sum<CNT>(s2, red);
  if (tid == 0) bcast = t;
  __syncthreads();
  const double bnorm = sqrt(bcast);
  const double ref = ref_norm > 0.0 ? ref_norm : bnorm;

  T* cur = A;
  T* alt = B;
  int step = 0;
  double res = 0.0;
  if (ref_norm > 0.0 || bnorm > 0.0) {
    while (true) {
      // residual check
      double r2 = 0.0;
      for (int q = tid; q < N; q += CNT) {
        int i, j, k;
        cell_ijk<T>(q, L.nx, L.ny, i, j, k);
        const T cv = cur[q];
        const T r = lap7(L, load_nbrs(L, cur, i, j, k, (size_t)q, cv), cv) - Bv[q];
        r2 += (double)r * (double)r;
      }
      t = block_sum<CNT>(r2, red);
      if (tid == 0) bcast = t;
      __syncthreads();
      res = sqrt(bcast);
      if (res <= tol * ref || step >= max_steps) break;

      const int qs = step < nsched ? step : nsched - 1;
      const int s = ssched[qs];
      const double* co = scoef + 3 * scoff[qs];
      // stages: Y_1 -> alt; Y_j overwrites Y_{j-2}
      for (int jst = 1; jst <= s; ++jst) {
        const T mu = (T)co[3 * (jst - 1) + 0];
        const T nu = (T)co[3 * (jst - 1) + 1];
        const T c = (T)co[3 * (jst - 1) + 2];
        // Y_{j-1} lives in `cur` for odd j, in `alt` for even j (Y_0 in cur)
        const T* yp = (jst & 1) ? cur : alt;
        T* yw = (jst & 1) ? alt : cur;  // Y_{j-2} slot (or the free slot for j = 1)
        for (int q = tid; q < N; q += CNT) {
          int i, j, k;
          cell_ijk<T>(q, L.nx, L.ny, i, j, k);
          const T cv = yp[q];
          const T r = lap7(L, load_nbrs(L, yp, i, j, k, (size_t)q, cv), cv) - Bv[q];
          yw[q] = (jst == 1) ? cv + c * r : mu * cv + nu * yw[q] + c * r;
        }
        __syncthreads();
      }
      if (s & 1) {
        T* tmp = cur;
        cur = alt;
        alt = tmp;
      }
      if (remove_mean) {
        double sm = 0.0;
        for (int q = tid; q < N; q += CNT) sm += (double)cur[q];
        t = block_sum<CNT>(sm, red);
        if (tid == 0) bcast = t;
        __syncthreads();
        const T m = (T)(bcast / (double)N);
        for (int q = tid; q < N; q += CNT) cur[q] -= m;
        __syncthreads();
      }
      ++step;
    }
  }
  for (int q = tid; q < N; q += CNT) u_out[q] = cur[q];
  if (tid == 0) {
    if (steps_out) *steps_out = step;
    if (res_out) *res_out = res;
  }
}

// ---------------------------------------------------------------- one-wavefront variant
// Levels of at most 256 cells without Dirichlet data (the coarsest level of
// a V-cycle): one wavefront, CPL cells per lane, the six neighbour indices of
// every cell precomputed once (-1 marks the homogeneous ghost -c), sums by a
// fixed xor butterfly across the wavefront.  A lone wavefront cannot hide
// instruction latency behind other waves, so the loop body is kept short.
template <int CPL>
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

template <typename T, int CPL>
__global__ __launch_bounds__(WAVE) void k_coarse_wave(LevelView<T> L, const T* __restrict__ b,
                                                      T* __restrict__ u_out, CoarseSchedule cs, double tol,
                                                      int max_steps, int remove_mean, int* steps_out,
                                                      const int* __restrict__ stop) {
  __shared__ T A[WAVE * CPL], B[WAVE * CPL];
  __shared__ int ssched[COARSE_MAX_SCHED];
  __shared__ int scoff[COARSE_MAX_SCHED];
  __shared__ double scoef[3 * COARSE_MAX_COEF];
  lds_poison(A, WAVE * CPL);
  lds_poison(B, WAVE * CPL);
  lds_poison(scoef, 3 * COARSE_MAX_COEF);
  lds_poison_sync();
  if (stop != nullptr && *stop) return;
  const int lane = threadIdx.x;
  const int nx = L.nx, ny = L.ny, nz = L.nz, N = nx * ny * nz;
  const int nsched = min(cs.nsched, COARSE_MAX_SCHED);
  for (int q = lane; q < nsched; q += WAVE) {
    ssched[q] = cs.sched[q];
    scoff[q] = cs.coff[q];
  }
  const int ncoef = nsched > 0 ? min(cs.coff[nsched - 1] + cs.sched[nsched - 1], COARSE_MAX_COEF) : 0;
  for (int q = lane; q < 3 * ncoef; q += WAVE) scoef[q] = cs.coef[q];
  int nb[CPL][6];
  bool on[CPL];
  T bv[CPL];
  double b2 = 0.0;
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int q = lane + WAVE * c;
    on[c] = q < N;
    bv[c] = (T)0;
    for (int d = 0; d < 6; ++d) nb[c][d] = -1;
    if (on[c]) {
      const int i = q % nx, j = (q / nx) % ny, k = q / (nx * ny);
      const int sy = nx, sz = nx * ny;
      const bool per = L.periodic != 0;
      nb[c][0] = i > 0 ? q - 1 : (per ? q + nx - 1 : -1);
      nb[c][1] = i < nx - 1 ? q + 1 : (per ? q - (nx - 1) : -1);
      nb[c][2] = j > 0 ? q - sy : (per ? q + (ny - 1) * sy : -1);
      nb[c][3] = j < ny - 1 ? q + sy : (per ? q - (ny - 1) * sy : -1);
      nb[c][4] = k > 0 ? q - sz : (per ? q + (nz - 1) * sz : -1);
      nb[c][5] = k < nz - 1 ? q + sz : (per ? q - (nz - 1) * sz : -1);
      bv[c] = b[q];
      A[q] = (T)0;
      b2 += (double)bv[c] * (double)bv[c];
    }
  }
  const double bnorm = sqrt(wave_sum<CPL>(b2));
  __syncthreads();
  T* cur = A;
  T* alt = B;
  auto lapr = [&](const T* Y, int c, T cv) -> T {
    T n6[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) n6[d] = nb[c][d] >= 0 ? Y[nb[c][d]] : -cv;
    return ((n6[0] + n6[1]) - (T)2 * cv) * L.ihx2 + ((n6[2] + n6[3]) - (T)2 * cv) * L.ihy2 +
           ((n6[4] + n6[5]) - (T)2 * cv) * L.ihz2 - bv[c];
  };
  int step = 0;
  if (bnorm > 0.0) {
    T rchk[CPL];  // the stop test's M u - b, which is also the first stage's
    while (true) {
      double r2 = 0.0;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        rchk[c] = (T)0;
        if (!on[c]) continue;
        const int q = lane + WAVE * c;
        const T r = lapr(cur, c, cur[q]);
        rchk[c] = r;
        r2 += (double)r * (double)r;
      }
      const double res = sqrt(wave_sum<CPL>(r2));
      if (res <= tol * bnorm || step >= max_steps) break;
      const int qs = step < nsched ? step : nsched - 1;
      const int s = ssched[qs];
      const double* co = scoef + 3 * scoff[qs];
      for (int jst = 1; jst <= s; ++jst) {
        const T mu = (T)co[3 * (jst - 1)], nu = (T)co[3 * (jst - 1) + 1], cc = (T)co[3 * (jst - 1) + 2];
        const T* yp = (jst & 1) ? cur : alt;
        T* yw = (jst & 1) ? alt : cur;
        T outv[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          const int q = lane + WAVE * c;
          outv[c] = (T)0;
          if (!on[c]) continue;
          const T cv = yp[q];
          const T r = jst == 1 ? rchk[c] : lapr(yp, c, cv);
          outv[c] = (jst == 1) ? cv + cc * r : mu * cv + nu * yw[q] + cc * r;
        }
#pragma unroll
        for (int c = 0; c < CPL; ++c)
          if (on[c]) yw[lane + WAVE * c] = outv[c];
        __syncthreads();
      }
      if (s & 1) {
        T* t = cur;
        cur = alt;
        alt = t;
      }
      if (remove_mean) {
        double sm = 0.0;
#pragma unroll
        for (int c = 0; c < CPL; ++c)
          if (on[c]) sm += (double)cur[lane + WAVE * c];
        const T m = (T)(wave_sum<CPL>(sm) / (double)N);
#pragma unroll
        for (int c = 0; c < CPL; ++c)
          if (on[c]) cur[lane + WAVE * c] -= m;
        __syncthreads();
      }
      ++step;
    }
  }
#pragma unroll
  for (int c = 0; c < CPL; ++c)
    if (on[c]) u_out[lane + WAVE * c] = cur[lane + WAVE * c];
  if (lane == 0 && steps_out) *steps_out = step;
}

template <typename T>
void launch_coarse_solve(const LevelView<T>& L, const T* b, const T* u_in, T* u, CoarseSchedule cs,
                         double tol, double ref_norm, int max_steps, int remove_mean, int* steps_out,
                         double* res_out, const int* stop, hipStream_t st) {
  const size_t N = (size_t)L.nx * L.ny * L.nz;
  const size_t shm = 3 * N * sizeof(T);
  if (L.faces == nullptr && u_in == nullptr && res_out == nullptr && ref_norm <= 0.0 && N <= 4 * WAVE) {
    if (N <= WAVE)
      hipLaunchKernelGGL((k_coarse_wave<T, 1>), dim3(1), dim3(WAVE), 0, st, L, b, u, cs, tol, max_steps,
                         remove_mean, steps_out, stop);
    else
      hipLaunchKernelGGL((k_coarse_wave<T, 4>), dim3(1), dim3(WAVE), 0, st, L, b, u, cs, tol, max_steps,
                         remove_mean, steps_out, stop);
    return;
  }
  if (N <= 256)
    hipLaunchKernelGGL((k_coarse_solve<T, 64>), dim3(1), dim3(64), shm, st, L, b, u_in, u, cs, tol, ref_norm,
                       max_steps, remove_mean, steps_out, res_out, stop);
  else
    hipLaunchKernelGGL((k_coarse_solve<T, 256>), dim3(1), dim3(256), shm, st, L, b, u_in, u, cs, tol,
                       ref_norm, max_steps, remove_mean, steps_out, res_out, stop);
}

template void launch_coarse_solve<double>(const LevelView<double>&, const double*, const double*, double*,
                                          CoarseSchedule, double, double, int, int, int*, double*,
                                          const int*, hipStream_t);
template void launch_coarse_solve<float>(const LevelView<float>&, const float*, const float*, float*, CoarseSchedule,
                                         double, double, int, int, int*, double*, const int*, hipStream_t);

}  // namespace rkl
