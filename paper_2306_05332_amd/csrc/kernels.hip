// gfx950 kernels of the RKL-multigrid Poisson solver (memory-bound stencils,
// no matrix cores: every kernel streams HBM with 64-wide coalesced rows).
//
//   k_stage          one RKL stage (App. A eq. RKL_intermediate_source)
//   k_residual       r = b - M u with float64 partial sums of r^2 and r
//   k_resid_restrict b_{l+1} = R(b_l - M_l u_l) (Sec. 2.1 steps 2a/2b,
//                    eq. restriction_example_3D) with float64 r^2 partials and
//                    the coarse sum for the periodic mean removal (Sec. 2.3)
//   k_prolong_add    u_l += P(u_{l+1}) (eq. prolongation_example_3D)
//   k_reduce         fixed-order sum of per-block partials
//   k_scale / k_sub_mean / k_fill / k_add_cast / k_cast: elementwise helpers
#include "kernels.h"

namespace rkl {

// 3-D launch shape for z-marching stencil kernels: a 64 x 4 thread tile in
// (x, y), each thread walking KZ consecutive z planes so that the z
// neighbours stay in registers.
constexpr int TX = 64, TY = 4, KZ = 8;
constexpr int NT = TX * TY;

static inline dim3 grid3(int nx, int ny, int nz, int kz = KZ) {
  return dim3((nx + TX - 1) / TX, (ny + TY - 1) / TY, (nz + kz - 1) / kz);
}

// ---------------------------------------------------------------- RKL stage
// Y_j = mu * Y_{j-1} + nu * Y_{j-2} + c * (M Y_{j-1} - b), c = mu~_j tau.
// first != 0: Y_1 = Y_0 + c (M Y_0 - b) (ypp unused).  yout may alias ypp
// (each cell reads its own Y_{j-2} value before writing Y_j), never yp.
template <typename T>
__global__ __launch_bounds__(NT) void k_stage(LevelView<T> L, const T* __restrict__ yp,
                                              const T* ypp, const T* __restrict__ b, T* yout,
                                              T mu, T nu, T c, int first) {
  const int i = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int k0 = blockIdx.z * KZ;
  if (i >= L.nx || j >= L.ny) return;
  const int k1 = min(k0 + KZ, L.nz);
  const size_t sz = (size_t)L.nx * L.ny;
  for (int k = k0; k < k1; ++k) {
    const size_t idx = (size_t)k * sz + (size_t)j * L.nx + i;
    const T cv = yp[idx];
    const Nbrs<T> n = load_nbrs(L, yp, i, j, k, idx, cv);
    const T r = lap7(L, n, cv) - b[idx];
    T out;
    if (first) out = cv + c * r;
    else out = mu * cv + nu * ypp[idx] + c * r;
    yout[idx] = out;
  }
}

// ---------------------------------------------------------------- residual
// r = b - M u (u == nullptr means u = 0).  Writes r as TR when r_out != nullptr.
// part[2*blk] = sum r^2, part[2*blk+1] = sum r (float64, fixed order).
template <typename TU, typename TR>
__global__ __launch_bounds__(NT) void k_residual(LevelView<TU> L, const TU* __restrict__ u,
                                                 const TU* __restrict__ b, TR* __restrict__ r_out,
                                                 double* __restrict__ part) {
  __shared__ double sh[NT / WAVE];
  const int i = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int k0 = blockIdx.z * KZ;
  double s2 = 0.0, s1 = 0.0;
  if (i < L.nx && j < L.ny) {
    const int k1 = min(k0 + KZ, L.nz);
    const size_t sz = (size_t)L.nx * L.ny;
    for (int k = k0; k < k1; ++k) {
      const size_t idx = (size_t)k * sz + (size_t)j * L.nx + i;
      TU m;
      if (u) {
        const TU cv = u[idx];
        m = lap7(L, load_nbrs(L, u, i, j, k, idx, cv), cv);
      } else {
        // M 0: only the Dirichlet boundary terms 2 g / h^2 survive
        m = (TU)0;
        if (!L.periodic && L.faces) {
          Nbrs<TU> n = {0, 0, 0, 0, 0, 0};
          if (i == 0) n.xm = dir_ghost(L, 0, (size_t)k * L.ny + j, (TU)0);
          if (i == L.nx - 1) n.xp = dir_ghost(L, 1, (size_t)k * L.ny + j, (TU)0);
          if (j == 0) n.ym = dir_ghost(L, 2, (size_t)k * L.nx + i, (TU)0);
          if (j == L.ny - 1) n.yp = dir_ghost(L, 3, (size_t)k * L.nx + i, (TU)0);
          if (k == 0) n.zm = dir_ghost(L, 4, (size_t)j * L.nx + i, (TU)0);
          if (k == L.nz - 1) n.zp = dir_ghost(L, 5, (size_t)j * L.nx + i, (TU)0);
          m = lap7(L, n, (TU)0);
        }
      }
      const TU r = b[idx] - m;
      if (r_out) r_out[idx] = (TR)r;
      s2 += (double)r * (double)r;
      s1 += (double)r;
    }
  }
  const double t2 = block_sum<NT>(s2, sh);
  const double t1 = block_sum<NT>(s1, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    const size_t blk = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    part[2 * blk] = t2;
    part[2 * blk + 1] = t1;
  }
}

// ---------------------------------------------------------------- residual + restriction
// One thread per coarse cell: the residual b - M u of its 8 children, averaged
// (eq. restriction_example_3D).  part[2*blk] = sum over fine cells of r^2,
// part[2*blk+1] = sum of the coarse values written.
template <typename T>
__global__ __launch_bounds__(NT) void k_resid_restrict(LevelView<T> F, const T* __restrict__ u,
                                                       const T* __restrict__ b, T* __restrict__ bc,
                                                       double* __restrict__ part) {
  __shared__ double sh[NT / WAVE];
  const int cnx = F.nx / 2, cny = F.ny / 2, cnz = F.nz / 2;
  const int ic = blockIdx.x * TX + threadIdx.x;
  const int jc = blockIdx.y * TY + threadIdx.y;
  const int kc0 = blockIdx.z * KZ;
  double s2 = 0.0, s1 = 0.0;
  if (ic < cnx && jc < cny) {
    const int kc1 = min(kc0 + KZ, cnz);
    const size_t fsz = (size_t)F.nx * F.ny;
    for (int kc = kc0; kc < kc1; ++kc) {
      T acc = (T)0;
#pragma unroll
      for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) {
            const int i = 2 * ic + dx, j = 2 * jc + dy, k = 2 * kc + dz;
            const size_t idx = (size_t)k * fsz + (size_t)j * F.nx + i;
            const T cv = u[idx];
            const T r = b[idx] - lap7(F, load_nbrs(F, u, i, j, k, idx, cv), cv);
            acc += r;
            s2 += (double)r * (double)r;
          }
      const T v = acc * (T)0.125;
      bc[((size_t)kc * cny + jc) * cnx + ic] = v;
      s1 += (double)v;
    }
  }
  const double t2 = block_sum<NT>(s2, sh);
  const double t1 = block_sum<NT>(s1, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    const size_t blk = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    part[2 * blk] = t2;
    part[2 * blk + 1] = t1;
  }
}

// ---------------------------------------------------------------- prolongation + correction
// Coarse value at (I, J, K) with the error-equation ghosts: periodic wrap, or
// odd reflection per axis for homogeneous Dirichlet (eq. error_ghost applied
// along each axis the index leaves).
template <typename T>
__device__ __forceinline__ T coarse_at(const T* __restrict__ e, int I, int J, int K, int cnx,
                                       int cny, int cnz, int periodic) {
  T sgn = (T)1;
  if (periodic) {
    I = (I + cnx) % cnx;
    J = (J + cny) % cny;
    K = (K + cnz) % cnz;
  } else {
    if (I < 0) { I = 0; sgn = -sgn; }
    if (I >= cnx) { I = cnx - 1; sgn = -sgn; }
    if (J < 0) { J = 0; sgn = -sgn; }
    if (J >= cny) { J = cny - 1; sgn = -sgn; }
    if (K < 0) { K = 0; sgn = -sgn; }
    if (K >= cnz) { K = cnz - 1; sgn = -sgn; }
  }
  return sgn * e[((size_t)K * cny + J) * cnx + I];
}

// fine[i,j,k] += sum over the 8 nearest coarse cells of (w_x w_y w_z / 64) e,
// w = 3 on the parent's side, 1 on the neighbour's side.
template <typename T>
__global__ __launch_bounds__(NT) void k_prolong_add(int fnx, int fny, int fnz, int periodic,
                                                    const T* __restrict__ e, T* __restrict__ fine) {
  const int i = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int k0 = blockIdx.z * KZ;
  if (i >= fnx || j >= fny) return;
  const int cnx = fnx / 2, cny = fny / 2, cnz = fnz / 2;
  const int k1 = min(k0 + KZ, fnz);
  const int I = i >> 1, J = j >> 1;
  const int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1;
  for (int k = k0; k < k1; ++k) {
    const int K = k >> 1, sz = (k & 1) ? 1 : -1;
    T acc = (T)0;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          const T w = (T)((dz ? 1 : 3) * (dy ? 1 : 3) * (dx ? 1 : 3)) / (T)64;
          acc += w * coarse_at(e, I + dx * sx, J + dy * sy, K + dz * sz, cnx, cny, cnz, periodic);
        }
    const size_t idx = ((size_t)k * fny + j) * fnx + i;
    fine[idx] += acc;
  }
}

// ---------------------------------------------------------------- restriction alone
template <typename T>
__global__ __launch_bounds__(NT) void k_restrict(int fnx, int fny, int fnz, const T* __restrict__ fine,
                                                 T* __restrict__ coarse) {
  const int cnx = fnx / 2, cny = fny / 2, cnz = fnz / 2;
  const int ic = blockIdx.x * TX + threadIdx.x;
  const int jc = blockIdx.y * TY + threadIdx.y;
  const int kc0 = blockIdx.z * KZ;
  if (ic >= cnx || jc >= cny) return;
  const int kc1 = min(kc0 + KZ, cnz);
  for (int kc = kc0; kc < kc1; ++kc) {
    T acc = (T)0;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx)
          acc += fine[((size_t)(2 * kc + dz) * fny + (2 * jc + dy)) * fnx + (2 * ic + dx)];
    coarse[((size_t)kc * cny + jc) * cnx + ic] = acc * (T)0.125;
  }
}

// ---------------------------------------------------------------- reductions
// out[q] = sum over b of part[b * stride + q] for q < nq, in a fixed order.
constexpr int RED_NT = 1024;
__global__ __launch_bounds__(RED_NT) void k_reduce(const double* __restrict__ part, int nblk,
                                                   int stride, int nq, double* __restrict__ out) {
  __shared__ double sh[RED_NT / WAVE];
  for (int q = 0; q < nq; ++q) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += RED_NT) v += part[(size_t)b * stride + q];
    const double t = block_sum<RED_NT>(v, sh);
    if (threadIdx.x == 0) out[q] = t;
  }
}

// ---------------------------------------------------------------- elementwise
constexpr int EW_NT = 256;

template <typename T>
__global__ __launch_bounds__(EW_NT) void k_fill(T* __restrict__ a, size_t n, T v) {
  for (size_t q = (size_t)blockIdx.x * EW_NT + threadIdx.x; q < n; q += (size_t)gridDim.x * EW_NT)
    a[q] = v;
}

// out = c * in, with float64 block partial sums of out into part[blk]
__global__ __launch_bounds__(EW_NT) void k_scale(const double* __restrict__ in, double* __restrict__ out,
                                                 size_t n, double c, double* __restrict__ part) {
  __shared__ double sh[EW_NT / WAVE];
  double s = 0.0;
  for (size_t q = (size_t)blockIdx.x * EW_NT + threadIdx.x; q < n; q += (size_t)gridDim.x * EW_NT) {
    const double v = c * in[q];
    out[q] = v;
    s += v;
  }
  const double t = block_sum<EW_NT>(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// a -= sum[0] / count
template <typename T>
__global__ __launch_bounds__(EW_NT) void k_sub_mean(T* __restrict__ a, size_t n,
                                                    const double* __restrict__ sum, double count) {
  const T m = (T)(sum[0] / count);
  for (size_t q = (size_t)blockIdx.x * EW_NT + threadIdx.x; q < n; q += (size_t)gridDim.x * EW_NT)
    a[q] -= m;
}

// part[blk] = float64 sum of a over the block's share
template <typename T>
__global__ __launch_bounds__(EW_NT) void k_sum(const T* __restrict__ a, size_t n, double* __restrict__ part) {
  __shared__ double sh[EW_NT / WAVE];
  double s = 0.0;
  for (size_t q = (size_t)blockIdx.x * EW_NT + threadIdx.x; q < n; q += (size_t)gridDim.x * EW_NT)
    s += (double)a[q];
  const double t = block_sum<EW_NT>(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// u64 += (double) e
template <typename TE>
__global__ __launch_bounds__(EW_NT) void k_add_cast(double* __restrict__ u, const TE* __restrict__ e,
                                                    size_t n) {
  for (size_t q = (size_t)blockIdx.x * EW_NT + threadIdx.x; q < n; q += (size_t)gridDim.x * EW_NT)
    u[q] += (double)e[q];
}

// ================================================================ launchers
static inline unsigned ew_blocks(size_t n) {
  size_t b = (n + EW_NT - 1) / EW_NT;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}

size_t stencil_blocks(int nx, int ny, int nz) {
  dim3 g = grid3(nx, ny, nz);
  return (size_t)g.x * g.y * g.z;
}

size_t ew_block_count(size_t n) { return ew_blocks(n); }

template <typename T>
void launch_stage(const LevelView<T>& L, const T* yp, const T* ypp, const T* b, T* yout, double mu,
                  double nu, double c, int first, hipStream_t st) {
  hipLaunchKernelGGL(k_stage<T>, grid3(L.nx, L.ny, L.nz), dim3(TX, TY), 0, st, L, yp, ypp, b, yout,
                     (T)mu, (T)nu, (T)c, first);
}

template <typename TU, typename TR>
void launch_residual(const LevelView<TU>& L, const TU* u, const TU* b, TR* r_out, double* part,
                     hipStream_t st) {
  hipLaunchKernelGGL((k_residual<TU, TR>), grid3(L.nx, L.ny, L.nz), dim3(TX, TY), 0, st, L, u, b,
                     r_out, part);
}

template <typename T>
void launch_resid_restrict(const LevelView<T>& F, const T* u, const T* b, T* bc, double* part,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_resid_restrict<T>, grid3(F.nx / 2, F.ny / 2, F.nz / 2), dim3(TX, TY), 0, st, F,
                     u, b, bc, part);
}

template <typename T>
void launch_prolong_add(int fnx, int fny, int fnz, int periodic, const T* e, T* fine, hipStream_t st) {
  hipLaunchKernelGGL(k_prolong_add<T>, grid3(fnx, fny, fnz), dim3(TX, TY), 0, st, fnx, fny, fnz,
                     periodic, e, fine);
}

template <typename T>
void launch_restrict(int fnx, int fny, int fnz, const T* fine, T* coarse, hipStream_t st) {
  hipLaunchKernelGGL(k_restrict<T>, grid3(fnx / 2, fny / 2, fnz / 2), dim3(TX, TY), 0, st, fnx, fny,
                     fnz, fine, coarse);
}

void launch_reduce(const double* part, int nblk, int stride, int nq, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(RED_NT), 0, st, part, nblk, stride, nq, out);
}

template <typename T>
void launch_fill(T* a, size_t n, T v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill<T>, dim3(ew_blocks(n)), dim3(EW_NT), 0, st, a, n, v);
}

void launch_scale(const double* in, double* out, size_t n, double c, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_scale, dim3(ew_blocks(n)), dim3(EW_NT), 0, st, in, out, n, c, part);
}

template <typename T>
void launch_sub_mean(T* a, size_t n, const double* sum, double count, hipStream_t st) {
  hipLaunchKernelGGL(k_sub_mean<T>, dim3(ew_blocks(n)), dim3(EW_NT), 0, st, a, n, sum, count);
}

template <typename T>
void launch_sum(const T* a, size_t n, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_sum<T>, dim3(ew_blocks(n)), dim3(EW_NT), 0, st, a, n, part);
}

template <typename TE>
void launch_add_cast(double* u, const TE* e, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_add_cast<TE>, dim3(ew_blocks(n)), dim3(EW_NT), 0, st, u, e, n);
}

// explicit instantiations
template void launch_stage<double>(const LevelView<double>&, const double*, const double*, const double*,
                                   double*, double, double, double, int, hipStream_t);
template void launch_stage<float>(const LevelView<float>&, const float*, const float*, const float*,
                                  float*, double, double, double, int, hipStream_t);
template void launch_residual<double, double>(const LevelView<double>&, const double*, const double*,
                                              double*, double*, hipStream_t);
template void launch_residual<double, float>(const LevelView<double>&, const double*, const double*,
                                             float*, double*, hipStream_t);
template void launch_residual<float, float>(const LevelView<float>&, const float*, const float*, float*,
                                            double*, hipStream_t);
template void launch_resid_restrict<double>(const LevelView<double>&, const double*, const double*,
                                            double*, double*, hipStream_t);
template void launch_resid_restrict<float>(const LevelView<float>&, const float*, const float*, float*,
                                           double*, hipStream_t);
template void launch_prolong_add<double>(int, int, int, int, const double*, double*, hipStream_t);
template void launch_prolong_add<float>(int, int, int, int, const float*, float*, hipStream_t);
template void launch_restrict<double>(int, int, int, const double*, double*, hipStream_t);
template void launch_fill<double>(double*, size_t, double, hipStream_t);
template void launch_fill<float>(float*, size_t, float, hipStream_t);
template void launch_sub_mean<double>(double*, size_t, const double*, double, hipStream_t);
template void launch_sub_mean<float>(float*, size_t, const double*, double, hipStream_t);
template void launch_sum<double>(const double*, size_t, double*, hipStream_t);
template void launch_sum<float>(const float*, size_t, double*, hipStream_t);
template void launch_add_cast<float>(double*, const float*, size_t, hipStream_t);
template void launch_add_cast<double>(double*, const double*, size_t, hipStream_t);

}  // namespace rkl
