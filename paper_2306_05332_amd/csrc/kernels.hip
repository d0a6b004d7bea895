// gfx950 kernels of the RKL-multigrid Poisson solver (memory-bound stencils,
// no matrix cores: every kernel streams HBM with 64-wide coalesced rows).
//
//   k_stage          one RKL stage (App. A eq. RKL_intermediate_source), used
//                    on levels too small for the fused tau-step
//   k_restrict       8-point average (eq. restriction_example_3D); 4-point
//                    (eq. restriction_example_2D) for a one-plane fine grid
//   k_reduce         fixed-order sum of per-block partials
//   k_check          convergence test of the V-cycle loop on the device
//   k_scale / k_sub_mean / k_copy_sub_mean / k_fill / k_sum / k_add_cast:
//                    elementwise helpers
// Kernels launched inside a V-cycle take `stop`: once the device-side
// convergence test has set it, they return at once (the host may have queued
// more cycles than were needed).
#include "kernels.h"

#include <algorithm>

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
                                              T mu, T nu, T c, int first, int kz, const int* __restrict__ stop) {
  if (stop != nullptr && *stop) return;
  const int i = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int k0 = blockIdx.z * kz;
  if (i >= L.nx || j >= L.ny) return;
  const int k1 = min(k0 + kz, L.nz);
  const size_t sz = (size_t)L.nx * L.ny;
  for (int k = k0; k < k1; ++k) {
    const size_t idx = (size_t)k * sz + (size_t)j * L.nx + i;
    T cv = (T)0, lap = (T)0;
    if (yp != nullptr) {  // yp == nullptr: the iterate is zero (homogeneous ghosts)
      cv = yp[idx];
      lap = lap7(L, load_nbrs(L, yp, i, j, k, idx, cv), cv);
    }
    const T r = lap - b[idx];
    T out;
    if (first) out = cv + c * r;
    else out = mu * cv + nu * ypp[idx] + c * r;
    yout[idx] = out;
  }
}

// ---------------------------------------------------------------- red-black Gauss-Seidel, one colour
// uout = uin, then the cells with (i + j + k) % 2 == colour get
// u + (omega / D_cell)(M u - b) evaluated on uin (Sec. 2.2.4); D_cell = 2 sum
// h^-2 plus h_d^-2 per Dirichlet face of the cell (the operator's diagonal).
template <typename T>
__global__ __launch_bounds__(256) void k_gsrb_half(LevelView<T> L, const T* __restrict__ uin, T* __restrict__ uout,
                                                   const T* __restrict__ b, int colour, T coef, Batch bt,
                                                   const int* __restrict__ stop) {
  {
    const long long mb = blockIdx.y;
    uin += mb * bt.s0;
    uout += mb * bt.s0;
    b += mb * bt.s0;
    if (stop != nullptr) stop += mb * bt.stop_stride;
  }
  if (stop != nullptr && *stop) return;
  const size_t n = (size_t)L.nx * L.ny * L.nz;
  for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (size_t)gridDim.x * 256) {
    const int i = (int)(q % L.nx), j = (int)((q / L.nx) % L.ny), k = (int)(q / ((size_t)L.nx * L.ny));
    const T c = uin[q];
    T y = c;
    if (((i + j + k) & 1) == colour) {
      T cf = coef;
      if (!L.periodic) {
        const T d = (T)2 * (L.ihx2 + L.ihy2 + L.ihz2);
        T extra = (T)0;
        if (i == 0) extra += L.ihx2;
        if (i == L.nx - 1) extra += L.ihx2;
        if (j == 0) extra += L.ihy2;
        if (j == L.ny - 1) extra += L.ihy2;
        if (k == 0) extra += L.ihz2;
        if (k == L.nz - 1) extra += L.ihz2;
        if (extra != (T)0) cf = coef * d / (d + extra);
      }
      y = c + cf * (lap7(L, load_nbrs(L, uin, i, j, k, q, c), c) - b[q]);
    }
    uout[q] = y;
  }
}

// ---------------------------------------------------------------- Dirichlet data into the right-hand side
// The finest-level ghost 2 g - u (Sec. 2.3, eq. solution_ghost) contributes
// 2 g h_d^-2 to (M u) at a face cell plus the homogeneous part -u h_d^-2, so
// M u - f = M_0 u - (f - sum 2 g h_d^-2) with M_0 the operator with ghost -u.
// dst = src minus those terms (dst may be src).
__global__ __launch_bounds__(NT) void k_fold_faces(int nx, int ny, int nz, double ihx2, double ihy2, double ihz2,
                                                   const double* __restrict__ faces, const double* src, double* dst,
                                                   int kz) {
  const int i = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int k0 = blockIdx.z * kz;
  if (i >= nx || j >= ny) return;
  const int k1 = min(k0 + kz, nz);
  for (int k = k0; k < k1; ++k) {
    const size_t c = ((size_t)k * ny + j) * nx + i;
    double t = 0.0;
    if (i == 0) t += faces[face_off(0, nx, ny, nz) + (size_t)k * ny + j] * ihx2;
    if (i == nx - 1) t += faces[face_off(1, nx, ny, nz) + (size_t)k * ny + j] * ihx2;
    if (j == 0) t += faces[face_off(2, nx, ny, nz) + (size_t)k * nx + i] * ihy2;
    if (j == ny - 1) t += faces[face_off(3, nx, ny, nz) + (size_t)k * nx + i] * ihy2;
    if (k == 0) t += faces[face_off(4, nx, ny, nz) + (size_t)j * nx + i] * ihz2;
    if (k == nz - 1) t += faces[face_off(5, nx, ny, nz) + (size_t)j * nx + i] * ihz2;
    if (t != 0.0 || src != dst) dst[c] = src[c] - 2.0 * t;
  }
}

// ---------------------------------------------------------------- acceleration g = -grad(phi)
// 4th-order differences (Sec. 3, eq. 4thorder_acceleration) with two ghost
// layers: periodic wrap, or odd reflection about the Dirichlet face value g
// (phi_{-m} = 2 g - phi_{m-1}, m = 1, 2; g = 0 without face data).  ihz = 0
// (hz = inf, a two-dimensional grid) gives g_z = 0 without z reads.
__global__ __launch_bounds__(NT) void k_gradient(int nx, int ny, int nz, double ihx, double ihy, double ihz,
                                                 int periodic, const double* __restrict__ faces,
                                                 const double* __restrict__ phi, double* __restrict__ gx,
                                                 double* __restrict__ gy, double* __restrict__ gz, int kz) {
  const int i = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int k0 = blockIdx.z * kz;
  if (i >= nx || j >= ny) return;
  const int k1 = min(k0 + kz, nz);
  const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
  auto fv = [&](int face, size_t idx) -> double {
    return faces != nullptr ? faces[face_off(face, nx, ny, nz) + idx] : 0.0;
  };
  for (int k = k0; k < k1; ++k) {
    const size_t c = (size_t)k * sz + (size_t)j * sy + i;
    // value at offset d in {-2,-1,1,2} along an axis of length n at position p
    auto along = [&](int p, int n, int d, size_t stride, int flo, int fhi, size_t fidx) -> double {
      const int q = p + d;
      if (q >= 0 && q < n) return phi[c + (ptrdiff_t)d * (ptrdiff_t)stride];
      if (periodic) {
        const int w = ((q % n) + n) % n;  // also for axes shorter than the stencil
        return phi[c + (ptrdiff_t)(w - p) * (ptrdiff_t)stride];
      }
      if (q < 0) {
        const int m = -q;  // ghost layer m: mirror cell m - 1
        return 2.0 * fv(flo, fidx) - phi[c + (ptrdiff_t)(m - 1 - p) * (ptrdiff_t)stride];
      }
      const int m = q - (n - 1);  // mirror cell n - m
      return 2.0 * fv(fhi, fidx) - phi[c + (ptrdiff_t)(n - m - p) * (ptrdiff_t)stride];
    };
    auto deriv = [&](double m2, double m1, double p1, double p2, double ih) {
      return -(4.0 / 3.0) * (p1 - m1) * (0.5 * ih) + (1.0 / 3.0) * (p2 - m2) * (0.25 * ih);
    };
    const size_t fx = (size_t)k * ny + j, fy = (size_t)k * nx + i, fz = (size_t)j * nx + i;
    gx[c] = deriv(along(i, nx, -2, 1, 0, 1, fx), along(i, nx, -1, 1, 0, 1, fx), along(i, nx, 1, 1, 0, 1, fx),
                  along(i, nx, 2, 1, 0, 1, fx), ihx);
    gy[c] = deriv(along(j, ny, -2, sy, 2, 3, fy), along(j, ny, -1, sy, 2, 3, fy), along(j, ny, 1, sy, 2, 3, fy),
                  along(j, ny, 2, sy, 2, 3, fy), ihy);
    if (ihz == 0.0)
      gz[c] = 0.0;
    else
      gz[c] = deriv(along(k, nz, -2, sz, 4, 5, fz), along(k, nz, -1, sz, 4, 5, fz), along(k, nz, 1, sz, 4, 5, fz),
                    along(k, nz, 2, sz, 4, 5, fz), ihz);
  }
}

// ---------------------------------------------------------------- max |M u - b|
template <typename T>
__global__ __launch_bounds__(256) void k_resid_absmax(LevelView<T> L, const T* __restrict__ u,
                                                      const T* __restrict__ b, double* __restrict__ part) {
  __shared__ double sh[256];
  const size_t n = (size_t)L.nx * L.ny * L.nz;
  double m = 0.0;
  for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (size_t)gridDim.x * 256) {
    const int i = (int)(q % L.nx), j = (int)((q / L.nx) % L.ny), k = (int)(q / ((size_t)L.nx * L.ny));
    const T c = u[q];
    const double r = (double)(lap7(L, load_nbrs(L, u, i, j, k, q, c), c) - b[q]);
    m = fmax(m, fabs(r));
    if (r != r) m = r;  // keep a NaN visible
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double a = sh[threadIdx.x], c = sh[threadIdx.x + w];
      sh[threadIdx.x] = (a != a || c != c) ? (a + c) : fmax(a, c);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_reduce_max(const double* __restrict__ part, int nblk, double* __restrict__ out) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int q = threadIdx.x; q < nblk; q += 256) {
    const double v = part[q];
    m = (v != v || m != m) ? (v + m) : fmax(m, v);
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double a = sh[threadIdx.x], c = sh[threadIdx.x + w];
      sh[threadIdx.x] = (a != a || c != c) ? (a + c) : fmax(a, c);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// ---------------------------------------------------------------- restriction alone
template <typename T>
__global__ __launch_bounds__(NT) void k_restrict(int fnx, int fny, int fnz, const T* __restrict__ fine,
                                                 T* __restrict__ coarse) {
  const bool flat = fnz == 1;
  const int cnx = fnx / 2, cny = fny / 2, cnz = flat ? 1 : fnz / 2;
  const int ic = blockIdx.x * TX + threadIdx.x;
  const int jc = blockIdx.y * TY + threadIdx.y;
  const int kc0 = blockIdx.z * KZ;
  if (ic >= cnx || jc >= cny) return;
  const int kc1 = min(kc0 + KZ, cnz);
  for (int kc = kc0; kc < kc1; ++kc) {
    T acc = (T)0;
    for (int dz = 0; dz < (flat ? 1 : 2); ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx)
          acc += fine[((size_t)(2 * kc + dz) * fny + (2 * jc + dy)) * fnx + (2 * ic + dx)];
    coarse[((size_t)kc * cny + jc) * cnx + ic] = acc * (flat ? (T)0.25 : (T)0.125);
  }
}

// ---------------------------------------------------------------- reductions
// out[q] = sum over b of part[b * stride + q] for q < nq, in a fixed order.
constexpr int RED_NT = 1024;
__global__ __launch_bounds__(RED_NT) void k_reduce(const double* __restrict__ part, int nblk,
                                                   int stride, int nq, double* __restrict__ out,
                                                   Batch bt, const int* __restrict__ stop) {
  __shared__ double sh[RED_NT / WAVE];
  {
    const long long mb = blockIdx.x;  // one workgroup per member; out stride s0
    part += mb * bt.part_stride;
    out += mb * bt.s0;
    if (stop != nullptr) stop += mb * bt.stop_stride;
  }
  if (stop != nullptr && *stop) return;
  for (int q = 0; q < nq; ++q) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += RED_NT) v += part[(size_t)b * stride + q];
    const double t = block_sum<RED_NT>(v, sh);
    if (threadIdx.x == 0) out[q] = t;
  }
}

// ---------------------------------------------------------------- convergence test
// One block: rel = sqrt(sum of part[b * stride]) / sqrt(res0sq) for the state at the
// start of cycle cs->m; records it and decides, in this order:
// non-finite -> RKL_ENONFINITE; rel <= tol -> done; three consecutive
// increases that end above twice the best residual so far -> RKL_EDIVERGED;
// with tol > 0, the last eight states all above 0.9 of the best state
// before them (the residual has stopped falling, as it does at the float64
// rounding floor of M u - f, about eps Lambda ||u|| / ||f||) -> RKL_ENOCONV,
// marked stalled (tol = 0 asks for exactly max_cycles cycles);
// m >= max_cycles -> RKL_ENOCONV.  Also stores the mean of the residual
// (part[b * stride + 1] / count) as a diagnostic.
__global__ __launch_bounds__(RED_NT) void k_check(const double* __restrict__ part, int nblk, int stride,
                                                  const double* __restrict__ res0sq, double tol,
                                                  int max_cycles, double count, ConvState* __restrict__ cs,
                                                  Batch bt) {
  __shared__ double sh[RED_NT / WAVE];
  {
    const long long mb = blockIdx.x;  // one workgroup per member
    part += mb * bt.part_stride;
    res0sq += mb;
    cs += mb;
  }
  if (cs->stop) return;
  double v2 = 0.0, v1 = 0.0;
  for (int b = threadIdx.x; b < nblk; b += RED_NT) {
    v2 += part[(size_t)b * stride];
    if (stride > 1) v1 += part[(size_t)b * stride + 1];
  }
  const double t2 = block_sum<RED_NT>(v2, sh);
  const double t1 = block_sum<RED_NT>(v1, sh);
  if (threadIdx.x != 0) return;
  const int m = cs->m;
  const double rel = sqrt(t2) / sqrt(res0sq[0]);
  cs->mean = t1 / count;
  if (m < CONV_HIST) cs->hist[m] = rel;
  cs->last[m & 3] = rel;
  // best residual up to the first of the last four states (three increases)
  // and before the last eight states (stall window)
  constexpr int SW = 8;
  double best3 = HUGE_VAL, bestw = HUGE_VAL;
  const int hmax = m < CONV_HIST ? m : CONV_HIST;
  for (int q = 0; q < hmax; ++q) {
    if (q <= m - 3) best3 = fmin(best3, cs->hist[q]);
    if (q <= m - SW) bestw = fmin(bestw, cs->hist[q]);
  }
  double recent = rel;
  for (int q = m - SW + 1; q < m; ++q)
    if (q >= 0 && q < CONV_HIST) recent = fmin(recent, cs->hist[q]);
  int status = 1;  // 1: keep going
  int stalled = 0;
  if (!isfinite(rel)) status = -5;
  else if (rel <= tol) status = 0;
  else if (m >= 3 && cs->last[m & 3] > cs->last[(m - 1) & 3] && cs->last[(m - 1) & 3] > cs->last[(m - 2) & 3] &&
           cs->last[(m - 2) & 3] > cs->last[(m - 3) & 3] && rel > 2.0 * best3)
    status = -4;
  else if (tol > 0.0 && m >= SW && m < CONV_HIST && recent > 0.9 * bestw) {
    status = -3;
    stalled = 1;
  } else if (m >= max_cycles) status = -3;
  cs->rel = rel;
  if (status != 1) {
    cs->status = status;
    cs->stalled = stalled;
    cs->result_m = m;
    cs->stop = 1;
  } else {
    cs->m = m + 1;
  }
}

// ---------------------------------------------------------------- elementwise
constexpr int EW_NT = 256;

template <typename T>
__global__ __launch_bounds__(EW_NT) void k_fill(T* __restrict__ a, size_t n, T v, Batch bt,
                                                const int* __restrict__ stop) {
  a += (long long)blockIdx.y * bt.s0;
  if (stop != nullptr) stop += (long long)blockIdx.y * bt.stop_stride;
  if (stop != nullptr && *stop) return;
  for (size_t q = (size_t)blockIdx.x * EW_NT + threadIdx.x; q < n; q += (size_t)gridDim.x * EW_NT)
    a[q] = v;
}

// One workgroup's share of out = c * (in - m), with float64 partial sums of
// out and of out^2 into part[2 blk], part[2 blk + 1].  The single and the
// batched source preparation share it, so both compute the same bits.
__device__ __forceinline__ void scale_shift_share(const double* __restrict__ in, double* __restrict__ out, size_t n,
                                                  double c, double m, double* __restrict__ part, double* sh) {
  double s = 0.0, s2 = 0.0;
  for (size_t q = (size_t)blockIdx.x * EW_NT + threadIdx.x; q < n; q += (size_t)gridDim.x * EW_NT) {
    const double v = c * (in[q] - m);
    out[q] = v;
    s += v;
    s2 += v * v;
  }
  const double t = block_sum<EW_NT>(s, sh);
  const double t2 = block_sum<EW_NT>(s2, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = t;
    part[2 * blockIdx.x + 1] = t2;
  }
}

// out = c * (in - sum[0] / count), or c * in when sum is nullptr
__global__ __launch_bounds__(EW_NT) void k_scale(const double* __restrict__ in, double* __restrict__ out,
                                                 size_t n, double c, const double* __restrict__ sum, double count,
                                                 double* __restrict__ part) {
  __shared__ double sh[EW_NT / WAVE];
  scale_shift_share(in, out, n, c, sum != nullptr ? sum[0] / count : 0.0, part, sh);
}

// member m: out + m * s0 = c * (tab[m] - sum[m * s1] / count) (sum nullptr:
// c * tab[m]), partials at part + m * part_stride
__global__ __launch_bounds__(EW_NT) void k_scale_tab(const double* const* __restrict__ tab, double* __restrict__ out,
                                                     size_t n, double c, const double* __restrict__ sum, double count,
                                                     double* __restrict__ part, Batch bt) {
  __shared__ double sh[EW_NT / WAVE];
  const long long mb = blockIdx.y;
  scale_shift_share(tab[mb], out + mb * bt.s0, n, c, sum != nullptr ? sum[mb * bt.s1] / count : 0.0,
                    part + mb * bt.part_stride, sh);
}

// tab[m] = src (member m at src + m * s0)
__global__ __launch_bounds__(EW_NT) void k_copy_tab(double* const* __restrict__ tab, const double* __restrict__ src,
                                                    size_t n, Batch bt) {
  double* dst = tab[blockIdx.y];
  src += (long long)blockIdx.y * bt.s0;
  for (size_t q = (size_t)blockIdx.x * EW_NT + threadIdx.x; q < n; q += (size_t)gridDim.x * EW_NT) dst[q] = src[q];
}

// a -= (sum of part[b * stride + q] over b < nblk) / count: every workgroup
// sums the partials itself in the same fixed order (so all of them subtract
// the same value), which saves the separate reduction launch
template <typename T>
__global__ __launch_bounds__(EW_NT) void k_sub_mean_part(T* __restrict__ a, size_t n, const double* __restrict__ part,
                                                         int nblk, int stride, int q, double count, Batch bt,
                                                         const int* __restrict__ stop) {
  __shared__ double sh[EW_NT / WAVE];
  __shared__ double mean;
  a += (long long)blockIdx.y * bt.s0;
  part += (long long)blockIdx.y * bt.part_stride;
  if (stop != nullptr) stop += (long long)blockIdx.y * bt.stop_stride;
  if (stop != nullptr && *stop) return;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblk; b += EW_NT) v += part[(size_t)b * stride + q];
  const double t = block_sum<EW_NT>(v, sh);
  if (threadIdx.x == 0) mean = t / count;
  __syncthreads();
  const T m = (T)mean;
  // eight elements per thread in flight at once (a loop of dependent
  // load-subtract-store steps would wait out the memory latency each time)
  const size_t gs = (size_t)gridDim.x * EW_NT;
  for (size_t i0 = (size_t)blockIdx.x * EW_NT + threadIdx.x; i0 < n; i0 += 8 * gs) {
    T v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const size_t i = i0 + k * gs;
      v[k] = i < n ? a[i] : (T)0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const size_t i = i0 + k * gs;
      if (i < n) a[i] = v[k] - m;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(EW_NT) void k_sub_mean(T* __restrict__ a, size_t n,
                                                    const double* __restrict__ sum, double count, Batch bt,
                                                    const int* __restrict__ stop) {
  a += (long long)blockIdx.y * bt.s0;
  sum += (long long)blockIdx.y * bt.s1;
  if (stop != nullptr) stop += (long long)blockIdx.y * bt.stop_stride;
  if (stop != nullptr && *stop) return;
  const T m = (T)(sum[0] / count);
  for (size_t q = (size_t)blockIdx.x * EW_NT + threadIdx.x; q < n; q += (size_t)gridDim.x * EW_NT)
    a[q] -= m;
}

// dst = src - sum[0] / count (dst and src distinct)
__global__ __launch_bounds__(EW_NT) void k_copy_sub_mean(double* __restrict__ dst, const double* __restrict__ src,
                                                         size_t n, const double* __restrict__ sum, double count) {
  const double m = sum[0] / count;
  for (size_t q = (size_t)blockIdx.x * EW_NT + threadIdx.x; q < n; q += (size_t)gridDim.x * EW_NT)
    dst[q] = src[q] - m;
}

// part[blk] = float64 sum of a over the workgroup's share (shared by k_sum
// and k_sum_tab so that both compute the same bits)
template <typename T>
__device__ __forceinline__ void sum_share(const T* __restrict__ a, size_t n, double* __restrict__ part, double* sh) {
  double s = 0.0;
  for (size_t q = (size_t)blockIdx.x * EW_NT + threadIdx.x; q < n; q += (size_t)gridDim.x * EW_NT)
    s += (double)a[q];
  const double t = block_sum<EW_NT>(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <typename T>
__global__ __launch_bounds__(EW_NT) void k_sum(const T* __restrict__ a, size_t n, double* __restrict__ part,
                                               Batch bt) {
  __shared__ double sh[EW_NT / WAVE];
  sum_share<T>(a + (long long)blockIdx.y * bt.s0, n, part + (long long)blockIdx.y * bt.part_stride, sh);
}

// the same over member m = tab[m]
__global__ __launch_bounds__(EW_NT) void k_sum_tab(const double* const* __restrict__ tab, size_t n,
                                                   double* __restrict__ part, Batch bt) {
  __shared__ double sh[EW_NT / WAVE];
  sum_share<double>(tab[blockIdx.y], n, part + (long long)blockIdx.y * bt.part_stride, sh);
}

// dst = src; skipped once the device-side loop has decided to stop (a cycle
// queued past the stopping one must not overwrite the answer)
template <typename T>
__global__ __launch_bounds__(EW_NT) void k_copy(T* __restrict__ dst, const T* __restrict__ src, size_t n,
                                                const int* __restrict__ stop) {
  if (stop != nullptr && *stop) return;
  for (size_t q = (size_t)blockIdx.x * EW_NT + threadIdx.x; q < n; q += (size_t)gridDim.x * EW_NT) dst[q] = src[q];
}

// u64 += (double) e
template <typename TE>
__global__ __launch_bounds__(EW_NT) void k_add_cast(double* __restrict__ u, const TE* __restrict__ e,
                                                    size_t n, Batch bt, const int* __restrict__ stop) {
  u += (long long)blockIdx.y * bt.s0;
  e += (long long)blockIdx.y * bt.s1;
  if (stop != nullptr) stop += (long long)blockIdx.y * bt.stop_stride;
  if (stop != nullptr && *stop) return;
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

void launch_fold_faces(int nx, int ny, int nz, double hx, double hy, double hz, const double* faces,
                       const double* src, double* dst, hipStream_t st) {
  const int kz = ((size_t)nx * ny * nz < ((size_t)1 << 21)) ? 1 : KZ;
  hipLaunchKernelGGL(k_fold_faces, grid3(nx, ny, nz, kz), dim3(TX, TY), 0, st, nx, ny, nz, 1.0 / (hx * hx),
                     1.0 / (hy * hy), 1.0 / (hz * hz), faces, src, dst, kz);
}

void launch_gradient(int nx, int ny, int nz, double hx, double hy, double hz, int periodic, const double* faces,
                     const double* phi, double* gx, double* gy, double* gz, hipStream_t st) {
  const int kz = ((size_t)nx * ny * nz < ((size_t)1 << 21)) ? 1 : KZ;
  hipLaunchKernelGGL(k_gradient, grid3(nx, ny, nz, kz), dim3(TX, TY), 0, st, nx, ny, nz, 1.0 / hx, 1.0 / hy,
                     1.0 / hz, periodic, faces, phi, gx, gy, gz, kz);
}

template <typename T>
void launch_gsrb_half(const LevelView<T>& L, const T* uin, T* uout, const T* b, int colour, double omega,
                      const int* stop, hipStream_t st, const Batch& bt) {
  const double d = 2.0 * ((double)L.ihx2 + (double)L.ihy2 + (double)L.ihz2);
  const size_t n = (size_t)L.nx * L.ny * L.nz;
  hipLaunchKernelGGL(k_gsrb_half<T>, dim3(ew_blocks(n), bt.nb), dim3(256), 0, st, L, uin, uout, b, colour,
                     (T)(omega / d), bt, stop);
}

template <typename T>
void launch_resid_absmax(const LevelView<T>& L, const T* u, const T* b, double* part, double* out, hipStream_t st) {
  const size_t n = (size_t)L.nx * L.ny * L.nz;
  const unsigned nb = ew_blocks(n);
  hipLaunchKernelGGL(k_resid_absmax<T>, dim3(nb), dim3(256), 0, st, L, u, b, part);
  hipLaunchKernelGGL(k_reduce_max, dim3(1), dim3(256), 0, st, part, (int)nb, out);
}

template void launch_gsrb_half<double>(const LevelView<double>&, const double*, double*, const double*, int, double,
                                       const int*, hipStream_t, const Batch&);
template void launch_gsrb_half<float>(const LevelView<float>&, const float*, float*, const float*, int, double,
                                      const int*, hipStream_t, const Batch&);
template void launch_resid_absmax<double>(const LevelView<double>&, const double*, const double*, double*, double*,
                                          hipStream_t);

template <typename T>
void launch_stage(const LevelView<T>& L, const T* yp, const T* ypp, const T* b, T* yout, double mu,
                  double nu, double c, int first, const int* stop, hipStream_t st) {
  // one plane per thread on small levels (each z step is a dependent round trip)
  const int kz = ((size_t)L.nx * L.ny * L.nz < ((size_t)1 << 21)) ? 1 : KZ;
  hipLaunchKernelGGL(k_stage<T>, grid3(L.nx, L.ny, L.nz, kz), dim3(TX, TY), 0, st, L, yp, ypp, b, yout,
                     (T)mu, (T)nu, (T)c, first, kz, stop);
}

template <typename T>
void launch_restrict(int fnx, int fny, int fnz, const T* fine, T* coarse, hipStream_t st) {
  const int cnz = fnz == 1 ? 1 : fnz / 2;  // one fine plane: two-dimensional
  hipLaunchKernelGGL(k_restrict<T>, grid3(fnx / 2, fny / 2, cnz), dim3(TX, TY), 0, st, fnx, fny, fnz, fine,
                     coarse);
}

void launch_reduce(const double* part, int nblk, int stride, int nq, double* out, const int* stop,
                   hipStream_t st, const Batch& bt) {
  hipLaunchKernelGGL(k_reduce, dim3(bt.nb), dim3(RED_NT), 0, st, part, nblk, stride, nq, out, bt, stop);
}

void launch_check(const double* part, int nblk, int stride, const double* res0sq, double tol, int max_cycles,
                  double count, ConvState* cs, hipStream_t st, const Batch& bt) {
  hipLaunchKernelGGL(k_check, dim3(bt.nb), dim3(RED_NT), 0, st, part, nblk, stride, res0sq, tol, max_cycles,
                     count, cs, bt);
}

void launch_scale_tab(const double* const* tab, double* out, size_t n, double c, const double* sum, double count,
                      double* part, hipStream_t st, const Batch& bt) {
  hipLaunchKernelGGL(k_scale_tab, dim3(ew_blocks(n), bt.nb), dim3(EW_NT), 0, st, tab, out, n, c, sum, count, part,
                     bt);
}

void launch_sum_tab(const double* const* tab, size_t n, double* part, hipStream_t st, const Batch& bt) {
  hipLaunchKernelGGL(k_sum_tab, dim3(ew_blocks(n), bt.nb), dim3(EW_NT), 0, st, tab, n, part, bt);
}

void launch_copy_tab(double* const* tab, const double* src, size_t n, hipStream_t st, const Batch& bt) {
  hipLaunchKernelGGL(k_copy_tab, dim3(ew_blocks(n), bt.nb), dim3(EW_NT), 0, st, tab, src, n, bt);
}

template <typename T>
void launch_fill(T* a, size_t n, T v, const int* stop, hipStream_t st, const Batch& bt) {
  hipLaunchKernelGGL(k_fill<T>, dim3(ew_blocks(n), bt.nb), dim3(EW_NT), 0, st, a, n, v, bt, stop);
}

void launch_scale(const double* in, double* out, size_t n, double c, const double* sum, double count, double* part,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_scale, dim3(ew_blocks(n)), dim3(EW_NT), 0, st, in, out, n, c, sum, count, part);
}

void launch_copy_sub_mean(double* dst, const double* src, size_t n, const double* sum, double count,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_copy_sub_mean, dim3(ew_blocks(n)), dim3(EW_NT), 0, st, dst, src, n, sum, count);
}

template <typename T>
void launch_sub_mean(T* a, size_t n, const double* sum, double count, const int* stop, hipStream_t st,
                     const Batch& bt) {
  hipLaunchKernelGGL(k_sub_mean<T>, dim3(ew_blocks(n), bt.nb), dim3(EW_NT), 0, st, a, n, sum, count, bt, stop);
}

// Every workgroup of k_sub_mean_part re-reads all nblk partials, so it gets
// about eight elements per thread (at most 2048 workgroups, at least 512 or
// one per 256 elements) rather than one: the partial sums then cost a few MB
// of L2 reads instead of one reduction per 256 elements.
static inline unsigned sub_mean_part_blocks(size_t n) {
  const size_t lo = std::min<size_t>(ew_blocks(n), 512);
  return (unsigned)std::max(lo, std::min<size_t>(n / ((size_t)EW_NT * 8), 2048));
}

template <typename T>
void launch_sub_mean_part(T* a, size_t n, const double* part, int nblk, int stride, int q, double count,
                          const int* stop, hipStream_t st, const Batch& bt) {
  hipLaunchKernelGGL(k_sub_mean_part<T>, dim3(sub_mean_part_blocks(n), bt.nb), dim3(EW_NT), 0, st, a, n, part, nblk,
                     stride, q, count, bt, stop);
}

template <typename T>
void launch_sum(const T* a, size_t n, double* part, hipStream_t st, const Batch& bt) {
  hipLaunchKernelGGL(k_sum<T>, dim3(ew_blocks(n), bt.nb), dim3(EW_NT), 0, st, a, n, part, bt);
}

template <typename T>
void launch_copy(T* dst, const T* src, size_t n, const int* stop, hipStream_t st) {
  hipLaunchKernelGGL(k_copy<T>, dim3(ew_blocks(n)), dim3(EW_NT), 0, st, dst, src, n, stop);
}

template <typename TE>
void launch_add_cast(double* u, const TE* e, size_t n, const int* stop, hipStream_t st, const Batch& bt) {
  hipLaunchKernelGGL(k_add_cast<TE>, dim3(ew_blocks(n), bt.nb), dim3(EW_NT), 0, st, u, e, n, bt, stop);
}

// explicit instantiations
template void launch_stage<double>(const LevelView<double>&, const double*, const double*, const double*,
                                   double*, double, double, double, int, const int*, hipStream_t);
template void launch_stage<float>(const LevelView<float>&, const float*, const float*, const float*,
                                  float*, double, double, double, int, const int*, hipStream_t);
template void launch_restrict<double>(int, int, int, const double*, double*, hipStream_t);
template void launch_restrict<float>(int, int, int, const float*, float*, hipStream_t);
template void launch_fill<double>(double*, size_t, double, const int*, hipStream_t, const Batch&);
template void launch_fill<float>(float*, size_t, float, const int*, hipStream_t, const Batch&);
template void launch_sub_mean<double>(double*, size_t, const double*, double, const int*, hipStream_t,
                                      const Batch&);
template void launch_sub_mean<float>(float*, size_t, const double*, double, const int*, hipStream_t, const Batch&);
template void launch_sub_mean_part<double>(double*, size_t, const double*, int, int, int, double, const int*,
                                           hipStream_t, const Batch&);
template void launch_sub_mean_part<float>(float*, size_t, const double*, int, int, int, double, const int*,
                                          hipStream_t, const Batch&);
template void launch_sum<double>(const double*, size_t, double*, hipStream_t, const Batch&);
template void launch_sum<float>(const float*, size_t, double*, hipStream_t, const Batch&);
template void launch_copy<double>(double*, const double*, size_t, const int*, hipStream_t);
template void launch_copy<float>(float*, const float*, size_t, const int*, hipStream_t);
template void launch_add_cast<float>(double*, const float*, size_t, const int*, hipStream_t, const Batch&);
template void launch_add_cast<double>(double*, const double*, size_t, const int*, hipStream_t, const Batch&);

}  // namespace rkl
