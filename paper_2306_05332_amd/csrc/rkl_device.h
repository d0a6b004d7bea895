// Device-side building blocks shared by the gfx950 kernels: level view,
// boundary ghosts fused into stencil loads, deterministic block reductions.
//
// Cell-centred 7-point Laplacian (Sec. 2.2.1 eq. discrete_laplace_3D); ghost
// cells (Sec. 2.3): finest-level Dirichlet ghost = 2 g - u_adj (eq.
// solution_ghost), coarse-level (error) Dirichlet ghost = -u_adj (eq.
// error_ghost), periodic wrap on every level (eq. periodic).  No ghost layer
// is stored: a stencil that leaves the box recomputes the ghost from the
// centre value, which is the adjacent active cell of a face ghost.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rkl {

constexpr int WAVE = 64;  // CDNA wavefront width

// A batch of identical grids handled by one launch: member m (blockIdx.y, or
// blockIdx.x for kernels with one workgroup per member) finds its arrays at
// base + m * stride.  A single solve is the batch {1, 0, 0, 0, 0}.
struct Batch {
  int nb;            // members
  long long s0, s1;  // element strides of the primary and secondary arrays
  int stop_stride;   // ints between members' stop flags
  int part_stride;   // doubles between members' partial-sum blocks
};
inline Batch single_batch() { return Batch{1, 0, 0, 0, 0}; }

// Stage coefficients of one s-stage tau-step in the working precision:
// Y_j = mu[j-1] Y_{j-1} + nu[j-1] Y_{j-2} + c[j-1] (M Y_{j-1} - b).
template <typename T, int S>
struct FCoef {
  T mu[S], nu[S], c[S];
};

template <typename T>
struct LevelView {
  int nx, ny, nz;
  T ihx2, ihy2, ihz2;     // 1 / h_d^2
  int periodic;           // 1: wrap; 0: Dirichlet
  const double* faces;    // finest-level Dirichlet face values or nullptr (homogeneous)
};

// Offsets of the six packed face arrays (x-, x+, y-, y+, z-, z+).
__host__ __device__ inline size_t face_off(int face, int nx, int ny, int nz) {
  const size_t fx = (size_t)ny * nz, fy = (size_t)nx * nz, fz = (size_t)nx * ny;
  switch (face) {
    case 0: return 0;
    case 1: return fx;
    case 2: return 2 * fx;
    case 3: return 2 * fx + fy;
    case 4: return 2 * fx + 2 * fy;
    default: return 2 * fx + 2 * fy + fz;
  }
}

template <typename T>
__device__ __forceinline__ T dir_ghost(const LevelView<T>& L, int face, size_t fidx, T c) {
  if (L.faces) return (T)(2.0 * L.faces[face_off(face, L.nx, L.ny, L.nz) + fidx]) - c;
  return -c;
}

// Six neighbours of cell (i,j,k) with value c, ghosts applied.
template <typename T>
struct Nbrs {
  T xm, xp, ym, yp, zm, zp;
};

template <typename T>
__device__ __forceinline__ Nbrs<T> load_nbrs(const LevelView<T>& L, const T* __restrict__ u,
                                             int i, int j, int k, size_t idx, T c) {
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
  Nbrs<T> n;
  if (i > 0) n.xm = u[idx - 1];
  else n.xm = L.periodic ? u[idx + (nx - 1)] : dir_ghost(L, 0, (size_t)k * ny + j, c);
  if (i < nx - 1) n.xp = u[idx + 1];
  else n.xp = L.periodic ? u[idx - (nx - 1)] : dir_ghost(L, 1, (size_t)k * ny + j, c);
  if (j > 0) n.ym = u[idx - sy];
  else n.ym = L.periodic ? u[idx + (size_t)(ny - 1) * sy] : dir_ghost(L, 2, (size_t)k * nx + i, c);
  if (j < ny - 1) n.yp = u[idx + sy];
  else n.yp = L.periodic ? u[idx - (size_t)(ny - 1) * sy] : dir_ghost(L, 3, (size_t)k * nx + i, c);
  if (k > 0) n.zm = u[idx - sz];
  else n.zm = L.periodic ? u[idx + (size_t)(nz - 1) * sz] : dir_ghost(L, 4, (size_t)j * nx + i, c);
  if (k < nz - 1) n.zp = u[idx + sz];
  else n.zp = L.periodic ? u[idx - (size_t)(nz - 1) * sz] : dir_ghost(L, 5, (size_t)j * nx + i, c);
  return n;
}

template <typename T>
__device__ __forceinline__ T lap7(const LevelView<T>& L, const Nbrs<T>& n, T c) {
  return ((n.xm + n.xp) - (T)2 * c) * L.ihx2 + ((n.ym + n.yp) - (T)2 * c) * L.ihy2 +
         ((n.zm + n.zp) - (T)2 * c) * L.ihz2;
}

// Deterministic sum over a workgroup of NT threads: fixed-order shuffle tree
// inside each wavefront, then wave 0 adds the per-wave sums in order.
// `sh` needs NT/64 doubles.  Result valid in thread 0.
// LDS-poison debug builds (-DRKL_LDS_POISON, see build_sanitized.py): every
// kernel fills its floating-point LDS arrays with NaN on entry, so a read of
// an element that no thread wrote in this launch turns the results into NaN
// and the parity tests fail.  Called by every thread of the workgroup before
// any early return; ordinary builds compile it to nothing.
template <typename T>
__device__ __forceinline__ void lds_poison(T* p, int n) {
#ifdef RKL_LDS_POISON
  const int nt = blockDim.x * blockDim.y * blockDim.z;
  for (int i = threadIdx.x; i < n; i += nt) p[i] = __builtin_nan("");
#else
  (void)p;
  (void)n;
#endif
}
__device__ __forceinline__ void lds_poison_sync() {
#ifdef RKL_LDS_POISON
  __syncthreads();
#endif
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  static_assert(NT % WAVE == 0, "block size must be a multiple of the wavefront");
  const int lane = threadIdx.x + threadIdx.y * blockDim.x;
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_down(v, off, WAVE);
  const int w = lane / WAVE;
  if ((lane % WAVE) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NT / WAVE; ++q) t += sh[q];
  }
  __syncthreads();
  return t;
}

// Sum over one wavefront with DPP row shifts and row broadcasts (GFX9 DPP
// controls row_shr:1,2,4,8, row_bcast:15, row_bcast:31): a fixed order, no
// LDS round trips.  Every lane returns the total (read from lane 63).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_mov_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, true);
  const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, true);
  return __hiloint2double(h2, l2);
}

// Whole-wavefront shift by one lane (GFX9 DPP wave_shl:1 / wave_shr:1); the
// end lanes receive 0.
constexpr int DPP_WAVE_SHL1 = 0x130;  // dst[i] = src[i + 1]
constexpr int DPP_WAVE_SHR1 = 0x138;  // dst[i] = src[i - 1]

template <int CTRL>
__device__ __forceinline__ float wshift(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}

template <int CTRL>
__device__ __forceinline__ double wshift(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_mov_f64<0x111, 0xf>(v);  // row_shr:1
  v += dpp_mov_f64<0x112, 0xf>(v);  // row_shr:2
  v += dpp_mov_f64<0x114, 0xf>(v);  // row_shr:4
  v += dpp_mov_f64<0x118, 0xf>(v);  // row_shr:8: lane 15 of each row holds the row sum
  v += dpp_mov_f64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_mov_f64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3: lane 63 holds the total
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

}  // namespace rkl
