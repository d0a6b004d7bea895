// LDS-tiled residual, residual + restriction, and prolongation + correction.
//
//   k_resid_tile<.., false>  r = b - M u (Sec. 2.1 eq. residual, opposite sign)
//                            with float64 partial sums of r^2 and r
//   k_resid_tile<.., false, true>  the same for u' = u + e (e float32), which
//                            it also writes: the mixed path's update of the
//                            float64 iterate folded into the next defect
//                            (Sec. 2.2.3), 32 bytes a cell against 20 + 20
//                            for the update and the defect apart
//   k_resid_tile<.., true>   b_{l+1} = R(b_l - M_l u_l): the 8-child average of
//                            eq. restriction_example_3D applied to the residual
//                            (Sec. 2.1 steps 2a/2b), with float64 partials of
//                            the fine r^2 and of the coarse values (the latter
//                            feed the periodic mean removal, Sec. 2.3)
//   k_prolong_tile           u_l += P(u_{l+1}) with the (27, 9, 9, 9, 3, 3, 3, 1)/64
//                            weights of eq. prolongation_example_3D and the
//                            error-equation ghosts of the coarse grid
//
// A fine level with a single z plane is two-dimensional (levels of a 3-D
// hierarchy always have an even number of planes): restriction then averages
// the 4 children of eq. restriction_example_2D, and prolongation takes the
// z-neighbour plane equal to the parent plane, which turns the trilinear
// weights into the (9, 3, 3, 1)/16 of eq. prolongation_example_2D
// (27 + 9 = 36, 9 + 3 = 12, 3 + 1 = 4 sixty-fourths).
//
// Both march upward in z.  The residual kernels keep four fine u planes of a
// 64 x 16 tile (plus a one-cell halo) in an LDS ring and handle one coarse
// plane (two fine planes) per step; the prolongation keeps three coarse
// planes of the tile's coarse footprint in LDS.  The next planes are loaded
// into registers while the current ones are processed, so each HBM word is
// read once per tile (halos come from L2).
#include "host_common.h"
#include "kernels.h"

namespace rkl {

constexpr int RNT = 256;
constexpr int RBX = 64, RBY = 16;                  // fine interior tile (32 x 8 coarse cells)
constexpr int RW = RBX + 2, RH = RBY + 2, RPL = RW * RH;
constexpr int RNU = (RPL + RNT - 1) / RNT;         // haloed-plane slots per thread
constexpr int RNI = (RBX * RBY) / RNT;             // interior slots per thread

__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  // consecutive workgroups go round-robin to the 8 XCDs: give each XCD a
  // contiguous run of tiles so neighbouring halos meet in one L2
  if ((nblk & 7) == 0) return (bid & 7) * (nblk >> 3) + (bid >> 3);
  return bid;
}

template <typename TU, typename TR, bool RESTRICT, bool ADD = false>
__global__ __launch_bounds__(RNT) void k_resid_tile(LevelView<TU> F, const TU* __restrict__ u,
                                                    const TU* __restrict__ b, TR* __restrict__ out,
                                                    int kc, int gx_tiles, int gy_tiles, int nblk,
                                                    double* __restrict__ part, Batch bt,
                                                    const int* __restrict__ stop, const float* __restrict__ e,
                                                    TU* __restrict__ unew) {
  static_assert(!ADD || !RESTRICT, "the update is folded into the plain defect only");
  {
    const long long mb = blockIdx.y;
    if (u != nullptr) u += mb * bt.s0;
    if (ADD) {
      e += mb * bt.s0;
      unew += mb * bt.s0;
    }
    b += mb * bt.s0;
    if (out != nullptr) out += mb * (RESTRICT ? bt.s1 : bt.s0);
    part += mb * bt.part_stride;
    if (stop != nullptr) stop += mb * bt.stop_stride;
  }
  __shared__ TU ring[4][RPL];
  __shared__ TU zs[RESTRICT ? RBY : 1][RESTRICT ? RBX : 1];
  __shared__ double red[RNT / WAVE];
  lds_poison(&ring[0][0], 4 * RPL);
  lds_poison(&zs[0][0], (RESTRICT ? RBY : 1) * (RESTRICT ? RBX : 1));
  lds_poison(red, RNT / WAVE);
  lds_poison_sync();
  if (stop != nullptr && *stop) return;
  const int tid = threadIdx.x;
  const int nx = F.nx, ny = F.ny, nz = F.nz;
  const bool per = F.periodic != 0;
  const size_t sxy = (size_t)nx * ny;
  const int bid = xcd_remap(blockIdx.x, nblk);
  const int tx = bid % gx_tiles, ty = (bid / gx_tiles) % gy_tiles, tzc = bid / (gx_tiles * gy_tiles);
  const int x0 = tx * RBX - 1, y0 = ty * RBY - 1;
  const int npair = (nz + 1) / 2;
  const int K0 = tzc * kc, K1 = min(K0 + kc, npair);

  int goff[RNU];
#pragma unroll
  for (int q = 0; q < RNU; ++q) {
    const int idx = tid + q * RNT;
    goff[q] = -1;
    if (idx < RPL) {
      const int gxr = x0 + idx % RW, gyr = y0 + idx / RW;
      if (per) goff[q] = ((gyr % ny + ny) % ny) * nx + (gxr % nx + nx) % nx;
      else if (gxr >= 0 && gxr < nx && gyr >= 0 && gyr < ny) goff[q] = gyr * nx + gxr;
    }
  }
  // interior slots
  int igx[RNI], igy[RNI];
  bool iin[RNI];
#pragma unroll
  for (int q = 0; q < RNI; ++q) {
    const int idx = tid + q * RNT;
    igx[q] = tx * RBX + idx % RBX;
    igy[q] = ty * RBY + idx / RBX;
    iin[q] = igx[q] < nx && igy[q] < ny;
  }
  // a two-dimensional level (one plane, ihz2 = 0) reads only its own plane:
  // the z terms carry no weight
  const bool flat = nz == 1 && F.ihz2 == (TU)0;
  auto plane_ok = [&](int p) { return flat ? p == 0 : (per ? true : (p >= 0 && p < nz)); };
  auto zw = [&](int p) { return per ? (p % nz + nz) % nz : p; };
  auto rslot = [](int p) { return (p + 8) & 3; };

  TU pa[RNU], pb[RNU];   // u planes in flight
  TU ba[RNI], bb[RNI];   // b planes in flight
  auto load_u = [&](int p, TU (&dst)[RNU]) {
    const bool ok = u != nullptr && plane_ok(p) && (per || p < nz);
    const size_t zo = ok ? (size_t)zw(p) * sxy : 0;
#pragma unroll
    for (int q = 0; q < RNU; ++q) {
      dst[q] = (ok && goff[q] >= 0) ? u[zo + goff[q]] : (TU)0;
      if (ADD && ok && goff[q] >= 0) dst[q] += (TU)e[zo + goff[q]];
    }
  };
  auto load_b = [&](int p, TU (&dst)[RNI]) {
    const bool ok = p >= 0 && p < nz;
    const size_t zo = ok ? (size_t)p * sxy : 0;
#pragma unroll
    for (int q = 0; q < RNI; ++q) dst[q] = (ok && iin[q]) ? b[zo + (size_t)igy[q] * nx + igx[q]] : (TU)0;
  };
  auto store_u = [&](int p, const TU (&src)[RNU]) {
    TU* d = ring[rslot(p)];
#pragma unroll
    for (int q = 0; q < RNU; ++q) {
      const int idx = tid + q * RNT;
      if (idx < RPL) d[idx] = src[q];
    }
  };

  // r = b - M u at interior slot q of fine plane p (ring holds p-1, p, p+1)
  auto resid = [&](int q, int p, TU bv) -> TU {
    const int idx = tid + q * RNT;
    const int o = (idx / RBX + 1) * RW + (idx % RBX + 1);
    const TU* Yc = ring[rslot(p)];
    const TU c = Yc[o];
    TU xm = Yc[o - 1], xp = Yc[o + 1], ym = Yc[o - RW], yp = Yc[o + RW];
    TU zm = ring[rslot(p - 1)][o], zp = ring[rslot(p + 1)][o];
    if (!per) {
      const int gx = igx[q], gy = igy[q];
      if (gx == 0) xm = dir_ghost(F, 0, (size_t)p * ny + gy, c);
      if (gx == nx - 1) xp = dir_ghost(F, 1, (size_t)p * ny + gy, c);
      if (gy == 0) ym = dir_ghost(F, 2, (size_t)p * nx + gx, c);
      if (gy == ny - 1) yp = dir_ghost(F, 3, (size_t)p * nx + gx, c);
      if (p == 0) zm = dir_ghost(F, 4, (size_t)gy * nx + gx, c);
      if (p == nz - 1) zp = dir_ghost(F, 5, (size_t)gy * nx + gx, c);
    }
    const TU lap = ((xm + xp) - (TU)2 * c) * F.ihx2 + ((ym + yp) - (TU)2 * c) * F.ihy2 +
                   ((zm + zp) - (TU)2 * c) * F.ihz2;
    return bv - lap;
  };

  double s2 = 0.0, s1 = 0.0;
  if (K0 < K1) {
    // ring: planes 2K0-1, 2K0 now; 2K0+1, 2K0+2 in flight
    {
      TU t0[RNU], t1[RNU];
      load_u(2 * K0 - 1, t0);
      load_u(2 * K0, t1);
      store_u(2 * K0 - 1, t0);
      store_u(2 * K0, t1);
    }
    load_u(2 * K0 + 1, pa);
    load_u(2 * K0 + 2, pb);
    load_b(2 * K0, ba);
    load_b(2 * K0 + 1, bb);
    for (int K = K0; K < K1; ++K) {
      const int p0 = 2 * K, p1 = 2 * K + 1;
      store_u(p1, pa);
      store_u(p1 + 1, pb);
      TU bc0[RNI], bc1[RNI];
#pragma unroll
      for (int q = 0; q < RNI; ++q) {
        bc0[q] = ba[q];
        bc1[q] = bb[q];
      }
      __syncthreads();
      if (K + 1 < K1) {
        load_u(2 * K + 3, pa);
        load_u(2 * K + 4, pb);
        load_b(2 * K + 2, ba);
        load_b(2 * K + 3, bb);
      }
      const bool has1 = p1 < nz;
#pragma unroll
      for (int q = 0; q < RNI; ++q) {
        TU r0 = (TU)0, r1 = (TU)0;
        if (iin[q]) {
          r0 = resid(q, p0, bc0[q]);
          s2 += (double)r0 * (double)r0;
          if (has1) {
            r1 = resid(q, p1, bc1[q]);
            s2 += (double)r1 * (double)r1;
          }
          if (!RESTRICT) {
            s1 += (double)r0 + (double)r1;
            if (ADD) {
              // u' of the cell, as the ring holds it, and r: non-temporal
              // hints (the form runs on levels beyond the last-level cache,
              // where neither is read again before it would be evicted;
              // 512^3 mixed solve 31.35 -> 30.78 ms)
              const int idx = tid + q * RNT;
              const int o = (idx / RBX + 1) * RW + (idx % RBX + 1);
              const size_t c0 = (size_t)p0 * sxy + (size_t)igy[q] * nx + igx[q];
              __builtin_nontemporal_store((TR)r0, out + c0);
              __builtin_nontemporal_store(ring[rslot(p0)][o], unew + c0);
              if (has1) {
                __builtin_nontemporal_store((TR)r1, out + c0 + sxy);
                __builtin_nontemporal_store(ring[rslot(p1)][o], unew + c0 + sxy);
              }
            } else if (out != nullptr) {
              out[(size_t)p0 * sxy + (size_t)igy[q] * nx + igx[q]] = (TR)r0;
              if (has1) out[(size_t)p1 * sxy + (size_t)igy[q] * nx + igx[q]] = (TR)r1;
            }
          }
        }
        if (RESTRICT) {
          const int idx = tid + q * RNT;
          zs[RESTRICT ? idx / RBX : 0][RESTRICT ? idx % RBX : 0] = r0 + r1;
        }
      }
      __syncthreads();
      if (RESTRICT) {
        const int cx = tid % (RBX / 2), cy = tid / (RBX / 2);  // 32 x 8 coarse cells, one per thread
        const int cnx = nx / 2, cny = ny / 2;
        const int gcx = tx * (RBX / 2) + cx, gcy = ty * (RBY / 2) + cy;
        if (gcx < cnx && gcy < cny) {
          const TU v = ((zs[2 * cy][2 * cx] + zs[2 * cy][2 * cx + 1]) +
                        (zs[2 * cy + 1][2 * cx] + zs[2 * cy + 1][2 * cx + 1])) * (nz == 1 ? (TU)0.25 : (TU)0.125);
          out[((size_t)K * cny + gcy) * cnx + gcx] = (TR)v;
          s1 += (double)v;
        }
        __syncthreads();
      }
    }
  }
  const double t2 = block_sum<RNT>(s2, red);
  const double t1 = block_sum<RNT>(s1, red);
  if (tid == 0) {
    part[2 * (size_t)blockIdx.x] = t2;
    part[2 * (size_t)blockIdx.x + 1] = t1;
  }
}

// ---------------------------------------------------------------- prolongation
constexpr int PNT = 256;
constexpr int PBX = 64, PBY = 8;                   // fine tile
constexpr int PCW = PBX / 2 + 2, PCH = PBY / 2 + 2, PCL = PCW * PCH;  // coarse footprint + halo
constexpr int PNF = PBX * PBY / PNT;               // fine slots per thread
constexpr int PNC = (PCL + PNT - 1) / PNT;         // coarse slots per thread

template <typename T>
__global__ __launch_bounds__(PNT) void k_prolong_tile(int fnx, int fny, int fnz, int periodic,
                                                      const T* __restrict__ e, T* __restrict__ fine, int kc,
                                                      int gx_tiles, int gy_tiles, int nblk, Batch bt,
                                                      const int* __restrict__ stop) {
  {
    const long long mb = blockIdx.y;
    e += mb * bt.s1;
    fine += mb * bt.s0;
    if (stop != nullptr) stop += mb * bt.stop_stride;
  }
  __shared__ T cr[3][PCL];
  lds_poison(&cr[0][0], 3 * PCL);
  lds_poison_sync();
  if (stop != nullptr && *stop) return;
  const int tid = threadIdx.x;
  const bool flat = fnz == 1;  // two-dimensional: one coarse plane, its own z neighbour
  const int cnx = fnx / 2, cny = fny / 2, cnz = flat ? 1 : fnz / 2;
  const int bid = xcd_remap(blockIdx.x, nblk);
  const int tx = bid % gx_tiles, ty = (bid / gx_tiles) % gy_tiles, tz = bid / (gx_tiles * gy_tiles);
  const int k0 = tz * kc, k1 = min(k0 + kc, fnz);  // kc is even
  const int cx0 = tx * (PBX / 2) - 1, cy0 = ty * (PBY / 2) - 1;
  const size_t fsxy = (size_t)fnx * fny, csxy = (size_t)cnx * cny;

  // coarse slots: in-plane offset and sign of the ghost (odd reflection per
  // axis for homogeneous Dirichlet, wrap for periodic)
  int coff[PNC];
  T csg[PNC];
#pragma unroll
  for (int q = 0; q < PNC; ++q) {
    const int idx = tid + q * PNT;
    coff[q] = -1;
    csg[q] = (T)1;
    if (idx < PCL) {
      int I = cx0 + idx % PCW, J = cy0 + idx / PCW;
      if (periodic) {
        I = (I % cnx + cnx) % cnx;
        J = (J % cny + cny) % cny;
      } else {
        if (I < 0) { I = 0; csg[q] = -csg[q]; }
        if (I >= cnx) { I = cnx - 1; csg[q] = -csg[q]; }
        if (J < 0) { J = 0; csg[q] = -csg[q]; }
        if (J >= cny) { J = cny - 1; csg[q] = -csg[q]; }
      }
      coff[q] = J * cnx + I;
    }
  }
  auto load_c = [&](int K, T (&dst)[PNC]) {
    T zs = (T)1;
    int Kw = K;
    if (flat) Kw = 0;
    else if (periodic) Kw = (K % cnz + cnz) % cnz;
    else {
      if (K < 0) { Kw = 0; zs = -zs; }
      if (K >= cnz) { Kw = cnz - 1; zs = -zs; }
    }
    const size_t zo = (size_t)Kw * csxy;
#pragma unroll
    for (int q = 0; q < PNC; ++q) dst[q] = coff[q] >= 0 ? zs * csg[q] * e[zo + coff[q]] : (T)0;
  };
  auto store_c = [&](int K, const T (&src)[PNC]) {
    T* d = cr[(K + 3) % 3];
#pragma unroll
    for (int q = 0; q < PNC; ++q) {
      const int idx = tid + q * PNT;
      if (idx < PCL) d[idx] = src[q];
    }
  };
  int fx[PNF], fy[PNF];
  bool fin[PNF];
#pragma unroll
  for (int q = 0; q < PNF; ++q) {
    const int idx = tid + q * PNT;
    fx[q] = tx * PBX + idx % PBX;
    fy[q] = ty * PBY + idx / PBX;
    fin[q] = fx[q] < fnx && fy[q] < fny;
  }
  if (k0 >= k1) return;
  {
    const int K = k0 >> 1;
    T c0[PNC], c1[PNC], c2[PNC];
    load_c(K - 1, c0);
    load_c(K, c1);
    load_c(K + 1, c2);
    store_c(K - 1, c0);
    store_c(K, c1);
    store_c(K + 1, c2);
  }
  T cn[PNC];
  T un[PNF];
  load_c((k0 >> 1) + 2, cn);
#pragma unroll
  for (int q = 0; q < PNF; ++q) un[q] = fin[q] ? fine[(size_t)k0 * fsxy + (size_t)fy[q] * fnx + fx[q]] : (T)0;
  __syncthreads();
  for (int k = k0; k < k1; ++k) {
    const int K = k >> 1, sz = (k & 1) ? 1 : -1;
    if (k > k0 && (k & 1) == 0) {
      // entering coarse plane K: K+1 was prefetched; K-2's slot is free
      __syncthreads();
      store_c(K + 1, cn);
      __syncthreads();
      load_c(K + 2, cn);
    }
    T uc[PNF];
#pragma unroll
    for (int q = 0; q < PNF; ++q) uc[q] = un[q];
    if (k + 1 < k1) {
#pragma unroll
      for (int q = 0; q < PNF; ++q)
        un[q] = fin[q] ? fine[(size_t)(k + 1) * fsxy + (size_t)fy[q] * fnx + fx[q]] : (T)0;
    }
    const T* Ca = cr[(K + 3) % 3];
    const T* Cb = cr[(K + sz + 3) % 3];
#pragma unroll
    for (int q = 0; q < PNF; ++q) {
      if (!fin[q]) continue;
      const int i = fx[q], j = fy[q];
      const int Il = (i >> 1) - cx0, Jl = (j >> 1) - cy0;
      const int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? PCW : -PCW;
      const int o = Jl * PCW + Il;
      // trilinear weights: 3/4 on the parent side, 1/4 on the neighbour side, per axis
      const T a = (T)27 * Ca[o] + (T)9 * (Ca[o + sx] + Ca[o + sy] + Cb[o]) +
                  (T)3 * (Ca[o + sx + sy] + Cb[o + sx] + Cb[o + sy]) + Cb[o + sx + sy];
      fine[(size_t)k * fsxy + (size_t)j * fnx + i] = uc[q] + a * (T)(1.0 / 64.0);
    }
  }
}

// ---------------------------------------------------------------- single-plane levels
// A level with one z plane (a two-dimensional level, or a 3-D grid of one
// plane) takes row-marching kernels instead of the tiles above, whose blocks
// would each see a single plane pair.  A lane owns one column pair (2I, 2I+1)
// -- one coarse column I -- and lanes 0 and 63 of a wavefront are halo: their
// pairs only feed the x neighbours of lanes 1 and 62 through wavefront DPP
// shifts, so a wavefront covers 62 coarse columns.  Each wavefront marches a
// chunk of row pairs (2J, 2J+1); the u rows 2J-1 .. 2J+2 stay in registers
// and the next rows are loaded one step ahead, so every row is read once.
// The z term of the single plane is the periodic self-neighbour (0) or the
// Dirichlet ghost pair (2 g - c on both sides; 0 for hz = inf); face data,
// where given, enters every Dirichlet ghost as 2 g - c.
constexpr int P2W = 4;    // wavefronts per workgroup, stacked in row chunks
constexpr int P2OX = 62;  // coarse columns (column pairs) per wavefront

struct Grid2D {
  int gx, gy, jc, nblk;
};

// npx column pairs, npy row pairs; chunks sized for ~4096 wavefronts
static Grid2D grid_2d(int npx, int npy) {
  Grid2D g;
  g.gx = (npx + P2OX - 1) / P2OX;
  const int chunks = std::max(1, (4096 + g.gx - 1) / g.gx);
  g.jc = std::max(4, (npy + chunks - 1) / chunks);
  const int nch = (npy + g.jc - 1) / g.jc;
  g.gy = (nch + P2W - 1) / P2W;
  g.nblk = g.gx * g.gy;
  return g;
}

template <typename TU, typename TR, bool RESTRICT>
__global__ __launch_bounds__(64 * P2W) void k_resid_2d(LevelView<TU> F, const TU* __restrict__ u,
                                                       const TU* __restrict__ b, TR* __restrict__ out, int jc,
                                                       int gx, double* __restrict__ part, Batch bt,
                                                       const int* __restrict__ stop) {
  {
    const long long mb = blockIdx.y;
    if (u != nullptr) u += mb * bt.s0;
    b += mb * bt.s0;
    if (out != nullptr) out += mb * (RESTRICT ? bt.s1 : bt.s0);
    part += mb * bt.part_stride;
    if (stop != nullptr) stop += mb * bt.stop_stride;
  }
  __shared__ double red[2][P2W];
  lds_poison(&red[0][0], 2 * P2W);
  lds_poison_sync();
  if (stop != nullptr && *stop) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nx = F.nx, ny = F.ny;
  const bool per = F.periodic != 0;
  const int tx = blockIdx.x % gx, ty = blockIdx.x / gx;
  const int npy = (ny + 1) / 2;
  const int J0 = (ty * P2W + w) * jc, J1 = min(J0 + jc, npy);  // wave-uniform
  const int I = tx * P2OX - 1 + lane;  // coarse column (unwrapped)
  const int c0u = 2 * I, c1u = 2 * I + 1;
  auto wrapx = [&](int c) { return per ? ((c % nx) + nx) % nx : min(max(c, 0), nx - 1); };
  auto wrapy = [&](int r) { return per ? ((r % ny) + ny) % ny : min(max(r, 0), ny - 1); };
  const int c0 = wrapx(c0u), c1 = wrapx(c1u);
  const bool own = lane >= 1 && lane <= 62;
  const bool in0 = own && c0u >= 0 && c0u < nx, in1 = own && c1u >= 0 && c1u < nx;
  const bool lo0 = !per && c0u == 0, hi0 = !per && c0u == nx - 1, hi1 = !per && c1u == nx - 1;
  const int cnx = nx / 2;

  auto ldrow = [&](const TU* a, int r, TU& v0, TU& v1) {
    const size_t ro = (size_t)wrapy(r) * nx;
    v0 = a[ro + c0];
    v1 = a[ro + c1];
  };
  // b - M u at row r, columns c0 / c1; (m0, m1) row r - 1, (p0, p1) row r + 1
  auto res = [&](TU m0, TU m1, TU x0, TU x1, TU p0, TU p1, int r, TU bv0, TU bv1, TU& r0, TU& r1) {
    TU xl = wshift<DPP_WAVE_SHR1>(x1), xr = wshift<DPP_WAVE_SHL1>(x0);  // columns 2I-1 and 2I+2
    TU xm0 = xl, xp0 = x1, xm1 = x0, xp1 = xr;
    TU z0 = (TU)0, z1 = (TU)0;  // z terms (periodic: the plane is its own neighbour)
    if (!per) {
      const int rc = min(max(r, 0), ny - 1);  // face index row (rows outside the box are not stored)
      if (lo0) xm0 = dir_ghost(F, 0, (size_t)rc, x0);
      if (hi0) xp0 = dir_ghost(F, 1, (size_t)rc, x0);
      if (hi1) xp1 = dir_ghost(F, 1, (size_t)rc, x1);
      if (r == 0) {
        m0 = dir_ghost(F, 2, (size_t)c0, x0);
        m1 = dir_ghost(F, 2, (size_t)c1, x1);
      }
      if (r == ny - 1) {
        p0 = dir_ghost(F, 3, (size_t)c0, x0);
        p1 = dir_ghost(F, 3, (size_t)c1, x1);
      }
      const size_t f0 = (size_t)rc * nx + c0, f1 = (size_t)rc * nx + c1;
      z0 = ((dir_ghost(F, 4, f0, x0) + dir_ghost(F, 5, f0, x0)) - (TU)2 * x0) * F.ihz2;
      z1 = ((dir_ghost(F, 4, f1, x1) + dir_ghost(F, 5, f1, x1)) - (TU)2 * x1) * F.ihz2;
    }
    r0 = bv0 - (((xm0 + xp0) - (TU)2 * x0) * F.ihx2 + ((m0 + p0) - (TU)2 * x0) * F.ihy2 + z0);
    r1 = bv1 - (((xm1 + xp1) - (TU)2 * x1) * F.ihx2 + ((m1 + p1) - (TU)2 * x1) * F.ihy2 + z1);
  };

  double s2 = 0.0, s1 = 0.0;
  if (J0 < J1) {
    TU w0a = 0, w0b = 0, w1a = 0, w1b = 0, w2a = 0, w2b = 0, w3a = 0, w3b = 0;  // u rows 2J-1 .. 2J+2
    TU b0a, b0b, b1a, b1b;                                                        // b rows 2J, 2J+1
    if (u != nullptr) {
      ldrow(u, 2 * J0 - 1, w0a, w0b);
      ldrow(u, 2 * J0, w1a, w1b);
      ldrow(u, 2 * J0 + 1, w2a, w2b);
      ldrow(u, 2 * J0 + 2, w3a, w3b);
    }
    ldrow(b, 2 * J0, b0a, b0b);
    ldrow(b, 2 * J0 + 1, b1a, b1b);
    for (int J = J0; J < J1; ++J) {
      TU n3a = 0, n3b = 0, n4a = 0, n4b = 0, nb0a = 0, nb0b = 0, nb1a = 0, nb1b = 0;
      if (J + 1 < J1) {
        if (u != nullptr) {
          ldrow(u, 2 * J + 3, n3a, n3b);
          ldrow(u, 2 * J + 4, n4a, n4b);
        }
        ldrow(b, 2 * J + 2, nb0a, nb0b);
        ldrow(b, 2 * J + 3, nb1a, nb1b);
      }
      const int ra = 2 * J, rb = 2 * J + 1;
      TU r00, r01, r10, r11;
      res(w0a, w0b, w1a, w1b, w2a, w2b, ra, b0a, b0b, r00, r01);
      res(w1a, w1b, w2a, w2b, w3a, w3b, rb, b1a, b1b, r10, r11);
      const bool rowb = rb < ny;
      if (in0) s2 += (double)r00 * (double)r00 + (rowb ? (double)r10 * (double)r10 : 0.0);
      if (in1) s2 += (double)r01 * (double)r01 + (rowb ? (double)r11 * (double)r11 : 0.0);
      if (RESTRICT) {
        if (own && I >= 0 && I < cnx) {
          const TU v = ((r00 + r01) + (r10 + r11)) * (TU)0.25;
          out[(size_t)J * cnx + I] = (TR)v;
          s1 += (double)v;
        }
      } else {
        if (in0) {
          s1 += (double)r00 + (rowb ? (double)r10 : 0.0);
          if (out != nullptr) {
            out[(size_t)ra * nx + c0u] = (TR)r00;
            if (rowb) out[(size_t)rb * nx + c0u] = (TR)r10;
          }
        }
        if (in1) {
          s1 += (double)r01 + (rowb ? (double)r11 : 0.0);
          if (out != nullptr) {
            out[(size_t)ra * nx + c1u] = (TR)r01;
            if (rowb) out[(size_t)rb * nx + c1u] = (TR)r11;
          }
        }
      }
      w0a = w2a; w0b = w2b;
      w1a = w3a; w1b = w3b;
      w2a = n3a; w2b = n3b;
      w3a = n4a; w3b = n4b;
      b0a = nb0a; b0b = nb0b;
      b1a = nb1a; b1b = nb1b;
    }
  }
  const double t2 = wave_sum_dpp(s2), t1 = wave_sum_dpp(s1);
  if (lane == 0) {
    red[0][w] = t2;
    red[1][w] = t1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
#pragma unroll
    for (int q = 0; q < P2W; ++q) {
      a += red[0][q];
      c += red[1][q];
    }
    part[2 * (size_t)blockIdx.x] = a;
    part[2 * (size_t)blockIdx.x + 1] = c;
  }
}

// fine += P(e) on a single-plane level: (9, 3, 3, 1)/16 weights of eq.
// prolongation_example_2D; coarse ghosts wrap (periodic) or take -e
// (homogeneous Dirichlet, a corner ghost the product of both signs)
template <typename T>
__global__ __launch_bounds__(64 * P2W) void k_prolong_2d(int fnx, int fny, int periodic, const T* __restrict__ e,
                                                         T* __restrict__ fine, int jc, int gx, Batch bt,
                                                         const int* __restrict__ stop) {
  {
    const long long mb = blockIdx.y;
    e += mb * bt.s1;
    fine += mb * bt.s0;
    if (stop != nullptr) stop += mb * bt.stop_stride;
  }
  if (stop != nullptr && *stop) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int cnx = fnx / 2, cny = fny / 2;
  const bool per = periodic != 0;
  const int tx = blockIdx.x % gx, ty = blockIdx.x / gx;
  const int J0 = (ty * P2W + w) * jc, J1 = min(J0 + jc, cny);
  const int I = tx * P2OX - 1 + lane;
  int Iw = I;
  T sx = (T)1;
  if (per) Iw = ((I % cnx) + cnx) % cnx;
  else if (I < 0 || I >= cnx) { Iw = min(max(I, 0), cnx - 1); sx = (T)-1; }
  const bool own = lane >= 1 && lane <= 62 && I >= 0 && I < cnx;
  // coarse row J (unwrapped) at this lane's column, and its x neighbours by DPP
  auto ldc = [&](int J, T& c, T& cm, T& cp) {
    int Jw = J;
    T sy = (T)1;
    if (per) Jw = ((J % cny) + cny) % cny;
    else if (J < 0 || J >= cny) { Jw = min(max(J, 0), cny - 1); sy = (T)-1; }
    c = sx * sy * e[(size_t)Jw * cnx + Iw];
    cm = wshift<DPP_WAVE_SHR1>(c);
    cp = wshift<DPP_WAVE_SHL1>(c);
  };
  if (J0 >= J1) return;
  T am, amm, amp, ac, acm, acp, ap, apm, app;  // rows J-1, J, J+1: value, x-1, x+1
  ldc(J0 - 1, am, amm, amp);
  ldc(J0, ac, acm, acp);
  const size_t f0 = (size_t)(2 * I);
  auto ldf = [&](int r, T& v0, T& v1) {
    v0 = (T)0;
    v1 = (T)0;
    if (own && r < fny) {
      v0 = fine[(size_t)r * fnx + f0];
      v1 = fine[(size_t)r * fnx + f0 + 1];
    }
  };
  T u0a, u0b, u1a, u1b;
  ldf(2 * J0, u0a, u0b);
  ldf(2 * J0 + 1, u1a, u1b);
  for (int J = J0; J < J1; ++J) {
    ldc(J + 1, ap, apm, app);
    T n0a = 0, n0b = 0, n1a = 0, n1b = 0;
    if (J + 1 < J1) {
      ldf(2 * J + 2, n0a, n0b);
      ldf(2 * J + 3, n1a, n1b);
    }
    const T k = (T)(1.0 / 16.0);
    // fine (2I, 2J): neighbours I-1, J-1; (2I+1, 2J): I+1, J-1; (2I, 2J+1): I-1, J+1; (2I+1, 2J+1): I+1, J+1
    const T p00 = ((T)9 * ac + (T)3 * (acm + am) + amm) * k;
    const T p01 = ((T)9 * ac + (T)3 * (acp + am) + amp) * k;
    const T p10 = ((T)9 * ac + (T)3 * (acm + ap) + apm) * k;
    const T p11 = ((T)9 * ac + (T)3 * (acp + ap) + app) * k;
    if (own) {
      fine[(size_t)(2 * J) * fnx + f0] = u0a + p00;
      fine[(size_t)(2 * J) * fnx + f0 + 1] = u0b + p01;
      fine[(size_t)(2 * J + 1) * fnx + f0] = u1a + p10;
      fine[(size_t)(2 * J + 1) * fnx + f0 + 1] = u1b + p11;
    }
    am = ac; amm = acm; amp = acp;
    ac = ap; acm = apm; acp = app;
    u0a = n0a; u0b = n0b; u1a = n1a; u1b = n1b;
  }
}

// ---------------------------------------------------------------- launchers
struct TileGrid {
  int gx, gy, gz, kc, nblk;
};

static TileGrid resid_grid(int nx, int ny, int nz) {
  TileGrid g;
  g.gx = (nx + RBX - 1) / RBX;
  g.gy = (ny + RBY - 1) / RBY;
  const int npair = (nz + 1) / 2;
  const int xy = g.gx * g.gy;
  int chunks = (1024 + xy - 1) / xy;
  chunks = std::max(1, std::min(chunks, npair));
  g.kc = std::max(1, std::min(8, (npair + chunks - 1) / chunks));
  g.gz = (npair + g.kc - 1) / g.kc;
  g.nblk = g.gx * g.gy * g.gz;
  return g;
}

size_t resid_blocks(int nx, int ny, int nz) {
  if (nz == 1) return (size_t)grid_2d((nx + 1) / 2, (ny + 1) / 2).nblk;
  return (size_t)resid_grid(nx, ny, nz).nblk;
}

template <typename TU, typename TR>
void launch_residual(const LevelView<TU>& L, const TU* u, const TU* b, TR* r_out, double* part,
                     const int* stop, hipStream_t st, const Batch& bt) {
  if (L.nz == 1) {
    const Grid2D g = grid_2d((L.nx + 1) / 2, (L.ny + 1) / 2);
    hipLaunchKernelGGL((k_resid_2d<TU, TR, false>), dim3(g.nblk, bt.nb), dim3(64 * P2W), 0, st, L, u, b, r_out,
                       g.jc, g.gx, part, bt, stop);
    return;
  }
  const TileGrid g = resid_grid(L.nx, L.ny, L.nz);
  hipLaunchKernelGGL((k_resid_tile<TU, TR, false>), dim3(g.nblk, bt.nb), dim3(RNT), 0, st, L, u, b, r_out,
                     g.kc, g.gx, g.gy, g.nblk, part, bt, stop, (const float*)nullptr, (TU*)nullptr);
}

void launch_residual_add(const LevelView<double>& L, const double* u, const float* e, const double* b,
                         double* u_out, float* r_out, double* part, const int* stop, hipStream_t st) {
  if (L.nz == 1) fail(RKL_EINVAL, "the folded update is built for 3-D levels");
  if (u == nullptr || e == nullptr || u_out == nullptr || r_out == nullptr || u_out == u)
    fail(RKL_EINVAL, "folded update: bad buffers");
  const TileGrid g = resid_grid(L.nx, L.ny, L.nz);
  const Batch bt = single_batch();
  hipLaunchKernelGGL((k_resid_tile<double, float, false, true>), dim3(g.nblk, 1), dim3(RNT), 0, st, L, u, b, r_out,
                     g.kc, g.gx, g.gy, g.nblk, part, bt, stop, e, u_out);
}

template <typename T>
void launch_resid_restrict(const LevelView<T>& F, const T* u, const T* b, T* bc, double* part,
                           const int* stop, hipStream_t st, const Batch& bt) {
  if (F.nz == 1) {  // restriction happens below the finest level only: no face data
    const Grid2D g = grid_2d(F.nx / 2, F.ny / 2);
    hipLaunchKernelGGL((k_resid_2d<T, T, true>), dim3(g.nblk, bt.nb), dim3(64 * P2W), 0, st, F, u, b, bc, g.jc,
                       g.gx, part, bt, stop);
    return;
  }
  const TileGrid g = resid_grid(F.nx, F.ny, F.nz);
  hipLaunchKernelGGL((k_resid_tile<T, T, true>), dim3(g.nblk, bt.nb), dim3(RNT), 0, st, F, u, b, bc, g.kc,
                     g.gx, g.gy, g.nblk, part, bt, stop, (const float*)nullptr, (T*)nullptr);
}

template <typename T>
void launch_prolong_add(int fnx, int fny, int fnz, int periodic, const T* e, T* fine, const int* stop,
                        hipStream_t st, const Batch& bt) {
  if (fnz == 1) {
    const Grid2D g2 = grid_2d(fnx / 2, fny / 2);
    hipLaunchKernelGGL(k_prolong_2d<T>, dim3(g2.nblk, bt.nb), dim3(64 * P2W), 0, st, fnx, fny, periodic, e, fine,
                       g2.jc, g2.gx, bt, stop);
    return;
  }
  TileGrid g;
  g.gx = (fnx + PBX - 1) / PBX;
  g.gy = (fny + PBY - 1) / PBY;
  const int xy = g.gx * g.gy;
  int chunks = (1024 + xy - 1) / xy;
  chunks = std::max(1, std::min(chunks, fnz / 2));
  g.kc = std::max(2, std::min(16, (fnz + chunks - 1) / chunks));
  g.kc += g.kc & 1;  // even: chunks start on a coarse plane
  g.gz = (fnz + g.kc - 1) / g.kc;
  g.nblk = g.gx * g.gy * g.gz;
  hipLaunchKernelGGL(k_prolong_tile<T>, dim3(g.nblk, bt.nb), dim3(PNT), 0, st, fnx, fny, fnz, periodic, e,
                     fine, g.kc, g.gx, g.gy, g.nblk, bt, stop);
}

template void launch_residual<double, double>(const LevelView<double>&, const double*, const double*,
                                              double*, double*, const int*, hipStream_t, const Batch&);
template void launch_residual<double, float>(const LevelView<double>&, const double*, const double*,
                                             float*, double*, const int*, hipStream_t, const Batch&);
template void launch_residual<float, float>(const LevelView<float>&, const float*, const float*, float*,
                                            double*, const int*, hipStream_t, const Batch&);
template void launch_resid_restrict<double>(const LevelView<double>&, const double*, const double*,
                                            double*, double*, const int*, hipStream_t, const Batch&);
template void launch_resid_restrict<float>(const LevelView<float>&, const float*, const float*, float*,
                                           double*, const int*, hipStream_t, const Batch&);
template void launch_prolong_add<double>(int, int, int, int, const double*, double*, const int*,
                                         hipStream_t, const Batch&);
template void launch_prolong_add<float>(int, int, int, int, const float*, float*, const int*, hipStream_t,
                                        const Batch&);

}  // namespace rkl
