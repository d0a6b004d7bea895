// Fused s-stage RKL tau-step: all stages of one tau-step (App. A eq.
// RKL_intermediate_source) in a single HBM pass.
//
// Each workgroup owns a BX x BY output tile and a chunk of z planes and
// marches upward through z.  Plane by plane it keeps, in LDS rings of three
// planes, the stage values Y_0 (= u), Y_1, ..., Y_{S-1} over the tile plus a
// halo that shrinks by one cell per stage (Y_j is needed on a halo of S - j
// cells so that stage j+1 has its 7-point stencil).  Stage j of plane p runs
// in the iteration that loads u plane p + j, so Y_{j-1} on planes p-1, p, p+1
// and Y_{j-2} on plane p are resident.  Y_S goes straight to HBM, so u and b
// are read once and Y_S is written once: 3 words per cell instead of the
// 3 + 4 (s - 1) words of stage-by-stage sweeps.  The next u plane is loaded
// into registers while the current stages compute.
//
// Boundaries: periodic tiles fetch wrapped halo planes and compute the halo
// stages as the periodic images they are; Dirichlet stencils that leave the
// box use the ghost of Sec. 2.3 built from the centre value (2 g - c on the
// finest level with data, -c otherwise).  Optionally the kernel also returns
// the float64 partial sums of (M u - b)^2 over its output cells (the residual
// of the tau-step's input), so a convergence check costs no extra pass.
#include <map>
#include <mutex>
#include <tuple>

#include "host_common.h"
#include "kernels.h"

namespace rkl {

constexpr int FNT = 256;


__device__ __forceinline__ int slot3(int p) { return (p % 3 + 3) % 3; }

template <typename T, int S, int BX, int BY>
__global__ __launch_bounds__(FNT) void k_fused_tau(LevelView<T> L, const T* __restrict__ u,
                                                   const T* __restrict__ b, T* __restrict__ out,
                                                   FCoef<T, S> co, int zc, int gx_tiles, int gy_tiles,
                                                   int nblk, double* __restrict__ part,
                                                   Batch bt, const int* __restrict__ stop) {
  {
    const long long mb = blockIdx.y;
    if (u != nullptr) u += mb * bt.s0;
    b += mb * bt.s0;
    out += mb * bt.s0;
    if (part != nullptr) part += mb * bt.part_stride;
    if (stop != nullptr) stop += mb * bt.stop_stride;
  }
  constexpr int W = BX + 2 * S, H = BY + 2 * S, PL = W * H;
  constexpr int NU = (PL + FNT - 1) / FNT;                                      // u slots per thread
  constexpr int NB = ((BX + 2 * S - 2) * (BY + 2 * S - 2) + FNT - 1) / FNT;     // stage slots (stage 1 is largest)
  __shared__ T ring[S][3][PL];
  __shared__ double red[FNT / WAVE];
  lds_poison(&ring[0][0][0], S * 3 * PL);
  lds_poison(red, FNT / WAVE);
  lds_poison_sync();

  if (stop != nullptr && *stop) return;
  const int tid = threadIdx.x;
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const bool per = L.periodic != 0;
  const size_t sxy = (size_t)nx * ny;

  // XCD-aware tile order: consecutive workgroups are dealt round-robin to the
  // 8 XCDs, so give each XCD a contiguous run of tiles (its halos then meet
  // in that XCD's L2).
  int bid = blockIdx.x;
  if ((nblk & 7) == 0) bid = (bid & 7) * (nblk >> 3) + (bid >> 3);
  const int tx = bid % gx_tiles;
  const int ty = (bid / gx_tiles) % gy_tiles;
  const int tz = bid / (gx_tiles * gy_tiles);
  const int x0 = tx * BX - S, y0 = ty * BY - S;  // origin of the haloed plane
  const int z0 = tz * zc, z1 = min(z0 + zc, nz);

  // u-load slots: global xy offset (-1: outside a Dirichlet box)
  int goff[NU];
#pragma unroll
  for (int q = 0; q < NU; ++q) {
    const int idx = tid + q * FNT;
    goff[q] = -1;
    if (idx < PL) {
      const int gxr = x0 + idx % W, gyr = y0 + idx / W;
      if (per) goff[q] = ((gyr % ny + ny) % ny) * nx + (gxr % nx + nx) % nx;
      else if (gxr >= 0 && gxr < nx && gyr >= 0 && gyr < ny) goff[q] = gyr * nx + gxr;
    }
  }
  // stage slots, fixed for the whole z march: LDS offset, wrapped global
  // coordinates and flags (bit 0 active, bit 1 owned output cell)
  int so[S][NB], sgx[S][NB], sgy[S][NB], sfl[S][NB];
#pragma unroll
  for (int j = 1; j <= S; ++j) {
    const int hj = S - j;
    const int Wj = BX + 2 * hj, Hj = BY + 2 * hj;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int idx = tid + k * FNT;
      so[j - 1][k] = 0;
      sgx[j - 1][k] = 0;
      sgy[j - 1][k] = 0;
      sfl[j - 1][k] = 0;
      if (idx < Wj * Hj) {
        const int lx = idx % Wj + (S - hj), ly = idx / Wj + (S - hj);
        const int gxr = x0 + lx, gyr = y0 + ly;
        const bool inbox = gxr >= 0 && gxr < nx && gyr >= 0 && gyr < ny;
        so[j - 1][k] = ly * W + lx;
        sgx[j - 1][k] = per ? (gxr % nx + nx) % nx : gxr;
        sgy[j - 1][k] = per ? (gyr % ny + ny) % ny : gyr;
        const bool active = per || inbox;
        const bool own = inbox && lx >= S && lx < S + BX && ly >= S && ly < S + BY;
        sfl[j - 1][k] = (active ? 1 : 0) | (own ? 2 : 0);
      }
    }
  }
  auto plane_ok = [&](int p) { return per || (p >= 0 && p < nz); };
  auto zw = [&](int p) { return per ? (p % nz + nz) % nz : p; };
  auto stage_on = [&](int j, int p) {
    const int hj = S - j;
    return p >= z0 - hj && p <= z1 - 1 + hj && plane_ok(p);
  };

  // register prefetch of the next iteration's u plane and stage right-hand sides
  T pre[NU];
  T bnx[S][NB];
  auto prefetch = [&](int zl) {
    {
      const bool ok = plane_ok(zl);
      const size_t zo = ok ? (size_t)zw(zl) * sxy : 0;
#pragma unroll
      for (int q = 0; q < NU; ++q) pre[q] = (ok && u != nullptr && goff[q] >= 0) ? u[zo + goff[q]] : (T)0;
    }
#pragma unroll
    for (int j = 1; j <= S; ++j) {
      const int p = zl - j;
      const bool on = stage_on(j, p);
      const size_t zo = on ? (size_t)zw(p) * sxy : 0;
#pragma unroll
      for (int k = 0; k < NB; ++k)
        bnx[j - 1][k] = (on && (sfl[j - 1][k] & 1)) ? b[zo + (size_t)sgy[j - 1][k] * nx + sgx[j - 1][k]] : (T)0;
    }
  };

  const int zlast = z1 - 1 + S;
  double r2 = 0.0;
  prefetch(z0 - S);
  for (int zl = z0 - S; zl <= zlast; ++zl) {
    T bcur[S][NB];
#pragma unroll
    for (int j = 0; j < S; ++j)
#pragma unroll
      for (int k = 0; k < NB; ++k) bcur[j][k] = bnx[j][k];
    {
      T* dst = ring[0][slot3(zl)];
#pragma unroll
      for (int q = 0; q < NU; ++q) {
        const int idx = tid + q * FNT;
        if (idx < PL) dst[idx] = pre[q];
      }
    }
    __syncthreads();
    if (zl < zlast) prefetch(zl + 1);

#pragma unroll
    for (int j = 1; j <= S; ++j) {
      const int p = zl - j;
      if (stage_on(j, p)) {
        const int hj = S - j;
        const int nreg = (BX + 2 * hj) * (BY + 2 * hj);
        const T* Ym = ring[j - 1][slot3(p - 1)];
        const T* Yc = ring[j - 1][slot3(p)];
        const T* Yq = ring[j - 1][slot3(p + 1)];
        const T* Y2 = ring[j >= 2 ? j - 2 : 0][slot3(p)];
        T* Yw = ring[j < S ? j : 0][slot3(p)];
        const size_t zo = (size_t)zw(p) * sxy;
        const bool zlo = per || p > 0, zhi = per || p < nz - 1;
        const bool pown = p >= z0 && p < z1;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          if (tid + k * FNT >= nreg) break;
          const int fl = sfl[j - 1][k];
          if (!(fl & 1)) continue;
          const int o = so[j - 1][k];
          const int gx = sgx[j - 1][k], gy = sgy[j - 1][k];
          const T c = Yc[o];
          T xm = Yc[o - 1], xp = Yc[o + 1], ym = Yc[o - W], yp = Yc[o + W];
          T zm = Ym[o], zp = Yq[o];
          if (!per) {
            if (gx == 0) xm = dir_ghost(L, 0, (size_t)p * ny + gy, c);
            if (gx == nx - 1) xp = dir_ghost(L, 1, (size_t)p * ny + gy, c);
            if (gy == 0) ym = dir_ghost(L, 2, (size_t)p * nx + gx, c);
            if (gy == ny - 1) yp = dir_ghost(L, 3, (size_t)p * nx + gx, c);
            if (!zlo) zm = dir_ghost(L, 4, (size_t)gy * nx + gx, c);
            if (!zhi) zp = dir_ghost(L, 5, (size_t)gy * nx + gx, c);
          }
          const T lap = ((xm + xp) - (T)2 * c) * L.ihx2 + ((ym + yp) - (T)2 * c) * L.ihy2 +
                        ((zm + zp) - (T)2 * c) * L.ihz2;
          const T r = lap - bcur[j - 1][k];
          const bool own = (fl & 2) && pown;
          T y;
          if (j == 1) {
            y = c + co.c[0] * r;
            if (part != nullptr && own) r2 += (double)r * (double)r;
          } else {
            y = co.mu[j - 1] * c + co.nu[j - 1] * Y2[o] + co.c[j - 1] * r;
          }
          if (j < S) Yw[o] = y;
          else if (own) out[zo + (size_t)gy * nx + gx] = y;
        }
      }
      __syncthreads();
    }
  }
  if (part != nullptr) {
    const double t = block_sum<FNT>(r2, red);
    if (tid == 0) part[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------- z-queue variant
// Same algorithm, different storage: every thread owns fixed (x, y) columns
// of the stage-1 region for the whole z march and keeps, per column, register
// queues of the last three planes of u and of Y_1 .. Y_{S-1} (the z
// neighbours) and of b for the planes the stages are working on.  LDS holds
// only the plane each stage reads its x/y neighbours from: u's current plane
// and, double-buffered, the current plane of Y_1 .. Y_{S-1}.  So b is read once
// per cell, a tile can be larger for the same LDS, and the outputs of Y_S are
// stored one iteration later, together with the next prefetch.
template <typename T, int S, int BX, int BY, int NT, int PD, int DS>
__global__ __launch_bounds__(NT) void k_tau_zq(LevelView<T> L, const T* __restrict__ u, const T* __restrict__ b,
                                               T* __restrict__ out, FCoef<T, S> co, int zc, int gx_tiles,
                                               int gy_tiles, int nblk, double* __restrict__ part,
                                               Batch bt, const int* __restrict__ stop) {
  {
    const long long mb = blockIdx.y;
    if (u != nullptr) u += mb * bt.s0;
    b += mb * bt.s0;
    out += mb * bt.s0;
    if (part != nullptr) part += mb * bt.part_stride;
    if (stop != nullptr) stop += mb * bt.stop_stride;
  }
  constexpr int W0 = BX + 2 * S, H0 = BY + 2 * S, P0 = W0 * H0;          // haloed u plane
  constexpr int W1 = W0 - 2, H1 = H0 - 2, P1 = W1 * H1;                  // stage-1 region = slot region
  constexpr int NB = (P1 + NT - 1) / NT;
  constexpr int NRING = P0 - P1;
  constexpr int NR = (NRING + NT - 1) / NT;
  constexpr int NY = S > 1 ? S - 1 : 1;
  __shared__ T su[P0];
  __shared__ T sy[NY][2][P0];
  __shared__ double red[NT / WAVE];
  lds_poison(su, P0);
  lds_poison(&sy[0][0][0], NY * 2 * P0);
  lds_poison(red, NT / WAVE);
  lds_poison_sync();

  if (stop != nullptr && *stop) return;
  const int tid = threadIdx.x;
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const bool per = L.periodic != 0;
  const size_t sxy = (size_t)nx * ny;
  int bid = blockIdx.x;
  if ((nblk & 7) == 0) bid = (bid & 7) * (nblk >> 3) + (bid >> 3);
  const int tx = bid % gx_tiles;
  const int ty = (bid / gx_tiles) % gy_tiles;
  const int tz = bid / (gx_tiles * gy_tiles);
  const int x0 = tx * BX - S, y0 = ty * BY - S;
  const int z0 = tz * zc, z1 = min(z0 + zc, nz);

  // slot metadata: LDS offset, wrapped global xy offset, flags: bits 0-7
  // depth (distance to the haloed plane's edge), bit 8 active, bit 9 owned
  // output cell, bits 10-13 on the x-, x+, y-, y+ face of a Dirichlet box
  int sg[NB], sf[NB];
  auto so = [&](int k) {  // LDS offset of slot k (compile-time divisors)
    const int idx = tid + k * NT;
    return (idx / W1 + 1) * W0 + idx % W1 + 1;
  };
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int idx = tid + k * NT;
    sg[k] = 0;
    sf[k] = 0;
    if (idx < P1) {
      const int lx = idx % W1 + 1, ly = idx / W1 + 1;
      const int gxr = x0 + lx, gyr = y0 + ly;
      const bool inbox = gxr >= 0 && gxr < nx && gyr >= 0 && gyr < ny;
      const int gx = per ? (gxr % nx + nx) % nx : gxr;
      const int gy = per ? (gyr % ny + ny) % ny : gyr;
      const int d = min(min(lx, ly), min(W0 - 1 - lx, H0 - 1 - ly));
      const bool active = per || inbox;
      const bool own = inbox && d >= S;
      sg[k] = active ? gy * nx + gx : 0;
      int bf = 0;
      if (!per && inbox) bf = (gx == 0 ? 1 : 0) | (gx == nx - 1 ? 2 : 0) | (gy == 0 ? 4 : 0) | (gy == ny - 1 ? 8 : 0);
      sf[k] = d | (active ? 256 : 0) | (own ? 512 : 0) | (bf << 10);
    }
  }
  // ring positions: the outer edge of the haloed plane
  int ro[NR], rg[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int idx = tid + r * NT;
    ro[r] = -1;
    rg[r] = -1;
    if (idx < NRING) {
      int lx, ly;
      if (idx < W0) { lx = idx; ly = 0; }
      else if (idx < 2 * W0) { lx = idx - W0; ly = H0 - 1; }
      else if (idx < 2 * W0 + H0 - 2) { lx = 0; ly = idx - 2 * W0 + 1; }
      else { lx = W0 - 1; ly = idx - 2 * W0 - (H0 - 2) + 1; }
      ro[r] = ly * W0 + lx;
      const int gxr = x0 + lx, gyr = y0 + ly;
      if (per) rg[r] = ((gyr % ny + ny) % ny) * nx + (gxr % nx + nx) % nx;
      else if (gxr >= 0 && gxr < nx && gyr >= 0 && gyr < ny) rg[r] = gyr * nx + gxr;
    }
  }
  auto plane_ok = [&](int p) { return per || (p >= 0 && p < nz); };
  auto zw = [&](int p) { return per ? (p % nz + nz) % nz : p; };
  auto stage_on = [&](int j, int p) {
    const int hj = S - j;
    return p >= z0 - hj && p <= z1 - 1 + hj && plane_ok(p);
  };

  T uq0[NB], uq1[NB], uq2[NB];   // u at planes zl-2, zl-1, zl
  T yq0[NY][NB], yq1[NY][NB], yq2[NY][NB];  // Y_j at planes zl-j-2, zl-j-1, zl-j
  T bq[S][NB];                   // bq[j-1] = b at plane zl-j
  T unx[NB], bnx[NB], rnx[NR];   // in flight: u(zl+1), b(zl), ring u(zl)
  T unx2[NB], bnx2[NB], rnx2[NR]; // two-deep prefetch (PD == 2): the set after
  T yst[DS ? NB : 1];            // Y_S awaiting its store (DS: deferred stores)
  int yso[DS ? NB : 1];          // its plane (or -1)
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    uq0[k] = uq1[k] = uq2[k] = (T)0;
    for (int j = 0; j < NY; ++j) yq0[j][k] = yq1[j][k] = yq2[j][k] = (T)0;
    for (int j = 0; j < S; ++j) bq[j][k] = (T)0;
    if (DS) {
      yst[DS ? k : 0] = (T)0;
      yso[DS ? k : 0] = -1;
    }
  }
  auto prefetch_to = [&](int zl, T (&un)[NB], T (&bn)[NB], T (&rn)[NR]) {
    // u(zl + 1) and b(zl) at the slots, u(zl) on the ring
    {
      const int p = zl + 1;
      const bool ok = u != nullptr && plane_ok(p);
      const size_t zo = ok ? (size_t)zw(p) * sxy : 0;
#pragma unroll
      for (int k = 0; k < NB; ++k) un[k] = (ok && (sf[k] & 256)) ? u[zo + sg[k]] : (T)0;
    }
    {
      const int p = zl;
      const bool ok = u != nullptr && plane_ok(p);
      const size_t zo = ok ? (size_t)zw(p) * sxy : 0;
#pragma unroll
      for (int r = 0; r < NR; ++r) rn[r] = (ok && rg[r] >= 0) ? u[zo + rg[r]] : (T)0;
    }
    {
      const int p = zl;
      const bool ok = plane_ok(p) && p >= z0 - (S - 1) && p <= z1 - 1 + (S - 1);
      const size_t zo = ok ? (size_t)zw(p) * sxy : 0;
#pragma unroll
      for (int k = 0; k < NB; ++k) bn[k] = (ok && (sf[k] & 256)) ? b[zo + sg[k]] : (T)0;
    }
  };
  auto flush = [&]() {
    if (!DS) return;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      if (yso[DS ? k : 0] >= 0) out[(size_t)yso[DS ? k : 0] * sxy + sg[k]] = yst[DS ? k : 0];
      yso[DS ? k : 0] = -1;
    }
  };

  const int zfirst = z0 - S, zlast = z1 - 1 + S;
  double r2 = 0.0;
  // state before iteration zfirst: u(zfirst) and u(zfirst - 1) needed
  prefetch_to(zfirst - 1, unx, bnx, rnx);  // u(zfirst), ring u(zfirst - 1), b(zfirst - 1)
  if (PD == 2 && zfirst < zlast) prefetch_to(zfirst, unx2, bnx2, rnx2);
  {
    // u(zfirst - 1) at the slots seeds the queue
    const int p = zfirst - 1;
    const bool ok = u != nullptr && plane_ok(p);
    const size_t zo = ok ? (size_t)zw(p) * sxy : 0;
#pragma unroll
    for (int k = 0; k < NB; ++k) uq2[k] = (ok && (sf[k] & 256)) ? u[zo + sg[k]] : (T)0;
  }
  for (int zl = zfirst; zl <= zlast; ++zl) {
    // shift the queues: u(zl) arrives, b(zl - 1) arrives
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      uq0[k] = uq1[k];
      uq1[k] = uq2[k];
      uq2[k] = unx[k];
#pragma unroll
      for (int j = S - 1; j > 0; --j) bq[j][k] = bq[j - 1][k];
      bq[0][k] = bnx[k];
    }
    // u's current plane (zl - 1) into LDS: slots from the queue, ring from flight
#pragma unroll
    for (int k = 0; k < NB; ++k)
      if (tid + k * NT < P1) su[so(k)] = uq1[k];
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (ro[r] >= 0) su[ro[r]] = rnx[r];
    __syncthreads();
    flush();
    if (PD == 2) {
      // the set in flight moves up; the one after it is issued now
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        unx[q] = unx2[q];
        bnx[q] = bnx2[q];
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) rnx[r] = rnx2[r];
      if (zl + 1 < zlast) prefetch_to(zl + 1, unx2, bnx2, rnx2);
    } else {
      if (zl < zlast) prefetch_to(zl, unx, bnx, rnx);
    }

#pragma unroll
    for (int j = 1; j <= S; ++j) {
      const int p = zl - j;
      const bool on = stage_on(j, p);
      const bool zlo = per || p > 0, zhi = per || p < nz - 1;
      const bool pown = p >= z0 && p < z1;
      const T* Xc = (j == 1) ? su : sy[j >= 2 ? j - 2 : 0][p & 1];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const int fl = sf[k];
        T y = (T)0;
        const bool act = on && (fl & 256) && (fl & 255) >= j && (tid + k * NT < P1);
        if (act) {
          const int o = so(k);
          T c, zm, zp, y2;
          if (j == 1) {
            c = uq1[k];
            zm = uq0[k];
            zp = uq2[k];
            y2 = (T)0;
          } else {
            c = yq1[j - 2][k];
            zm = yq0[j - 2][k];
            zp = yq2[j - 2][k];
            y2 = (j == 2) ? uq0[k] : yq0[j >= 3 ? j - 3 : 0][k];
          }
          T xm = Xc[o - 1], xp = Xc[o + 1], ym = Xc[o - W0], yp = Xc[o + W0];
          if (!per && ((fl >> 10) != 0 || !zlo || !zhi)) {
            const int gy = sg[k] / nx, gx = sg[k] - gy * nx;
            if (fl & (1 << 10)) xm = dir_ghost(L, 0, (size_t)p * ny + gy, c);
            if (fl & (2 << 10)) xp = dir_ghost(L, 1, (size_t)p * ny + gy, c);
            if (fl & (4 << 10)) ym = dir_ghost(L, 2, (size_t)p * nx + gx, c);
            if (fl & (8 << 10)) yp = dir_ghost(L, 3, (size_t)p * nx + gx, c);
            if (!zlo) zm = dir_ghost(L, 4, (size_t)gy * nx + gx, c);
            if (!zhi) zp = dir_ghost(L, 5, (size_t)gy * nx + gx, c);
          }
          const T lap = ((xm + xp) - (T)2 * c) * L.ihx2 + ((ym + yp) - (T)2 * c) * L.ihy2 +
                        ((zm + zp) - (T)2 * c) * L.ihz2;
          const T r = lap - bq[j - 1][k];
          if (j == 1) {
            y = c + co.c[0] * r;
            if (part != nullptr && (fl & 512) && pown) r2 += (double)r * (double)r;
          } else {
            y = co.mu[j - 1] * c + co.nu[j - 1] * y2 + co.c[j - 1] * r;
          }
          if (j == S && (fl & 512) && pown) {
            if (DS) {
              yst[k] = y;
              yso[k] = zw(p);
            } else {
              out[(size_t)zw(p) * sxy + sg[k]] = y;
            }
          }
        }
        if (j < S) {
          yq0[j - 1][k] = yq1[j - 1][k];
          yq1[j - 1][k] = yq2[j - 1][k];
          yq2[j - 1][k] = y;
          if (act) sy[j - 1][p & 1][so(k)] = y;
        }
      }
      if (j < S) __syncthreads();
    }
    if (S == 1) __syncthreads();
  }
  flush();
  if (part != nullptr) {
    const double t = block_sum<NT>(r2, red);
    if (tid == 0) part[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------- launch
// Variants (tile family and shape) and the workgroup target that sets the
// z-chunk length.  Every variant computes the same cells with the same
// arithmetic; they differ only in how a level is cut into workgroups.
template <typename T, int S>
constexpr bool zq_instantiated() {
  return S == 2 || S == 3;
}

template <typename T>
constexpr int fused_max_s() {
  return sizeof(T) == 8 ? 3 : 4;
}

template <typename T, int S>
constexpr bool strip_instantiated() {
  return sizeof(T) == 8 ? S <= 2 : S <= 3;
}

// The 2-D strip kernel takes up to 4 stages in one pass (two s = 2 tau-steps
// of a pre-smoothing pair included): without y-halo rows its registers allow
// it, 8 x segments per lane up to s = 2 (float64) / 4 (float32), 4 beyond.
constexpr int STRIP2D_MAX_S = 4;
template <typename T, int S>
constexpr int strip2d_rows(bool want8) {
  return (want8 && (sizeof(T) == 4 || S <= 2)) ? 8 : 4;
}

// 2-D levels: the FLAT strip kernel only (face data folded beforehand)
template <typename T>
bool fused_tau_supported(const LevelView<T>& L, int s) {
  if (level_is_2d(L)) return s >= 1 && s <= STRIP2D_MAX_S && L.nx >= 16 && L.ny >= 8 && L.faces == nullptr;
  return s >= 1 && s <= fused_max_s<T>() && L.nx >= 16 && L.ny >= 8 && L.nz >= 8;
}

template <typename T>
bool fused_variant_ok(int variant, int s) {
  if (s < 1) return false;
  if (variant_is_2d(variant)) return s <= STRIP2D_MAX_S;
  if (s > fused_max_s<T>()) return false;
  const bool dbl = sizeof(T) == 8;
  switch (variant) {
    case FV_RING_64x8:
    case FV_RING_64x4: return true;
    case FV_ZQ_64x32:
    case FV_ZQ_64x16: return s == 2 || s == 3;
    case FV_STRIP_8x4:
    case FV_STRIP_8x1:
    case FV_STRIP_4x4:
    case FV_STRIP_5x1:
    case FV_STRIPYX_8x4:
    case FV_STRIPYX_8x8: return dbl ? s <= 2 : s <= 3;
    case FV_STRIPYX_4x8: return s <= 3;  // float64 s = 3: 239 VGPRs, 2 waves per SIMD
    case FV_STRIPYX_2x8:
    case FV_STRIPYX_2x16: return s <= 2;  // shared halo rows come from the R = 2 own rows
    default: return false;
  }
}

template <typename T>
static bool variant_fits(const LevelView<T>& L, int variant) {
  return variant_is_2d(variant) == level_is_2d(L);
}

static bool is_strip(int variant) {
  return variant == FV_STRIP_8x4 || variant == FV_STRIP_8x1 || variant == FV_STRIP_4x4 || variant == FV_STRIP_5x1 ||
         variant == FV_STRIPYX_8x4 || variant == FV_STRIPYX_4x8 || variant == FV_STRIPYX_8x8 ||
         variant == FV_STRIPYX_2x8 || variant == FV_STRIPYX_2x16;
}
static void strip_shape(int variant, int& R, int& WY) {
  switch (variant) {
    case FV_STRIP_8x4: R = 8; WY = 4; return;
    case FV_STRIP_8x1: R = 8; WY = 1; return;
    case FV_STRIP_4x4: R = 4; WY = 4; return;
    case FV_STRIP_5x1: R = 5; WY = 1; return;
    case FV_STRIPYX_8x4: R = 8; WY = 4; return;
    case FV_STRIPYX_4x8: R = 4; WY = 8; return;
    case FV_STRIPYX_8x8: R = 8; WY = 8; return;
    case FV_STRIPYX_2x8: R = 2; WY = 8; return;
    default: R = 2; WY = 16; return;  // FV_STRIPYX_2x16
  }
}

static void variant_tile(int variant, int& bx, int& by) {
  bx = 64;
  switch (variant) {
    case FV_RING_64x4: by = 4; break;
    case FV_ZQ_64x32: by = 32; break;
    case FV_ZQ_64x16: by = 16; break;
    default: by = 8; break;
  }
}

struct FusedGrid {
  int gx, gy, gz, zc, nblk;
};

// z chunks: aim for `target` workgroups; a chunk spans 4 .. zc_max planes
// (short chunks keep small levels from being one long serial march)
static FusedGrid fused_grid(int bx, int by, int nx, int ny, int nz, int target, int zc_max = 32) {
  FusedGrid g;
  g.gx = (nx + bx - 1) / bx;
  g.gy = (ny + by - 1) / by;
  const int xy = g.gx * g.gy;
  const int chunks = std::max(1, (target + xy - 1) / xy);
  g.zc = std::max(4, std::min(zc_max, (nz + chunks - 1) / chunks));
  g.gz = (nz + g.zc - 1) / g.zc;
  g.nblk = g.gx * g.gy * g.gz;
  return g;
}

size_t fused_tau_blocks_max(int nx, int ny, int nz) {
  // shortest chunk of each family (ring / z-queue: 4 planes; strip: 1 plane)
  // with its smallest tile: 64 x 4 (ring), 56 output columns x 4 rows (strip,
  // s <= 4; the 2-D form's segments are wider)
  const size_t ring = (size_t)((nx + 63) / 64) * ((ny + 3) / 4) * ((nz + 3) / 4);
  const size_t strip = (size_t)((nx + 55) / 56) * ((ny + 3) / 4) * (size_t)nz;
  // 2-D form: segments of >= 4 x 56 columns per wavefront, chunks of one row
  const size_t strip2d = nz == 1 ? (size_t)((nx + 223) / 224) * (size_t)ny : 0;
  return std::max(ring, std::max(strip, strip2d));
}

// ---- tuning table
namespace {
struct TuneKey {
  int nx, ny, nz, periodic, dbl, s;
  bool operator<(const TuneKey& o) const {
    return std::tie(nx, ny, nz, periodic, dbl, s) < std::tie(o.nx, o.ny, o.nz, o.periodic, o.dbl, o.s);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, FusedChoice> g_tune;
int g_tune_gen = 0;
}  // namespace

void tune_install(int nx, int ny, int nz, int periodic, int dbl, int s, FusedChoice c) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const TuneKey k{nx, ny, nz, periodic ? 1 : 0, dbl ? 1 : 0, s};
  if (c.variant == FV_HEUR) g_tune.erase(k);
  else g_tune[k] = c;
  ++g_tune_gen;
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  ++g_tune_gen;
}

int tune_generation() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_tune_gen;
}

// Built-in choice (what the tuner picked on gfx950 for most shapes): the
// strip kernel, 8-row strips for large float64 levels and 4-row strips
// otherwise; stage counts the strip kernel is not built for take the
// z-queue kernel on large levels and the LDS-ring kernel on small ones.
template <typename T>
FusedChoice fused_heuristic(const LevelView<T>& L, int s) {
  if (level_is_2d(L)) return FusedChoice{(sizeof(T) == 8 && s <= 2) ? FV_STRIP2D_8 : FV_STRIP2D_4, 2048};
  if (fused_variant_ok<T>(FV_STRIP_4x4, s)) {
    const bool big = (size_t)L.nx * L.ny * L.nz >= ((size_t)192 * 192 * 192);
    if (sizeof(T) == 8 && L.periodic && big) return FusedChoice{FV_STRIP_8x4, 1024};
    return FusedChoice{FV_STRIP_4x4, 1024};
  }
  if (fused_variant_ok<T>(FV_ZQ_64x32, s) && L.nx >= 128 && L.ny >= 128 && L.nz >= 64) return FusedChoice{FV_ZQ_64x32, 256};
  return FusedChoice{FV_RING_64x4, 1024};
}

template <typename T>
FusedChoice fused_choice(const LevelView<T>& L, int s) {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(TuneKey{L.nx, L.ny, L.nz, L.periodic ? 1 : 0, sizeof(T) == 8 ? 1 : 0, s});
    if (it != g_tune.end() && fused_variant_ok<T>(it->second.variant, s) && variant_fits(L, it->second.variant))
      return it->second;
  }
  return fused_heuristic<T>(L, s);
}

template <typename T, int S>
FCoef<T, S> make_fcoef(const StageCoef* co) {
  FCoef<T, S> fc;
  for (int j = 0; j < S; ++j) {
    fc.mu[j] = (T)co[j].mu;
    fc.nu[j] = (T)co[j].nu;
    fc.c[j] = (T)co[j].c;
  }
  return fc;
}

template <typename T, int S>
void launch_fused_S(const LevelView<T>& L, FusedChoice c, const T* u, const T* b, T* out, const StageCoef* co,
                    double* part, const int* stop, const Batch& bt, hipStream_t st) {
  const FCoef<T, S> fc = make_fcoef<T, S>(co);
  if (variant_is_2d(c.variant)) {
    if constexpr (S <= STRIP2D_MAX_S) {
      if (strip2d_rows<T, S>(c.variant == FV_STRIP2D_8) == 8)
        return launch_strip2d<T, S, strip2d_rows<T, S>(true), 1>(L, c.target, u, b, out, fc, part, stop, bt, st);
      return launch_strip2d<T, S, 4, 1>(L, c.target, u, b, out, fc, part, stop, bt, st);
    }
    return;  // not reached: fused_tau_supported bounds s on 2-D levels
  }
  if constexpr (S > fused_max_s<T>()) {
    return;  // not reached: 3-D levels take at most fused_max_s stages
  } else {
  if (is_strip(c.variant) && L.faces != nullptr) c = FusedChoice{FV_RING_64x8, 1024};  // strips take no face data
  if (is_strip(c.variant)) {
    if constexpr (sizeof(T) == 8 && S == 3) {
      if (c.variant == FV_STRIPYX_4x8)
        return launch_strip_yx<T, S, 4, 8>(L, c.target, u, b, out, fc, part, stop, bt, st);
    }
    if constexpr (strip_instantiated<T, S>()) {
      if (c.variant == FV_STRIP_8x4) return launch_strip<T, S, 8, 4>(L, c.target, u, b, out, fc, part, stop, bt, st);
      if (c.variant == FV_STRIP_8x1) return launch_strip<T, S, 8, 1>(L, c.target, u, b, out, fc, part, stop, bt, st);
      if (c.variant == FV_STRIP_4x4) return launch_strip<T, S, 4, 4>(L, c.target, u, b, out, fc, part, stop, bt, st);
      if (c.variant == FV_STRIP_5x1) return launch_strip<T, S, 5, 1>(L, c.target, u, b, out, fc, part, stop, bt, st);
      if (c.variant == FV_STRIPYX_8x4)
        return launch_strip_yx<T, S, 8, 4>(L, c.target, u, b, out, fc, part, stop, bt, st);
      if (c.variant == FV_STRIPYX_4x8)
        return launch_strip_yx<T, S, 4, 8>(L, c.target, u, b, out, fc, part, stop, bt, st);
      if (c.variant == FV_STRIPYX_8x8)
        return launch_strip_yx<T, S, 8, 8>(L, c.target, u, b, out, fc, part, stop, bt, st);
      if constexpr (S <= 2) {
        if (c.variant == FV_STRIPYX_2x8)
          return launch_strip_yx<T, S, 2, 8>(L, c.target, u, b, out, fc, part, stop, bt, st);
        if (c.variant == FV_STRIPYX_2x16)
          return launch_strip_yx<T, S, 2, 16>(L, c.target, u, b, out, fc, part, stop, bt, st);
      }
    }
  }
  int bx, by;
  variant_tile(c.variant, bx, by);
  const FusedGrid g = fused_grid(bx, by, L.nx, L.ny, L.nz, c.target);
  if constexpr (zq_instantiated<T, S>()) {
    if (c.variant == FV_ZQ_64x32) {
      hipLaunchKernelGGL((k_tau_zq<T, S, 64, 32, 512, 1, 0>), dim3(g.nblk, bt.nb), dim3(512), 0, st, L, u, b, out,
                         fc, g.zc, g.gx, g.gy, g.nblk, part, bt, stop);
      return;
    }
    if (c.variant == FV_ZQ_64x16) {
      hipLaunchKernelGGL((k_tau_zq<T, S, 64, 16, 256, 1, 0>), dim3(g.nblk, bt.nb), dim3(256), 0, st, L, u, b, out,
                         fc, g.zc, g.gx, g.gy, g.nblk, part, bt, stop);
      return;
    }
  }
  if (c.variant == FV_RING_64x4) {
    hipLaunchKernelGGL((k_fused_tau<T, S, 64, 4>), dim3(g.nblk, bt.nb), dim3(FNT), 0, st, L, u, b, out, fc, g.zc,
                       g.gx, g.gy, g.nblk, part, bt, stop);
    return;
  }
  hipLaunchKernelGGL((k_fused_tau<T, S, 64, 8>), dim3(g.nblk, bt.nb), dim3(FNT), 0, st, L, u, b, out, fc, g.zc,
                     g.gx, g.gy, g.nblk, part, bt, stop);
  }
}

template <typename T>
size_t fused_tau_blocks_as(const LevelView<T>& L, FusedChoice c, int s) {
  if (variant_is_2d(c.variant)) {
    const bool r8 = c.variant == FV_STRIP2D_8 && (sizeof(T) == 4 || s <= 2);
    return (size_t)strip_grid(s, r8 ? 8 : 4, 1, L.nx, 1, L.ny, c.target, true).nblk;
  }
  if (is_strip(c.variant) && L.faces != nullptr) c = FusedChoice{FV_RING_64x8, 1024};
  if (is_strip(c.variant)) {
    int R, WY;
    strip_shape(c.variant, R, WY);
    return (size_t)strip_grid(s, R, WY, L.nx, L.ny, L.nz, c.target).nblk;
  }
  int bx, by;
  variant_tile(c.variant, bx, by);
  return (size_t)fused_grid(bx, by, L.nx, L.ny, L.nz, c.target).nblk;
}

template <typename T>
int fused_chunk_blocks(const LevelView<T>& L, int variant, int s) {
  if (variant_is_2d(variant)) {
    const bool r8 = variant == FV_STRIP2D_8 && (sizeof(T) == 4 || s <= 2);
    return strip_grid(s, r8 ? 8 : 4, 1, L.nx, 1, L.ny, 1, true).per;
  }
  if (!is_strip(variant)) return 0;
  int R, WY;
  strip_shape(variant, R, WY);
  return strip_grid(s, R, WY, L.nx, L.ny, L.nz, 1).per;
}

template <typename T>
size_t fused_tau_blocks(const LevelView<T>& L, int s) {
  return fused_tau_blocks_as<T>(L, fused_choice<T>(L, s), s);
}

template <typename T>
bool launch_fused_tau_as(const LevelView<T>& L, FusedChoice c, const T* u, const T* b, T* out, int s,
                         const StageCoef* co, double* part, const int* stop, hipStream_t st, const Batch& bt) {
  if (!fused_tau_supported<T>(L, s) || !fused_variant_ok<T>(c.variant, s) || !variant_fits(L, c.variant) ||
      c.target < 1)
    return false;
  switch (s) {
    case 1: launch_fused_S<T, 1>(L, c, u, b, out, co, part, stop, bt, st); return true;
    case 2: launch_fused_S<T, 2>(L, c, u, b, out, co, part, stop, bt, st); return true;
    case 3: launch_fused_S<T, 3>(L, c, u, b, out, co, part, stop, bt, st); return true;
    case 4: launch_fused_S<T, 4>(L, c, u, b, out, co, part, stop, bt, st); return true;
    default: return false;
  }
}

template <typename T>
bool launch_fused_tau(const LevelView<T>& L, const T* u, const T* b, T* out, int s, const StageCoef* co,
                      double* part, const int* stop, hipStream_t st, const Batch& bt) {
  if (!fused_tau_supported<T>(L, s)) return false;
  return launch_fused_tau_as<T>(L, fused_choice<T>(L, s), u, b, out, s, co, part, stop, st, bt);
}

template <typename T, int S>
static bool launch_pro_S(const LevelView<T>& L, int variant, int target, const T* u, const T* e, const T* b, T* out,
                         const StageCoef* co, const int* stop, const Batch& bt, hipStream_t st) {
  if constexpr (S > fused_max_s<T>() || !strip_instantiated<T, S>()) {
    return false;
  } else {
    const FCoef<T, S> fc = make_fcoef<T, S>(co);
    switch (variant) {
      case FV_STRIP_8x4: launch_strip_pro<T, S, 8, 4, false>(L, target, u, e, b, out, fc, stop, bt, st); return true;
      case FV_STRIP_8x1: launch_strip_pro<T, S, 8, 1, false>(L, target, u, e, b, out, fc, stop, bt, st); return true;
      case FV_STRIP_4x4: launch_strip_pro<T, S, 4, 4, false>(L, target, u, e, b, out, fc, stop, bt, st); return true;
      case FV_STRIPYX_8x4: launch_strip_pro<T, S, 8, 4, true>(L, target, u, e, b, out, fc, stop, bt, st); return true;
      case FV_STRIPYX_4x8: launch_strip_pro<T, S, 4, 8, true>(L, target, u, e, b, out, fc, stop, bt, st); return true;
      case FV_STRIPYX_8x8: launch_strip_pro<T, S, 8, 8, true>(L, target, u, e, b, out, fc, stop, bt, st); return true;
      default: break;
    }
    if constexpr (S <= 2) {
      if (variant == FV_STRIPYX_2x8) {
        launch_strip_pro<T, S, 2, 8, true>(L, target, u, e, b, out, fc, stop, bt, st);
        return true;
      }
      if (variant == FV_STRIPYX_2x16) {
        launch_strip_pro<T, S, 2, 16, true>(L, target, u, e, b, out, fc, stop, bt, st);
        return true;
      }
    }
    return false;
  }
}

template <typename T>
bool launch_fused_tau_pro(const LevelView<T>& L, const T* u, const T* e, const T* b, T* out, int s,
                          const StageCoef* co, const int* stop, hipStream_t st, const Batch& bt) {
  if (u == nullptr || e == nullptr || L.faces != nullptr || level_is_2d(L) || !fused_tau_supported<T>(L, s))
    return false;
  if ((L.nx | L.ny | L.nz) & 1) return false;
  FusedChoice c = fused_choice<T>(L, s);
  // The five-row strip (odd R) has no fused form: its levels (128^3 and
  // below in the tuned table) take the fused four-row strips, measured faster
  // than the separate prolongation in both precisions once the grid is sized
  // from occupancy (float64 256^3 solve 6.07 ms against 6.15; the stacked
  // two-row strips gave no gain there).  The float64 eight-row forms run out
  // of registers with the fusion (one wavefront per SIMD): those levels take
  // the stacked two-row strips, the leanest fused form.
  // A level that takes another form than its tuned variant sizes the grid
  // from that form's occupancy (target 0), not from the tuned target.
  if (c.variant == FV_STRIP_5x1) c = FusedChoice{FV_STRIP_4x4, 0};
  const bool dbl8 = sizeof(T) == 8 && (c.variant == FV_STRIP_8x4 || c.variant == FV_STRIP_8x1 ||
                                       c.variant == FV_STRIPYX_8x4 || c.variant == FV_STRIPYX_8x8);
  if (dbl8) c = FusedChoice{s <= 2 ? FV_STRIPYX_2x8 : FV_STRIP_4x4, 0};
  if (!is_strip(c.variant) || !fused_variant_ok<T>(c.variant, s) || c.target < 0) return false;
  switch (s) {
    case 1: return launch_pro_S<T, 1>(L, c.variant, c.target, u, e, b, out, co, stop, bt, st);
    case 2: return launch_pro_S<T, 2>(L, c.variant, c.target, u, e, b, out, co, stop, bt, st);
    case 3: return launch_pro_S<T, 3>(L, c.variant, c.target, u, e, b, out, co, stop, bt, st);
    default: return false;
  }
}

template <typename T, int S>
static int launch_rs_S(const LevelView<T>& L, int variant, int target, const T* u, const T* b, T* out, T* bc,
                       const StageCoef* co, double* part, const int* stop, const Batch& bt, hipStream_t st) {
  if constexpr (S < 2 || S > 3) {
    return 0;  // the form needs s >= 2 (b of a halo row in registers); none is built beyond 3
  } else {
    const FCoef<T, S> fc = make_fcoef<T, S>(co);
    if constexpr (S <= 2) {
      if (variant == FV_STRIPYX_2x8)
        return launch_strip_rs<T, S, 2, 8, true>(L, target, u, b, out, bc, fc, part, stop, bt, st);
    }
    if constexpr (sizeof(T) == 4) {
      if (variant == FV_STRIP_4x4)
        return launch_strip_rs<T, S, 4, 4, false>(L, target, u, b, out, bc, fc, part, stop, bt, st);
      if constexpr (S <= 2) {
        if (variant == FV_STRIPYX_8x4)
          return launch_strip_rs<T, S, 8, 4, true>(L, target, u, b, out, bc, fc, part, stop, bt, st);
      }
    }
    return 0;
  }
}

template <typename T>
int launch_fused_tau_rs(const LevelView<T>& L, const T* u, const T* b, T* out, T* bc, int s, const StageCoef* co,
                        double* part, const int* stop, hipStream_t st, const Batch& bt) {
  if (u == nullptr || bc == nullptr || part == nullptr || L.faces != nullptr || level_is_2d(L) ||
      !fused_tau_supported<T>(L, s))
    return 0;
  if ((L.nx | L.ny | L.nz) & 1) return 0;
  FusedChoice c = fused_choice<T>(L, s);
  if (!is_strip(c.variant) || c.target < 1) return 0;
  // Forms built (s >= 2): the stacked two-row strips (eight wavefronts that
  // share their y halos; s = 2), every float64 level; in float32 also the
  // stacked eight-row strips (four wavefronts; s = 2), which levels of 192^3
  // and more and levels tuned for them take, and the four-row strips of four
  // wavefronts (s = 2, 3) for the other levels not tuned for the two-row
  // stacked strips.  Measured on gfx950 at 256^3 (fused pass against
  // tau-step + separate residual pass): float64 134 us against 92 + 65 us;
  // float32 77 (stacked two-row) or 83 (four-row) against 43 + 40 us; at
  // 128^3, 26 against 16 + 15 us (float64).  Float32 mixed solves with the
  // stacked eight-row form instead of the two-row one: 256^3 5.24 against
  // 5.35 ms, 512^3 32.6 against 33.0 ms.  (A float64 four-row form needs 165
  // VGPRs, three wavefronts per SIMD.)
  const bool big = (size_t)L.nx * L.ny * L.nz >= ((size_t)192 * 192 * 192);
  if (sizeof(T) == 8) c.variant = FV_STRIPYX_2x8;
  else if (c.variant != FV_STRIPYX_2x8)
    c.variant = (big || c.variant == FV_STRIPYX_8x4) ? FV_STRIPYX_8x4 : FV_STRIP_4x4;
  if ((c.variant == FV_STRIPYX_2x8 || c.variant == FV_STRIPYX_8x4) && s > 2) c.variant = FV_STRIP_4x4;
  switch (s) {
    case 1: return launch_rs_S<T, 1>(L, c.variant, c.target, u, b, out, bc, co, part, stop, bt, st);
    case 2: return launch_rs_S<T, 2>(L, c.variant, c.target, u, b, out, bc, co, part, stop, bt, st);
    case 3: return launch_rs_S<T, 3>(L, c.variant, c.target, u, b, out, bc, co, part, stop, bt, st);
    default: return 0;
  }
}

template <typename T>
int tau_chunk_max(const LevelView<T>& L) {
  if (level_is_2d(L) || L.faces != nullptr || L.nx < 16 || L.ny < 8 || L.nz < 8) return 0;
  return sizeof(T) == 8 ? 2 : 3;
}

template <typename T>
void launch_tau_chunk(const LevelView<T>& L, const T* u, const T* v, const T* b, T* out, T* out2, int S,
                      const StageCoef* co, hipStream_t st) {
  if (S < 1 || S > tau_chunk_max<T>(L)) fail(RKL_EINVAL, "stage chunk of unsupported length");
  const int target = 1024;
  switch (S) {
    case 1: return launch_strip_ch<T, 1, 4, 4>(L, target, u, v, b, out, out2, make_fcoef<T, 1>(co), single_batch(), st);
    case 2: return launch_strip_ch<T, 2, 4, 4>(L, target, u, v, b, out, out2, make_fcoef<T, 2>(co), single_batch(), st);
    default:
      if constexpr (sizeof(T) == 4)
        return launch_strip_ch<T, 3, 4, 4>(L, target, u, v, b, out, out2, make_fcoef<T, 3>(co), single_batch(), st);
  }
}

template <typename T>
bool launch_gsrb_fused(const LevelView<T>& L, const T* u, const T* b, T* out, double omega, double* part,
                       const int* stop, hipStream_t st, const Batch& bt) {
  if (!fused_tau_supported<T>(L, 2) || L.faces != nullptr) return false;
  const double d = 2.0 * ((double)L.ihx2 + (double)L.ihy2 + (double)L.ihz2);
  const FusedChoice c = fused_choice<T>(L, 2);
  // the strip shape tuned for RKL s = 2 suits the two-stage pass; other
  // families (and the eight-row one-wavefront strips) use 4-row strips.  The
  // five-row strips keep their shape: on the 128^3 App. B problem an SOR
  // iteration (residual checks included) took 27.6 us in them against 37 us
  // in the 4-row strips.
  if (c.variant == FV_STRIP2D_4)
    launch_strip_gsrb<T, 4, 1, true>(L, c.target, u, b, out, omega / d, part, stop, bt, st);
  else if (c.variant == FV_STRIP2D_8)
    launch_strip_gsrb<T, 8, 1, true>(L, c.target, u, b, out, omega / d, part, stop, bt, st);
  else if (c.variant == FV_STRIP_8x4)
    launch_strip_gsrb<T, 8, 4, false>(L, c.target, u, b, out, omega / d, part, stop, bt, st);
  else if (c.variant == FV_STRIP_5x1)
    launch_strip_gsrb<T, 5, 1, false>(L, c.target, u, b, out, omega / d, part, stop, bt, st);
  else
    launch_strip_gsrb<T, 4, 4, false>(L, is_strip(c.variant) ? c.target : 1024, u, b, out, omega / d, part, stop,
                                      bt, st);
  return true;
}

template <typename T>
size_t gsrb_blocks(const LevelView<T>& L) {
  const FusedChoice c = fused_choice<T>(L, 2);
  if (variant_is_2d(c.variant))
    return (size_t)strip_grid(2, c.variant == FV_STRIP2D_4 ? 4 : 8, 1, L.nx, 1, L.ny, c.target, true).nblk;
  if (c.variant == FV_STRIP_8x4) return (size_t)strip_grid(2, 8, 4, L.nx, L.ny, L.nz, c.target).nblk;
  if (c.variant == FV_STRIP_5x1) return (size_t)strip_grid(2, 5, 1, L.nx, L.ny, L.nz, c.target).nblk;
  return (size_t)strip_grid(2, 4, 4, L.nx, L.ny, L.nz, is_strip(c.variant) ? c.target : 1024).nblk;
}

const char* fused_variant_name(int variant) {
  switch (variant) {
    case FV_RING_64x8: return "ring64x8";
    case FV_RING_64x4: return "ring64x4";
    case FV_ZQ_64x32: return "zq64x32";
    case FV_ZQ_64x16: return "zq64x16";
    case FV_STRIP_8x4: return "strip8x4";
    case FV_STRIP_8x1: return "strip8x1";
    case FV_STRIP_4x4: return "strip4x4";
    case FV_STRIP2D_8: return "strip2d8";
    case FV_STRIP2D_4: return "strip2d4";
    case FV_STRIP_5x1: return "strip5x1";
    case FV_STRIPYX_8x4: return "stripyx8x4";
    case FV_STRIPYX_4x8: return "stripyx4x8";
    case FV_STRIPYX_8x8: return "stripyx8x8";
    case FV_STRIPYX_2x8: return "stripyx2x8";
    case FV_STRIPYX_2x16: return "stripyx2x16";
    default: return "heuristic";
  }
}

#define RKL_FUSED_INST(T)                                                                                         \
  template bool fused_tau_supported<T>(const LevelView<T>&, int);                                                 \
  template bool fused_variant_ok<T>(int, int);                                                                    \
  template FusedChoice fused_choice<T>(const LevelView<T>&, int);                                                 \
  template size_t fused_tau_blocks<T>(const LevelView<T>&, int);                                                  \
  template size_t fused_tau_blocks_as<T>(const LevelView<T>&, FusedChoice, int);                                  \
  template int fused_chunk_blocks<T>(const LevelView<T>&, int, int);                                              \
  template bool launch_fused_tau<T>(const LevelView<T>&, const T*, const T*, T*, int, const StageCoef*, double*,  \
                                    const int*, hipStream_t, const Batch&);                                       \
  template bool launch_fused_tau_as<T>(const LevelView<T>&, FusedChoice, const T*, const T*, T*, int,             \
                                       const StageCoef*, double*, const int*, hipStream_t, const Batch&);       \
  template int tau_chunk_max<T>(const LevelView<T>&);                                                             \
  template void launch_tau_chunk<T>(const LevelView<T>&, const T*, const T*, const T*, T*, T*, int, const StageCoef*, \
                                    hipStream_t);                                                                 \
  template bool launch_fused_tau_pro<T>(const LevelView<T>&, const T*, const T*, const T*, T*, int,               \
                                        const StageCoef*, const int*, hipStream_t, const Batch&);                 \
  template int launch_fused_tau_rs<T>(const LevelView<T>&, const T*, const T*, T*, T*, int, const StageCoef*,     \
                                      double*, const int*, hipStream_t, const Batch&);
RKL_FUSED_INST(double)
RKL_FUSED_INST(float)
template bool launch_gsrb_fused<double>(const LevelView<double>&, const double*, const double*, double*, double,
                                        double*, const int*, hipStream_t, const Batch&);
template bool launch_gsrb_fused<float>(const LevelView<float>&, const float*, const float*, float*, double, double*,
                                       const int*, hipStream_t, const Batch&);
template size_t gsrb_blocks<double>(const LevelView<double>&);
template size_t gsrb_blocks<float>(const LevelView<float>&);
#undef RKL_FUSED_INST

}  // namespace rkl
