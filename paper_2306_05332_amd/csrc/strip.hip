// Fused s-stage RKL tau-step (App. A eq. RKL_intermediate_source), strip
// form: every wavefront works on its own and keeps its whole working set in
// registers.
//
// A wavefront's 64 lanes hold 64 consecutive x columns; the middle 64 - 2S
// are its output columns and S on each side are halo (stage j is valid on
// lanes j .. 63 - j, so after S stages the output lanes are exact).  Each
// lane owns a strip of R output rows in y plus S halo rows on either side,
// and the wavefront marches up through a chunk of z planes.  The x
// neighbours of a value come from the adjacent lanes by wavefront DPP shifts,
// the y neighbours are the lane's own adjacent rows, and the z neighbours are
// the lane's queue of the last three planes; so the inner loop has no LDS
// traffic and no barrier.  Stage 1 of plane z runs in the iteration that
// receives u(z + 1); stage j of plane z - j + 1 follows in the same
// iteration.  The next planes of u and b are loaded at the top of an
// iteration and consumed at its end.  u and b are read once (halo rows and
// planes are read again by the neighbouring strip or chunk, mostly from
// cache) and Y_S is written once: 3 words of HBM traffic per cell.
//
// Boundaries (Sec. 2.3): periodic boxes wrap rows, planes and columns
// (a wavefront may hold several periods of a short axis); Dirichlet stencils
// that leave the box take the homogeneous ghost -c of the operand being
// differentiated (finest-level face data is folded into the right-hand side
// before any relaxation, so no face array is read here).
// Optionally the kernel returns float64 partial sums of (M u - b)^2 over its
// output cells (the residual of the tau-step's input).
//
// x tiles hold 64 - 2S output columns, so nx is rarely a multiple of them;
// the last tile of a row of strips would then run mostly idle lanes (at
// nx = 256, S = 2: 16 of its 60 output lanes).  One-wavefront 3-D variants
// instead give that remainder of several interior strips to one wavefront,
// each strip in its own segment of rem + 2S lanes (StripMap).  A segment's
// rows are the base strip's shifted by a whole number of strips, which the
// lane folds into its column byte offset; the wavefront shifts then carry
// halo garbage across a segment boundary only into halo lanes.
//
// With GS = true the same two-stage pass is one red-black Gauss-Seidel
// (omega-SOR) iteration (Sec. 2.2.4): stage 1 updates the red cells
// ((i + j + k) even) from the old values, stage 2 the black cells from the
// new red ones, each by u += (omega / D_cell) (M u - b), i.e. the stage
// recurrence with mu = 1, nu = 0 applied to one colour.  D_cell is the
// operator's own diagonal: 2 sum h^-2, plus h_d^-2 for each Dirichlet face
// the cell touches (the ghost's -u term), so that omega = 1 solves each
// cell's row exactly.
//
// FLAT = true is the two-dimensional form (eq. discrete_laplace_2D).  The
// launcher hands the kernel a transposed view: the 2-D y axis becomes the
// marching axis (nz' = ny, ihz2' = ihy2) and the view has one row (ny' = 1,
// ihy2' = 0).  A lane's R "rows" are then R separate 64-column x segments of
// the same grid row, side by side (segment i starts OX columns after
// segment i - 1), so a wavefront still loads R values of u and of b per
// plane; there are no y-halo rows, and each segment keeps its own column,
// boundary flags and colour parity.
#include "kernels.h"

namespace rkl {

template <typename T, int S, int R, int WY, bool PER, bool UZ, bool GS, bool FLAT, bool SHY, bool NT>
__device__ __forceinline__ void tau_strip_body(LevelView<T> L, const T* __restrict__ u, const T* __restrict__ b,
                                               T* __restrict__ out, FCoef<T, S> co, int zc, int gx_tiles,
                                               int gy_tiles, int nblk, StripMap sm, double* __restrict__ part,
                                               Batch bt, const int* __restrict__ stop) {
  static_assert(!SHY || (WY > 1 && !FLAT && R >= S), "shared y halos need stacked 3-D strips of >= S rows");
  {
    const long long mb = blockIdx.y;
    if (!UZ) u += mb * bt.s0;
    b += mb * bt.s0;
    out += mb * bt.s0;
    if (part != nullptr) part += mb * bt.part_stride;
    if (stop != nullptr) stop += mb * bt.stop_stride;
  }
  constexpr int HY = FLAT ? 0 : S;  // halo rows on either side of the R output rows
  constexpr int NU = R + 2 * HY;    // rows held per lane
  constexpr int OX = 64 - 2 * S;    // output columns per wavefront (per segment when FLAT)
  constexpr int NY = S > 1 ? S - 1 : 1;
  constexpr int A1 = FLAT ? 0 : 1;  // first row of stage 1 (stage j starts at row A1 * j)
  __shared__ double red[WY];
  // SHY: the wavefronts of a workgroup are stacked in y, and each takes the
  // halo rows it shares with its neighbours from their registers through LDS
  // (double-buffered): [buffer][wavefront][side][row][lane], side 0 = the
  // wavefront's lowest S rows of u (and S - 1 of b) for the one below's upper
  // halo, side 1 = its highest rows for the one above's lower halo
  constexpr int XU = S, XB = S > 1 ? S - 1 : 1;
  __shared__ T xch[SHY ? 2 : 1][SHY ? WY : 1][2][SHY ? XU + XB : 1][64];
  if (stop != nullptr && *stop) return;

  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  const long long sxy = (long long)nx * ny;
  int bid = blockIdx.x;
  if ((nblk & 7) == 0) bid = (bid & 7) * (nblk >> 3) + (bid >> 3);  // neighbouring tiles on one XCD
  int tx, ty, tz;
  int xl = lane, xw = 64;  // lane within its x segment, segment width (halo lanes included)
  int yshift = 0;          // rows from the wavefront's base strip to this lane's strip
  if (!FLAT && WY == 1 && sm.pk > 0) {
    tz = bid / sm.per;
    const int r = bid - tz * sm.per, nfull = sm.txf * gy_tiles;
    if (r < nfull) {
      tx = r % sm.txf;
      ty = r / sm.txf;
    } else {
      tx = sm.txf;
      const int k = r - nfull;
      if (k < sm.npk) {  // packed remainder: pk interior strips side by side
        ty = sm.fi + k * sm.pk;
        xw = nx - sm.txf * OX + 2 * S;
        const int q = min(lane / xw, sm.pk - 1);  // lanes past the last segment: idle (never own)
        xl = lane - q * xw;
        yshift = q * R;
      } else {
        const int m = k - sm.npk;
        ty = m < sm.fi ? m : m + sm.npk * sm.pk;
      }
    }
  } else {
    tx = bid % gx_tiles;
    ty = (bid / gx_tiles) % gy_tiles;
    tz = bid / (gx_tiles * gy_tiles);
  }
  const int gxu = tx * OX - S + xl;          // column of this lane (unwrapped; 3-D form)
  const int y0 = FLAT ? 0 : (ty * WY + w) * R - S;  // row of strip index 0 (unwrapped, wave-uniform)
  const int z0 = tz * zc, z1 = min(z0 + zc, nz);
  const bool xin = gxu >= 0 && gxu < nx;
  const int gx = PER ? ((gxu % nx) + nx) % nx : min(max(gxu, 0), nx - 1);
  // byte offset of this lane's column (and, in a packed wavefront, of its strip's rows)
  const unsigned xb = ((unsigned)gx + (unsigned)yshift * (unsigned)nx) * (unsigned)sizeof(T);
  const bool xown = xl >= S && xl < xw - S && xin;
  const bool xlo = !PER && gxu == 0, xhi = !PER && gxu == nx - 1;
  // FLAT: per-segment column byte offsets and bit masks (bit i: segment i)
  unsigned sxb[FLAT ? R : 1];
  unsigned sown = 0, slo = 0, shi = 0, sodd = 0;
  if constexpr (FLAT) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int cu = ((tx * WY + w) * R + i) * OX - S + lane;
      const int c = PER ? ((cu % nx) + nx) % nx : min(max(cu, 0), nx - 1);
      sxb[i] = (unsigned)c * (unsigned)sizeof(T);
      if (lane >= S && lane < 64 - S && cu >= 0 && cu < nx) sown |= 1u << i;
      if (!PER && cu == 0) slo |= 1u << i;
      if (!PER && cu == nx - 1) shi |= 1u << i;
      if (c & 1) sodd |= 1u << i;
    }
  }
  auto colb = [&](int i) -> unsigned { if constexpr (FLAT) return sxb[i]; else return xb; };
  auto own = [&](int i) -> bool { if constexpr (FLAT) return (sown >> i) & 1u; else return xown; };
  auto atlo = [&](int i) -> bool { if constexpr (FLAT) return (slo >> i) & 1u; else return xlo; };
  auto athi = [&](int i) -> bool { if constexpr (FLAT) return (shi >> i) & 1u; else return xhi; };
  // colour parity of column and strip shift (the rows' own parity is in rodd)
  auto xpar = [&](int i) -> int { if constexpr (FLAT) return (sodd >> i) & 1u; else return (gx + yshift) & 1; };

  long long yoff[NU];    // row offsets in elements (wrapped or clamped), wave-uniform
  unsigned rin = 0;      // bit i: row i lies in the box
  unsigned rodd = 0;     // bit i: row i has an odd index (GS colouring)
#pragma unroll
  for (int i = 0; i < NU; ++i) {
    const int gyu = FLAT ? 0 : y0 + i;  // FLAT: every segment lies in the view's single row
    const bool in = gyu >= 0 && gyu < ny;
    const int gy = PER ? ((gyu % ny) + ny) % ny : min(max(gyu, 0), ny - 1);
    yoff[i] = (long long)gy * nx;
    if (in) rin |= 1u << i;
    if (gy & 1) rodd |= 1u << i;
  }
  // parity of plane p's index (wrapped for periodic boxes; |p| stays within a period of the box)
  auto zodd = [&](int p) -> int { return (PER ? (p < 0 ? p + nz : (p >= nz ? p - nz : p)) : p) & 1; };
  // plane p -> element offset of its (wrapped or clamped) plane; advanced by one
  // plane per iteration without divisions
  auto plane0 = [&](int p) -> long long {
    const int q = PER ? ((p % nz) + nz) % nz : min(max(p, 0), nz - 1);
    return (long long)q * sxy;
  };
  const long long nzs = (long long)nz * sxy;
  auto next_plane = [&](long long off, int p_next) -> long long {
    // off: offset of plane p_next - 1
    if (PER) return off + sxy == nzs ? 0 : off + sxy;
    return (p_next <= 0 || p_next >= nz) ? off : off + sxy;
  };
  auto row = [&](const T* __restrict__ a, long long poff, int i) -> T {
    const char* base = (const char*)(a + poff + yoff[i]);
    return *(const T*)(base + colb(i));
  };
  auto pin = [&](int p) { return PER || (p >= 0 && p < nz); };
  // rows read from memory: every row, or with SHY the wavefront's own R rows
  // plus the outer halo of the workgroup's lowest / highest wavefront
  auto gl = [&](int i) -> bool {
    if constexpr (!SHY) return true;
    else return (i >= S && i < S + R) || (i < S && w == 0) || (i >= S + R && w == WY - 1);
  };
  int xbuf = 0;
  // SHY: halo rows of Ux (u) and Bx (b, when DOB) from the neighbouring
  // wavefronts' registers; one barrier per exchange (the two buffers
  // alternate, so the next exchange cannot overwrite rows still being read)
  auto exchange = [&](T(&Ux)[NU], T(&Bx)[NU], bool dou, bool dob) {
    if constexpr (SHY) {
#pragma unroll
      for (int r = 0; r < S; ++r) {
        if (dou) {
          xch[xbuf][w][0][r][lane] = Ux[S + r];
          xch[xbuf][w][1][r][lane] = Ux[R + r];
        }
      }
#pragma unroll
      for (int r = 0; r < S - 1; ++r) {
        if (dob) {
          xch[xbuf][w][0][XU + r][lane] = Bx[S + r];
          xch[xbuf][w][1][XU + r][lane] = Bx[R + 1 + r];
        }
      }
      __syncthreads();
      if (w > 0) {
#pragma unroll
        for (int r = 0; r < S; ++r)
          if (dou) Ux[r] = xch[xbuf][w - 1][1][r][lane];
#pragma unroll
        for (int r = 0; r < S - 1; ++r)
          if (dob) Bx[1 + r] = xch[xbuf][w - 1][1][XU + r][lane];
      }
      if (w < WY - 1) {
#pragma unroll
        for (int r = 0; r < S; ++r)
          if (dou) Ux[R + S + r] = xch[xbuf][w + 1][0][r][lane];
#pragma unroll
        for (int r = 0; r < S - 1; ++r)
          if (dob) Bx[R + S + r] = xch[xbuf][w + 1][0][XU + r][lane];
      }
      xbuf ^= 1;
    }
  };
  // GS coefficient of row i, plane p: c * D / D_cell (Dirichlet faces add h_d^-2)
  const T dgs = (T)2 * (L.ihx2 + L.ihy2 + L.ihz2);
  auto gscoef = [&](T c, int i, int p) -> T {
    if (PER) return c;
    const int gyu = y0 + i;
    T extra = (T)0;
    if (atlo(i)) extra += L.ihx2;
    if (athi(i)) extra += L.ihx2;
    if (!FLAT && gyu == 0) extra += L.ihy2;
    if (!FLAT && gyu == ny - 1) extra += L.ihy2;
    if (p == 0) extra += L.ihz2;
    if (p == nz - 1) extra += L.ihz2;
    return extra == (T)0 ? c : c * dgs / (dgs + extra);
  };

  // 7-point M applied to the centre row i of plane p: X = centre plane,
  // Zm / Zp = planes below and above
  auto lap = [&](const T(&Zm)[NU], const T(&X)[NU], const T(&Zp)[NU], int i, int p) -> T {
    const T c = X[i];
    T xm = wshift<DPP_WAVE_SHR1>(c), xp = wshift<DPP_WAVE_SHL1>(c);
    T zm = Zm[i], zp = Zp[i];
    if constexpr (FLAT) {  // 5-point: x within the segment, 2-D y along the march
      if (!PER) {
        if (atlo(i)) xm = -c;
        if (athi(i)) xp = -c;
        if (p == 0) zm = -c;
        if (p == nz - 1) zp = -c;
      }
      return ((xm + xp) - (T)2 * c) * L.ihx2 + ((zm + zp) - (T)2 * c) * L.ihz2;
    } else {
      T ym = X[i - 1], yp = X[i + 1];
      if (!PER) {
        const int gyu = y0 + i;
        if (xlo) xm = -c;
        if (xhi) xp = -c;
        if (gyu == 0) ym = -c;
        if (gyu == ny - 1) yp = -c;
        if (p == 0) zm = -c;
        if (p == nz - 1) zp = -c;
      }
      return ((xm + xp) - (T)2 * c) * L.ihx2 + ((ym + yp) - (T)2 * c) * L.ihy2 +
             ((zm + zp) - (T)2 * c) * L.ihz2;
    }
  };

  T U0[NU], U1[NU], U2[NU], UN[NU];  // u at planes zl-1, zl, zl+1; zl+2 in flight
  T Yq[NY][3][NU];                   // Y_j at planes zl-j-1, zl-j, zl-j+1 (after stage j of iteration zl)
  T Bq[S][NU], BN[NU];               // b at planes zl, zl-1, ..; zl+1 in flight
  const int zs = z0 - (S - 1), ze = z1 + S - 2;  // iterations: stage 1 of plane zl, stage j of zl - j + 1
  long long ou = plane0(zs - 1);   // plane offset of the last u plane loaded
  long long ob = plane0(zs);       // plane offset of the last b plane loaded
  long long oo = plane0(zs - S + 1);  // plane offset of the stage-S output plane of iteration zs
#pragma unroll
  for (int i = 0; i < NU; ++i) {
    for (int j = 0; j < NY; ++j) Yq[j][0][i] = Yq[j][1][i] = Yq[j][2][i] = (T)0;
    for (int j = 0; j < S; ++j) Bq[j][i] = (T)0;
  }
  // rows outside a Dirichlet box and planes outside it read as 0
#pragma unroll
  for (int i = 0; i < NU; ++i)
    if (gl(i)) U0[i] = (UZ || !pin(zs - 1) || !(PER || ((rin >> i) & 1u))) ? (T)0 : row(u, ou, i);
  ou = next_plane(ou, zs);
#pragma unroll
  for (int i = 0; i < NU; ++i)
    if (gl(i)) U1[i] = (UZ || !pin(zs) || !(PER || ((rin >> i) & 1u))) ? (T)0 : row(u, ou, i);
  ou = next_plane(ou, zs + 1);
#pragma unroll
  for (int i = 0; i < NU; ++i)
    if (gl(i)) U2[i] = (UZ || !pin(zs + 1) || !(PER || ((rin >> i) & 1u))) ? (T)0 : row(u, ou, i);
#pragma unroll
  for (int i = A1; i < NU - A1; ++i)
    if (gl(i)) Bq[0][i] = (!pin(zs) || !(PER || ((rin >> i) & 1u))) ? (T)0 : row(b, ob, i);
  exchange(U0, Bq[0], !UZ, false);
  exchange(U1, Bq[0], !UZ, false);
  exchange(U2, Bq[0], !UZ, true);
  double r2 = 0.0;
  T YS[NU];  // Y_S of the iteration's output plane, stored after the queues advance

  for (int zl = zs; zl <= ze; ++zl) {
    // next planes: loads issued now, consumed at the end of the iteration
    // (the plane index is wrapped or clamped into the box); the last
    // iteration has no next plane to use and re-reads the planes just loaded
    // (cache hits) rather than fetching one more from memory
    const bool more = zl < ze;
    if (more) {
      ou = next_plane(ou, zl + 2);
      ob = next_plane(ob, zl + 1);
    }
    if (!UZ) {
#pragma unroll
      for (int i = 0; i < NU; ++i)
        if (gl(i)) UN[i] = row(u, ou, i);
    }
#pragma unroll
    for (int i = A1; i < NU - A1; ++i)
      if (gl(i)) BN[i] = row(b, ob, i);
    // stage 1 at plane zl, rows A1 .. NU-1-A1
    {
      const int p = zl;
      const bool on = pin(p) && p >= z0 - (S - 1) && p <= z1 - 1 + (S - 1);
      const bool pown = p >= z0 && p < z1;
      if (on) {
#pragma unroll
        for (int i = A1; i < NU - A1; ++i) {
          const T res = lap(U0, U1, U2, i, p) - Bq[0][i];
          T y;
          if (GS) {
            y = U1[i] + gscoef(co.c[0], i, p) * res;
            if ((xpar(i) ^ ((rodd >> i) & 1) ^ zodd(p)) != 0) y = U1[i];  // black cell: unchanged
          } else {
            y = U1[i] + co.c[0] * res;
          }
          if (part != nullptr && pown && i >= HY && i < HY + R && own(i) && ((rin >> i) & 1u))
            r2 += (double)res * (double)res;
          if constexpr (S == 1) YS[i] = y;
          else Yq[0][2][i] = y;
        }
      }
    }
    // stages 2 .. S at planes zl - j + 1, rows A1 j .. NU-1-A1 j
#pragma unroll
    for (int j = 2; j <= S; ++j) {
      const int p = zl - j + 1;
      const bool on = pin(p) && p >= z0 - (S - j) && p <= z1 - 1 + (S - j);
      if (on) {
#pragma unroll
        for (int i = A1 * j; i < NU - A1 * j; ++i) {
          const T(&Xm)[NU] = Yq[j - 2][0];
          const T(&Xc)[NU] = Yq[j - 2][1];
          const T(&Xp)[NU] = Yq[j - 2][2];
          const T y2 = (j == 2) ? U0[i] : Yq[j >= 3 ? j - 3 : 0][0][i];
          const T res = lap(Xm, Xc, Xp, i, p) - Bq[j - 1][i];
          T y;
          if (GS) {
            y = Xc[i] + gscoef(co.c[j - 1], i, p) * res;
            if ((xpar(i) ^ ((rodd >> i) & 1) ^ zodd(p)) == 0) y = Xc[i];  // red cell: unchanged
          } else {
            y = co.mu[j - 1] * Xc[i] + co.nu[j - 1] * y2 + co.c[j - 1] * res;
          }
          if (j == S) YS[i] = y;
          else Yq[j - 1][2][i] = y;
        }
      }
    }
    // advance the queues; Dirichlet planes outside the box and rows outside it read as 0
    const bool un_ok = pin(zl + 2), bn_ok = pin(zl + 1);
#pragma unroll
    for (int i = 0; i < NU; ++i) {
      const bool rok = PER || ((rin >> i) & 1u);
      U0[i] = U1[i];
      U1[i] = U2[i];
      U2[i] = (UZ || !un_ok || !rok) ? (T)0 : UN[i];
#pragma unroll
      for (int j = NY - 1; j >= 0; --j) {
        Yq[j][0][i] = Yq[j][1][i];
        Yq[j][1][i] = Yq[j][2][i];
      }
#pragma unroll
      for (int j = S - 1; j > 0; --j) Bq[j][i] = Bq[j - 1][i];
      Bq[0][i] = (!bn_ok || !rok) ? (T)0 : BN[i];
    }
    if (more) exchange(U2, Bq[0], !UZ, true);
    // stores after the wait for the loads above, so that the next
    // iteration's wait does not also wait for these writes; NT: with
    // non-temporal hints
    __builtin_amdgcn_sched_barrier(0);
    {
      const int p = zl - S + 1;
      if (p >= z0 && p < z1) {
#pragma unroll
        for (int i = HY; i < HY + R; ++i)
          if (own(i) && ((rin >> i) & 1u)) {
            T* dst = (T*)((char*)(out + oo + yoff[i]) + colb(i));
            if constexpr (NT) __builtin_nontemporal_store(YS[i], dst);
            else *dst = YS[i];
          }
      }
    }
    oo = next_plane(oo, zl - S + 2);
  }
  if (part != nullptr) {
    const double t = wave_sum_dpp(r2);
    if (lane == 0) red[w] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < WY; ++q) s += red[q];
      part[blockIdx.x] = s;
    }
  }
}

template <typename T, int S, int R, int WY, bool PER, bool UZ, bool GS, bool FLAT, bool NT>
__global__ __launch_bounds__(64 * WY) void k_tau_strip(LevelView<T> L, const T* __restrict__ u,
                                                       const T* __restrict__ b, T* __restrict__ out,
                                                       FCoef<T, S> co, int zc, int gx_tiles, int gy_tiles,
                                                       int nblk, StripMap sm, double* __restrict__ part, Batch bt,
                                                       const int* __restrict__ stop) {
  tau_strip_body<T, S, R, WY, PER, UZ, GS, FLAT, false, NT>(L, u, b, out, co, zc, gx_tiles, gy_tiles, nblk, sm,
                                                             part, bt, stop);
}

// the same with the y halo rows shared between the stacked wavefronts
template <typename T, int S, int R, int WY, bool PER, bool UZ, bool GS, bool NT>
__global__ __launch_bounds__(64 * WY) void k_tau_strip_yx(LevelView<T> L, const T* __restrict__ u,
                                                          const T* __restrict__ b, T* __restrict__ out,
                                                          FCoef<T, S> co, int zc, int gx_tiles, int gy_tiles,
                                                          int nblk, StripMap sm, double* __restrict__ part, Batch bt,
                                                          const int* __restrict__ stop) {
  tau_strip_body<T, S, R, WY, PER, UZ, GS, false, true, NT>(L, u, b, out, co, zc, gx_tiles, gy_tiles, nblk, sm,
                                                             part, bt, stop);
}

// flat: (nx, ny, nz) is the transposed view of a 2-D level (ny = 1, nz = the
// 2-D row count); a workgroup then spans WY * R segments of ox columns in x
StripGrid strip_grid(int s, int R, int WY, int nx, int ny, int nz, int target, bool flat) {
  StripGrid g;
  g.ox = 64 - 2 * s;
  g.map = StripMap{0, 0, 0, 0, 0};
  if (flat) {
    g.gx = (nx + g.ox * R * WY - 1) / (g.ox * R * WY);
    g.gy = 1;
  } else {
    g.gx = (nx + g.ox - 1) / g.ox;
    g.gy = (ny + R * WY - 1) / (R * WY);
  }
  int per = g.gx * g.gy;  // workgroups per z chunk
  if (!flat && WY == 1) {
    const int txf = nx / g.ox, rem = nx - txf * g.ox;
    const int pk = rem > 0 ? 64 / (rem + 2 * s) : 0;
    // interior strips: rows ty R - s .. ty R + R + s - 1 all inside 0 .. ny - 1
    const int fi = (s + R - 1) / R;
    const int li = ny - R - s >= 0 ? (ny - R - s) / R : -1;
    const int npk = (pk >= 2 && li >= fi) ? (li - fi + 1) / pk : 0;
    if (npk > 0) {
      g.map = StripMap{txf, pk, npk, fi, txf * g.gy + npk + (g.gy - npk * pk)};
      per = g.map.per;
    }
  }
  const int chunks = std::max(1, (target + per - 1) / per);
  // chunks down to one plane: on small (cache-resident, latency-bound) levels
  // a shorter serial march beats the re-read of the chunk's boundary planes
  g.zc = std::max(1, std::min(64, (nz + chunks - 1) / chunks));
  g.gz = (nz + g.zc - 1) / g.zc;
  g.per = per;
  g.nblk = per * g.gz;
  return g;
}

// Non-temporal output stores (float64 sweeps) pay off when a sweep's three
// arrays (u, b and the output, over every member of a batch) overflow the
// 256 MB last-level cache: the output then reaches HBM anyway, and its lines
// no longer evict the input lines that neighbouring strips and chunks
// re-read.  When the arrays fit, ordinary stores leave the output in that
// cache for the next sweep, which reads it.  (Measured on gfx950: 256^3
// float64 97.6 -> 82 us; float32 sweeps of the same size, whose arrays fit,
// were 20 % slower with the hints.)
constexpr size_t STRIP_NT_MIN_BYTES = (size_t)256 << 20;
template <typename T>
static int strip_nt(const LevelView<T>& L, const Batch& bt) {
  return 3 * (size_t)L.nx * L.ny * L.nz * sizeof(T) * (size_t)bt.nb > STRIP_NT_MIN_BYTES ? 1 : 0;
}

// The view the FLAT kernel marches: the 2-D level (nz = 1, ihz2 = 0) with y
// moved to the marching axis; the memory layout is unchanged.
template <typename T>
static LevelView<T> flat_view(const LevelView<T>& L) {
  LevelView<T> V = L;
  V.ny = 1;
  V.nz = L.ny;
  V.ihy2 = (T)0;
  V.ihz2 = L.ihy2;
  return V;
}

template <typename T, int S, int R, int WY, bool GS, bool FLAT, bool NT>
static void launch_strip_nt(const LevelView<T>& L, const StripGrid& g, const T* u, const T* b, T* out,
                            const FCoef<T, S>& fc, double* part, const int* stop, const Batch& bt, hipStream_t st) {
  const dim3 grid(g.nblk, bt.nb), block(64 * WY);
  if (L.periodic) {
    if (u == nullptr)
      hipLaunchKernelGGL((k_tau_strip<T, S, R, WY, true, true, GS, FLAT, NT>), grid, block, 0, st, L, u, b, out, fc,
                         g.zc, g.gx, g.gy, g.nblk, g.map, part, bt, stop);
    else
      hipLaunchKernelGGL((k_tau_strip<T, S, R, WY, true, false, GS, FLAT, NT>), grid, block, 0, st, L, u, b, out, fc,
                         g.zc, g.gx, g.gy, g.nblk, g.map, part, bt, stop);
  } else {
    if (u == nullptr)
      hipLaunchKernelGGL((k_tau_strip<T, S, R, WY, false, true, GS, FLAT, NT>), grid, block, 0, st, L, u, b, out, fc,
                         g.zc, g.gx, g.gy, g.nblk, g.map, part, bt, stop);
    else
      hipLaunchKernelGGL((k_tau_strip<T, S, R, WY, false, false, GS, FLAT, NT>), grid, block, 0, st, L, u, b, out,
                         fc, g.zc, g.gx, g.gy, g.nblk, g.map, part, bt, stop);
  }
}

template <typename T, int S, int R, int WY, bool GS, bool FLAT>
static void launch_strip_k(const LevelView<T>& L0, int target, const T* u, const T* b, T* out, const FCoef<T, S>& fc,
                           double* part, const int* stop, const Batch& bt, hipStream_t st) {
  const LevelView<T> L = FLAT ? flat_view(L0) : L0;
  const StripGrid g = strip_grid(S, R, WY, L.nx, L.ny, L.nz, target, FLAT);
  if constexpr (sizeof(T) == 8) {
    if (strip_nt<T>(L, bt)) return launch_strip_nt<T, S, R, WY, GS, FLAT, true>(L, g, u, b, out, fc, part, stop, bt, st);
  }
  launch_strip_nt<T, S, R, WY, GS, FLAT, false>(L, g, u, b, out, fc, part, stop, bt, st);
}

template <typename T, int S, int R, int WY>
void launch_strip(const LevelView<T>& L, int target, const T* u, const T* b, T* out, const FCoef<T, S>& fc,
                  double* part, const int* stop, const Batch& bt, hipStream_t st) {
  launch_strip_k<T, S, R, WY, false, false>(L, target, u, b, out, fc, part, stop, bt, st);
}

// stacked wavefronts with shared y halo rows (3-D levels, WY > 1)
template <typename T, int S, int R, int WY, bool NT>
static void launch_strip_yx_nt(const LevelView<T>& L, const StripGrid& g, const T* u, const T* b, T* out,
                               const FCoef<T, S>& fc, double* part, const int* stop, const Batch& bt, hipStream_t st) {
  const dim3 grid(g.nblk, bt.nb), block(64 * WY);
  if (L.periodic) {
    if (u == nullptr)
      hipLaunchKernelGGL((k_tau_strip_yx<T, S, R, WY, true, true, false, NT>), grid, block, 0, st, L, u, b, out, fc,
                         g.zc, g.gx, g.gy, g.nblk, g.map, part, bt, stop);
    else
      hipLaunchKernelGGL((k_tau_strip_yx<T, S, R, WY, true, false, false, NT>), grid, block, 0, st, L, u, b, out, fc,
                         g.zc, g.gx, g.gy, g.nblk, g.map, part, bt, stop);
  } else {
    if (u == nullptr)
      hipLaunchKernelGGL((k_tau_strip_yx<T, S, R, WY, false, true, false, NT>), grid, block, 0, st, L, u, b, out, fc,
                         g.zc, g.gx, g.gy, g.nblk, g.map, part, bt, stop);
    else
      hipLaunchKernelGGL((k_tau_strip_yx<T, S, R, WY, false, false, false, NT>), grid, block, 0, st, L, u, b, out,
                         fc, g.zc, g.gx, g.gy, g.nblk, g.map, part, bt, stop);
  }
}

template <typename T, int S, int R, int WY>
void launch_strip_yx(const LevelView<T>& L, int target, const T* u, const T* b, T* out, const FCoef<T, S>& fc,
                     double* part, const int* stop, const Batch& bt, hipStream_t st) {
  const StripGrid g = strip_grid(S, R, WY, L.nx, L.ny, L.nz, target, false);
  if constexpr (sizeof(T) == 8) {
    if (strip_nt<T>(L, bt)) return launch_strip_yx_nt<T, S, R, WY, true>(L, g, u, b, out, fc, part, stop, bt, st);
  }
  launch_strip_yx_nt<T, S, R, WY, false>(L, g, u, b, out, fc, part, stop, bt, st);
}

template <typename T, int S, int R, int WY>
void launch_strip2d(const LevelView<T>& L, int target, const T* u, const T* b, T* out, const FCoef<T, S>& fc,
                    double* part, const int* stop, const Batch& bt, hipStream_t st) {
  launch_strip_k<T, S, R, WY, false, true>(L, target, u, b, out, fc, part, stop, bt, st);
}

// one red-black GS / SOR iteration in one pass: the two-stage strip kernel
// with mu = 1, nu = 0, c = omega / D on the cells of each stage's colour
template <typename T, int R, int WY, bool FLAT>
void launch_strip_gsrb(const LevelView<T>& L, int target, const T* u, const T* b, T* out, double omega_over_d,
                       double* part, const int* stop, const Batch& bt, hipStream_t st) {
  FCoef<T, 2> fc;
  for (int j = 0; j < 2; ++j) {
    fc.mu[j] = (T)1;
    fc.nu[j] = (T)0;
    fc.c[j] = (T)omega_over_d;
  }
  launch_strip_k<T, 2, R, WY, true, FLAT>(L, target, u, b, out, fc, part, stop, bt, st);
}

#define RKL_STRIP_INST(T, S, R, WY)                                                                          \
  template void launch_strip<T, S, R, WY>(const LevelView<T>&, int, const T*, const T*, T*, const FCoef<T, S>&, \
                                          double*, const int*, const Batch&, hipStream_t);
RKL_STRIP_INST(double, 1, 8, 4)
RKL_STRIP_INST(double, 2, 8, 4)
RKL_STRIP_INST(double, 1, 8, 1)
RKL_STRIP_INST(double, 2, 8, 1)
RKL_STRIP_INST(float, 1, 8, 4)
RKL_STRIP_INST(float, 2, 8, 4)
RKL_STRIP_INST(float, 3, 8, 4)
RKL_STRIP_INST(float, 1, 8, 1)
RKL_STRIP_INST(float, 2, 8, 1)
RKL_STRIP_INST(float, 3, 8, 1)
RKL_STRIP_INST(double, 1, 4, 4)
RKL_STRIP_INST(double, 2, 4, 4)
RKL_STRIP_INST(float, 1, 4, 4)
RKL_STRIP_INST(float, 2, 4, 4)
RKL_STRIP_INST(float, 3, 4, 4)
RKL_STRIP_INST(double, 1, 5, 1)
RKL_STRIP_INST(double, 2, 5, 1)
RKL_STRIP_INST(float, 1, 5, 1)
RKL_STRIP_INST(float, 2, 5, 1)
RKL_STRIP_INST(float, 3, 5, 1)
#undef RKL_STRIP_INST
#define RKL_STRIPYX_INST(T, S, R, WY)                                                                        \
  template void launch_strip_yx<T, S, R, WY>(const LevelView<T>&, int, const T*, const T*, T*,               \
                                             const FCoef<T, S>&, double*, const int*, const Batch&, hipStream_t);
RKL_STRIPYX_INST(double, 1, 8, 4)
RKL_STRIPYX_INST(double, 2, 8, 4)
RKL_STRIPYX_INST(double, 1, 4, 8)
RKL_STRIPYX_INST(double, 2, 4, 8)
RKL_STRIPYX_INST(float, 1, 8, 4)
RKL_STRIPYX_INST(float, 2, 8, 4)
RKL_STRIPYX_INST(float, 3, 8, 4)
RKL_STRIPYX_INST(float, 1, 4, 8)
RKL_STRIPYX_INST(float, 2, 4, 8)
RKL_STRIPYX_INST(float, 3, 4, 8)
RKL_STRIPYX_INST(double, 1, 8, 8)
RKL_STRIPYX_INST(double, 2, 8, 8)
RKL_STRIPYX_INST(float, 1, 8, 8)
RKL_STRIPYX_INST(float, 2, 8, 8)
RKL_STRIPYX_INST(float, 3, 8, 8)
RKL_STRIPYX_INST(double, 1, 2, 8)
RKL_STRIPYX_INST(double, 2, 2, 8)
RKL_STRIPYX_INST(float, 1, 2, 8)
RKL_STRIPYX_INST(float, 2, 2, 8)
RKL_STRIPYX_INST(double, 1, 2, 16)
RKL_STRIPYX_INST(double, 2, 2, 16)
RKL_STRIPYX_INST(float, 1, 2, 16)
RKL_STRIPYX_INST(float, 2, 2, 16)
#undef RKL_STRIPYX_INST
#define RKL_STRIP2D_INST(T, S, R, WY)                                                                          \
  template void launch_strip2d<T, S, R, WY>(const LevelView<T>&, int, const T*, const T*, T*, const FCoef<T, S>&, \
                                            double*, const int*, const Batch&, hipStream_t);
RKL_STRIP2D_INST(double, 1, 8, 1)
RKL_STRIP2D_INST(double, 2, 8, 1)
RKL_STRIP2D_INST(double, 1, 4, 1)
RKL_STRIP2D_INST(double, 2, 4, 1)
RKL_STRIP2D_INST(float, 1, 8, 1)
RKL_STRIP2D_INST(float, 2, 8, 1)
RKL_STRIP2D_INST(float, 3, 8, 1)
RKL_STRIP2D_INST(float, 1, 4, 1)
RKL_STRIP2D_INST(float, 2, 4, 1)
RKL_STRIP2D_INST(float, 3, 4, 1)
RKL_STRIP2D_INST(double, 3, 4, 1)
RKL_STRIP2D_INST(double, 4, 4, 1)
RKL_STRIP2D_INST(float, 4, 8, 1)
RKL_STRIP2D_INST(float, 4, 4, 1)
#undef RKL_STRIP2D_INST
#define RKL_GSRB_INST(T, R, WY, FLAT)                                                                          \
  template void launch_strip_gsrb<T, R, WY, FLAT>(const LevelView<T>&, int, const T*, const T*, T*, double,     \
                                                  double*, const int*, const Batch&, hipStream_t);
RKL_GSRB_INST(double, 8, 4, false)
RKL_GSRB_INST(double, 4, 4, false)
RKL_GSRB_INST(float, 8, 4, false)
RKL_GSRB_INST(float, 4, 4, false)
RKL_GSRB_INST(double, 8, 1, true)
RKL_GSRB_INST(double, 4, 1, true)
RKL_GSRB_INST(float, 8, 1, true)
RKL_GSRB_INST(float, 4, 1, true)
#undef RKL_GSRB_INST

}  // namespace rkl
