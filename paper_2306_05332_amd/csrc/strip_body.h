// Body of the fused s-stage strip tau-step, shared by the translation units
// that instantiate its kernels (strip.hip: plain tau-steps; strip_forms64.hip
// and strip_forms32.hip: the prolongation, stage-chunk and restriction forms).
//
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
// before any relaxation, so no face array is read here).  The 3-D RKL forms
// (other than PRO) hold those ghosts in the operands themselves (GO): after
// each load and each stage, the row, column or plane just outside a face is
// set to minus its in-box neighbour, under wavefront-uniform branches that
// only the wavefronts touching a face take, so the stencil is the periodic
// one with no per-cell selects (those selects had made Dirichlet sweeps issue
// half as many VALU instructions again as periodic ones).  The GS, 2-D and
// PRO forms select the ghost inside the stencil (PRO: the operand fix-ups
// measured slower there, its registers being at the four-wave limit).
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
//
// With PRO = true the tau-step's input is u + P e, e being the next coarser
// level's correction and P the trilinear prolongation of eq.
// prolongation_example_3D (Sec. 2.1 steps 4-5: prolongation, correction and
// the first post-smoothing relaxation in one pass).  Along each axis a fine
// cell takes 3/4 of its parent coarse cell and 1/4 of the parent's
// neighbour on the fine cell's side; coarse ghosts wrap (periodic) or take
// -e (homogeneous Dirichlet).  R is even, so a strip's first row is an even
// row minus S and each held row's two coarse rows are fixed offsets from the
// strip's first coarse row.  A coarse plane is interpolated in x and y once,
// onto the lane's rows, and then serves the four fine planes around it
// (two queue slots); the corrected u itself is never stored.
//
// With RS = true the tau-step is the last pre-smoothing relaxation of a
// level and also produces the next level's right-hand side (Sec. 2.1 steps
// 2a-2b): r = b - M Y_S at every cell it owns, restricted by the 8-child
// average of eq. restriction_example_3D, so Y_S is not read back by a
// separate residual pass.  The residual needs Y_S one cell beyond the owned
// ones, so the tile keeps one more halo lane on either side in x, the chunk
// computes Y_S on one more plane on either side in z, and in y the
// workgroup's first and last computed rows are the residual's halo (tiles
// overlap by two rows; every owned row and its neighbours are rows the
// workgroup computes exactly).  The wavefronts put their Y_S rows of each
// plane into an LDS ring of four planes; after the iteration's barrier the
// residual of the plane below the newest one is taken from the ring, two
// rows (one coarse row) at a time: the y pair is summed in the lane, the z
// pair across two iterations, the x pair by a lane shift.  The float64
// partial sums are those of the separate residual + restriction pass:
// (fine r^2, sum of coarse values) per workgroup.
#pragma once

#include "kernels.h"

namespace rkl {

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
inline int strip_nt(const LevelView<T>& L, const Batch& bt) {
  return 3 * (size_t)L.nx * L.ny * L.nz * sizeof(T) * (size_t)bt.nb > STRIP_NT_MIN_BYTES ? 1 : 0;
}

// Minimum wavefronts per SIMD asked of the compiler for a strip kernel: the
// float64 stacked two-row strips (eight wavefronts) keep four per SIMD, two
// workgroups per CU (128 VGPRs), in their fused forms, whose Dirichlet
// instantiations would otherwise take a few registers more and lose half of
// their occupancy.
template <typename T, int R, int WY>
constexpr int strip_min_waves() {
  return (sizeof(T) == 8 && R == 2 && WY == 8) ? 4 : 1;
}

// floor(x / 2) for any sign
constexpr int fdiv2(int x) { return x >= 0 ? x / 2 : -((1 - x) / 2); }

template <typename T, int S, int R, int WY, bool PER, bool UZ, bool GS, bool FLAT, bool SHY, bool NT,
          bool PRO = false, bool CH = false, bool RS = false>
__device__ __forceinline__ void tau_strip_body(LevelView<T> L, const T* __restrict__ u, const T* __restrict__ b,
                                               T* __restrict__ out, FCoef<T, S> co, int zc, int gx_tiles,
                                               int gy_tiles, int nblk, StripMap sm, double* __restrict__ part,
                                               Batch bt, const int* __restrict__ stop,
                                               const T* __restrict__ ec = nullptr, const T* __restrict__ v = nullptr,
                                               T* __restrict__ out2 = nullptr, T* __restrict__ bc = nullptr) {
  static_assert(!SHY || (WY > 1 && !FLAT && R >= S), "shared y halos need stacked 3-D strips of >= S rows");
  static_assert(!PRO || (!UZ && !GS && !FLAT && R % 2 == 0), "prolongation fusion: 3-D RKL strips of even R");
  static_assert(!CH || (!UZ && !GS && !FLAT && !SHY && !PRO), "stage chunks: 3-D RKL strips, own halo rows");
  static_assert(!RS || (!UZ && !GS && !FLAT && !PRO && !CH && WY > 1 && R % 2 == 0 && S >= 2),
                "restriction fusion: stacked 3-D RKL strips of even R, s >= 2 (a b halo row in registers)");
  {
    const long long mb = blockIdx.y;
    if (PRO) ec += mb * bt.s1;
    if (RS) bc += mb * bt.s1;
    if (CH) {
      v += mb * bt.s0;
      out2 += mb * bt.s0;
    }
    if (!UZ) u += mb * bt.s0;
    b += mb * bt.s0;
    out += mb * bt.s0;
    if (part != nullptr) part += mb * bt.part_stride;
    if (stop != nullptr) stop += mb * bt.stop_stride;
  }
  constexpr int HY = FLAT ? 0 : S;  // halo rows on either side of the R output rows
  constexpr int NU = R + 2 * HY;    // rows held per lane
  constexpr int XH = RS ? S + 1 : S;  // halo lanes on either side of the output columns
  constexpr int OX = 64 - 2 * XH;   // output columns per wavefront (per segment when FLAT)
  constexpr int NY = S > 1 ? S - 1 : 1;
  constexpr int A1 = FLAT ? 0 : 1;  // first row of stage 1 (stage j starts at row A1 * j)
  constexpr int TR = WY * R;        // rows the workgroup's stages cover
  constexpr int TS = RS ? TR - 2 : TR;  // rows it owns (RS: all but the first and the last)
  constexpr int ZE = RS ? 1 : 0;    // planes of Y_S computed beyond the chunk on either side
  constexpr int MP = RS ? R / 2 : 1;  // RS: row pairs per wavefront
  __shared__ double red[WY];
  // RS: Y_S of the last four planes, every row the workgroup computes
  __shared__ T ysr[RS ? 4 : 1][RS ? TR : 1][64];
  // SHY: the wavefronts of a workgroup are stacked in y, and each takes the
  // halo rows it shares with its neighbours from their registers through LDS
  // (double-buffered): [buffer][wavefront][side][row][lane], side 0 = the
  // wavefront's lowest S rows of u (and S - 1 of b) for the one below's upper
  // halo, side 1 = its highest rows for the one above's lower halo
  constexpr int XU = S, XB = S > 1 ? S - 1 : 1;
  __shared__ T xch[SHY ? 2 : 1][SHY ? WY : 1][2][SHY ? XU + XB : 1][64];
  lds_poison(red, WY);
  lds_poison(&xch[0][0][0][0][0], (SHY ? 2 : 1) * (SHY ? WY : 1) * 2 * (SHY ? XU + XB : 1) * 64);
  if (RS) lds_poison(&ysr[0][0][0], (RS ? 4 * TR : 1) * 64);
  lds_poison_sync();
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
  const int gxu = tx * OX - XH + xl;         // column of this lane (unwrapped; 3-D form)
  const int ybase = ty * TS - (RS ? 1 : 0);  // first row the workgroup computes (unwrapped)
  const int y0 = FLAT ? 0 : ybase + w * R - S;  // row of strip index 0 (unwrapped, wave-uniform)
  const int z0 = tz * zc, z1 = min(z0 + zc, nz);
  const bool xin = gxu >= 0 && gxu < nx;
  const int gx = PER ? ((gxu % nx) + nx) % nx : min(max(gxu, 0), nx - 1);
  // byte offset of this lane's column (and, in a packed wavefront, of its strip's rows)
  const unsigned xb = ((unsigned)gx + (unsigned)yshift * (unsigned)nx) * (unsigned)sizeof(T);
  const bool xown = xl >= XH && xl < xw - XH && xin;
  const bool xlo = !PER && gxu == 0, xhi = !PER && gxu == nx - 1;
  // GO: Dirichlet ghosts held in the operands (3-D RKL forms).  xgl / xgr:
  // the wavefront holds the column just outside the low / high x face;
  // ylo / yhi: held row indices of the rows just outside the y faces (yg:
  // either is held)
  constexpr bool GO = !PER && !GS && !FLAT && !PRO;
  const bool xgl = GO && __ballot(gxu == -1) != 0ull, xgr = GO && __ballot(gxu == nx) != 0ull;
  const int ylo = FLAT ? -1 : -1 - y0, yhi = FLAT ? -1 : ny - y0;
  const bool yg = GO && ((ylo >= 0 && ylo < NU) || (yhi >= 0 && yhi < NU));
  const bool gface = yg || xgl || xgr;  // one uniform test for interior wavefronts
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
  // PRO: coarse geometry.  Held row i is fine row 2 cb + (i - S), cb being
  // the strip's first coarse row; its parent coarse row is cb + fdiv2(i - S)
  // and the parent's neighbour on its side is one row up (odd fine row) or
  // down (even).  Coarse rows CLO .. CHI (relative to cb) cover every held row.
  constexpr int CLO = PRO ? fdiv2(-S) - 1 : 0;
  constexpr int CHI = PRO ? fdiv2(NU - 1 - S) + 1 : 0;
  constexpr int NC = CHI - CLO + 1;
  auto cpar = [](int i) { return fdiv2(i - S) - CLO; };                             // parent, slot index
  auto cnb = [](int i) { return fdiv2(i - S) + (((i - S) & 1) ? 1 : -1) - CLO; };  // neighbour, slot index
  const int cnx = nx >> 1, cny = ny >> 1, cnz = nz >> 1;
  const long long csxy = (long long)cnx * cny;
  unsigned cxp = 0, cxn = 0;  // byte offsets of the lane's parent and neighbour coarse columns
  T sxn = (T)1;               // sign of the neighbour column (-1: Dirichlet ghost)
  long long coff[PRO ? NC : 1];
  T csg[PRO ? NC : 1];
  if constexpr (PRO) {
    const int I = gx >> 1;
    int In = I + ((gx & 1) ? 1 : -1);
    if (PER) In = In < 0 ? In + cnx : (In >= cnx ? In - cnx : In);
    else if (In < 0 || In >= cnx) {
      In = I;
      sxn = (T)-1;
    }
    cxp = (unsigned)I * (unsigned)sizeof(T);
    cxn = (unsigned)In * (unsigned)sizeof(T);
    const int cb = (ty * WY + w) * (R / 2);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      int J = cb + CLO + c;
      csg[c] = (T)1;
      if (PER) J = ((J % cny) + cny) % cny;
      else if (J < 0 || J >= cny) {
        J = J < 0 ? 0 : cny - 1;
        csg[c] = (T)-1;
      }
      coff[c] = (long long)J * cnx;
    }
  }
  // PRO, float64 (PDMA): a coarse plane's rows arrive in LDS by direct loads
  // (global_load_lds_dwordx4: 16 bytes per lane, nothing held in registers
  // while the stages run): of each needed row slot, the wavefront's coarse
  // columns cb0 .. cb0 + 35 (unwrapped; cb0 even and at most one left of lane
  // 0's parent), lane l < 18 fetching the column pair cb0 / 2 + l (pairs never
  // straddle the periodic wrap, the extent being even; Dirichlet clamps whole
  // pairs, and the clamped columns are never read).  cofp / cofn: the lane's
  // parent and neighbour column within that row (a Dirichlet ghost neighbour
  // reads the parent, with sign sxn = -1).
  constexpr bool PDMA = PRO && sizeof(T) == 8;
  constexpr int DMA_LANES = 18;
  __shared__ double cdma[PDMA ? WY : 1][PDMA ? NC : 1][2 * DMA_LANES];
  unsigned cdo = 0u;
  int cofp = 0, cofn = 0;
  if constexpr (PDMA) {
    int cb0 = fdiv2(tx * OX - S) - 1;
    cb0 -= cb0 & 1;
    const int cu = fdiv2(gxu);
    cofp = cu - cb0;
    cofn = cofp;
    if (!(sxn < (T)0)) cofn = cofp + ((gxu & 1) ? 1 : -1);
    const int cnp = cnx >> 1;  // column pairs per coarse row
    int pj = (cb0 >> 1) + min(lane, DMA_LANES - 1);
    pj = PER ? ((pj % cnp) + cnp) % cnp : min(max(pj, 0), cnp - 1);
    cdo = (unsigned)pj * 16u;
    lds_poison(&cdma[0][0][0], WY * NC * 2 * DMA_LANES);
    lds_poison_sync();
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
  // PRO: coarse row slot c is read when a row this wavefront loads uses it
  auto cneed = [&](int c) -> bool {
    bool need = false;
#pragma unroll
    for (int i = 0; i < NU; ++i)
      if (gl(i) && (cpar(i) == c || cnb(i) == c)) need = true;
    return need;
  };
  // PRO: issue the loads of coarse plane K (wrapped, or clamped for a
  // Dirichlet ghost plane, whose sign is returned): per coarse row slot the
  // parent and the neighbour column of the lane
  auto cload = [&](int K, T(&C)[PRO && !PDMA ? NC : 1][2]) -> T {
    T sz = (T)1;
    if constexpr (PRO) {
      int Kw;
      if (PER) Kw = ((K % cnz) + cnz) % cnz;
      else {
        Kw = K < 0 ? 0 : (K >= cnz ? cnz - 1 : K);
        if (K < 0 || K >= cnz) sz = (T)-1;
      }
      const T* __restrict__ ep = ec + (long long)Kw * csxy;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if constexpr (PDMA) {
          if (cneed(c) && lane < DMA_LANES) {
            const char* rb = (const char*)(ep + coff[c]);
            __builtin_amdgcn_global_load_lds((const void*)(rb + cdo),
                                             (__attribute__((address_space(3))) void*)&cdma[w][c][0], 16, 0, 0);
          }
        } else {
          C[c][0] = C[c][1] = (T)0;
          if (cneed(c)) {
            const char* rb = (const char*)(ep + coff[c]);
            C[c][0] = *(const T*)(rb + cxp);
            C[c][1] = *(const T*)(rb + cxn);
          }
        }
      }
    }
    return sz;
  };
  // PRO: E[i] = 64 x (coarse plane C interpolated in x and y onto held row i),
  // ghost signs included (x, then y, as eq. prolongation_example_3D weighs)
  auto cfin = [&](const T(&C)[PRO && !PDMA ? NC : 1][2], T sz, T(&E)[PRO ? NU : 1]) {
    if constexpr (PRO) {
      T X[NC];
      if constexpr (PDMA) {
        // vmcnt(0): the direct loads have landed in LDS (the fence keeps the
        // compiler from moving the reads above the wait)
        __builtin_amdgcn_s_waitcnt(0x0F70);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          X[c] = (T)0;
          if (cneed(c)) X[c] = (sz * csg[c]) * ((T)3 * (T)cdma[w][c][cofp] + sxn * (T)cdma[w][c][cofn]);
        }
      } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) X[c] = (sz * csg[c]) * ((T)3 * C[c][0] + sxn * C[c][1]);
      }
#pragma unroll
      for (int i = 0; i < NU; ++i)
        if (gl(i)) E[i] = (T)3 * X[cpar(i)] + X[cnb(i)];
    }
  };
  // PRO: EA / EB hold the interpolants of coarse planes Kl(p) = fdiv2(p - 1)
  // and Kl(p) + 1 for the fine plane p last loaded; the parent plane of p
  // (EB for even p, EA for odd p) weighs 3, the other 1
  T EA[PRO ? NU : 1], EB[PRO ? NU : 1];
  T CRw[PRO && !PDMA ? NC : 1][2];  // raw values of a coarse plane in flight (float32)
#pragma unroll
  for (int i = 0; i < (PRO ? NU : 1); ++i) EA[i] = EB[i] = (T)0;
  auto corr = [&](T v, int p, int i) -> T {  // v + (P e) at plane p, held row i
    if constexpr (PRO) return v + ((p & 1) ? ((T)3 * EA[i] + EB[i]) : (EA[i] + (T)3 * EB[i])) * (T)(1.0 / 64.0);
    else return v;
  };
  // PRO: make EA / EB current for fine plane p, given that they were for p - 1
  auto pro_step = [&](int p) {
    if constexpr (PRO) {
      if (p & 1) {
#pragma unroll
        for (int i = 0; i < NU; ++i) EA[i] = EB[i];
        const T sz = cload(fdiv2(p + 1), CRw);
        cfin(CRw, sz, EB);
      }
    }
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
      if (!PER && !GO) {
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

  // GO: set the held row / column just outside a face to minus its in-box
  // neighbour in one plane's rows of an operand; the column only in rows
  // IA .. IB - 1, those the next stage takes as stencil centres (the other
  // rows serve as y neighbours of the same column only)
  auto gfix = [&](T(&Y)[NU], int ia, int ib) {
    if constexpr (GO) {
      if (!gface) return;
      if (yg) {
#pragma unroll
        for (int i = 0; i < NU; ++i) {
          if (i + 1 < NU && i == ylo) Y[i] = -Y[i + 1];
          if (i >= 1 && i == yhi) Y[i] = -Y[i - 1];
        }
      }
      if (xgl) {
#pragma unroll
        for (int i = 0; i < NU; ++i) {
          if (i < ia || i >= ib) continue;
          const T l = wshift<DPP_WAVE_SHL1>(Y[i]);
          if (gxu == -1) Y[i] = -l;
        }
      }
      if (xgr) {
#pragma unroll
        for (int i = 0; i < NU; ++i) {
          if (i < ia || i >= ib) continue;
          const T r = wshift<DPP_WAVE_SHR1>(Y[i]);
          if (gxu == nx) Y[i] = -r;
        }
      }
    }
  };

  // GO: the plane just outside a z face, before a stage at plane p reads it
  // (zface: the chunk's stages can reach a z face)
  const bool zface = GO && (z0 <= S + 1 || z1 + S + 1 >= nz);
  auto zfix = [&](T(&Zm)[NU], const T(&X)[NU], T(&Zp)[NU], int p) {
    if constexpr (GO) {
      if (!zface) return;
      if (p == 0) {
#pragma unroll
        for (int i = 0; i < NU; ++i) Zm[i] = -X[i];
      }
      if (p == nz - 1) {
#pragma unroll
        for (int i = 0; i < NU; ++i) Zp[i] = -X[i];
      }
    }
  };

  T U0[NU], U1[NU], U2[NU], UN[NU];  // u at planes zl-1, zl, zl+1; zl+2 in flight
  T Yq[NY][3][NU];                   // Y_j at planes zl-j-1, zl-j, zl-j+1 (after stage j of iteration zl)
  T Bq[S][NU], BN[NU];               // b at planes zl, zl-1, ..; zl+1 in flight
  // iterations: stage 1 of plane zl, stage j of zl - j + 1
  const int zs = z0 - (S - 1) - ZE, ze = z1 + S - 2 + ZE;
  long long ou = plane0(zs - 1);   // plane offset of the last u plane loaded
  long long ob = plane0(zs);       // plane offset of the last b plane loaded
  long long oo = plane0(zs - S + 1);  // plane offset of the stage-S output plane of iteration zs
  long long oo2 = plane0(zs - S + 2);  // CH: plane offset of the stage-(S-1) output plane
  // CH: the chunk's Y_{j0-2} (pointwise input of its first stage) at the
  // plane of stage 1, and the next plane in flight
  T Vc[CH ? NU : 1], VN[CH ? NU : 1];
#pragma unroll
  for (int i = 0; i < NU; ++i) {
    for (int j = 0; j < NY; ++j) Yq[j][0][i] = Yq[j][1][i] = Yq[j][2][i] = (T)0;
    for (int j = 0; j < S; ++j) Bq[j][i] = (T)0;
  }
  // rows outside a Dirichlet box and planes outside it read as 0
  if constexpr (PRO) {
    const int kl = fdiv2(zs - 2);  // Kl(zs - 1)
    T sz = cload(kl, CRw);
    cfin(CRw, sz, EA);
    sz = cload(kl + 1, CRw);
    cfin(CRw, sz, EB);
  }
#pragma unroll
  for (int i = 0; i < NU; ++i)
    if (gl(i)) U0[i] = (UZ || !pin(zs - 1) || !(PER || ((rin >> i) & 1u))) ? (T)0 : corr(row(u, ou, i), zs - 1, i);
  ou = next_plane(ou, zs);
  pro_step(zs);
#pragma unroll
  for (int i = 0; i < NU; ++i)
    if (gl(i)) U1[i] = (UZ || !pin(zs) || !(PER || ((rin >> i) & 1u))) ? (T)0 : corr(row(u, ou, i), zs, i);
  ou = next_plane(ou, zs + 1);
  pro_step(zs + 1);
#pragma unroll
  for (int i = 0; i < NU; ++i)
    if (gl(i)) U2[i] = (UZ || !pin(zs + 1) || !(PER || ((rin >> i) & 1u))) ? (T)0 : corr(row(u, ou, i), zs + 1, i);
#pragma unroll
  for (int i = A1; i < NU - A1; ++i)
    if (gl(i)) Bq[0][i] = (!pin(zs) || !(PER || ((rin >> i) & 1u))) ? (T)0 : row(b, ob, i);
  if constexpr (CH) {
#pragma unroll
    for (int i = A1; i < NU - A1; ++i) Vc[i] = (!pin(zs) || !(PER || ((rin >> i) & 1u))) ? (T)0 : row(v, ob, i);
  }
  exchange(U0, Bq[0], !UZ, false);
  exchange(U1, Bq[0], !UZ, false);
  exchange(U2, Bq[0], !UZ, true);
  if constexpr (!UZ) {  // a zero input needs no ghosts
    gfix(U0, A1, NU - A1);
    gfix(U1, A1, NU - A1);
    gfix(U2, A1, NU - A1);
  }
  double r2 = 0.0;
  T YS[NU];  // Y_S of the iteration's output plane, stored after the queues advance
  // RS: pair k of the wavefront covers its held rows HY + 1 + 2k and the
  // next one (the last pair's second row is the b halo row above its own
  // rows, which the stages hold anyway; the workgroup's last pair would
  // start on its last computed row and is not taken).  The residual of plane
  // q runs at the end of iteration q + S, after the barrier that completes
  // the ring's plane q + 1 (placed at the top of the next iteration, where
  // the loads in flight would hide its latency, it needs more registers than
  // four wavefronts per SIMD allow and measured slower).  BR[k] / BB[k]: b
  // of the pair's two rows at planes q and q + 1, taken from the b queue
  // (Bq[S - 1] holds b of the plane whose Y_S an iteration computes);
  // acc[k]: the y-pair sums of the pair's even plane
  double rs2 = 0.0, rs1 = 0.0;
  T BR[MP][2], BB[MP][2], acc[MP];
  const int cnxr = nx >> 1;
  const long long cnxyr = (long long)cnxr * (ny >> 1);
#pragma unroll
  for (int k = 0; k < MP; ++k) BR[k][0] = BR[k][1] = BB[k][0] = BB[k][1] = acc[k] = (T)0;
  // RS: residual + restriction of plane q from the ring
  auto resid_plane = [&](int q) {
    if constexpr (RS) {
      if (q >= z0 && q < z1) {
        const int sl = (q - 1) & 3, sc = q & 3, su = (q + 1) & 3;
#pragma unroll
        for (int k = 0; k < MP; ++k) {
          const int a = w * R + 1 + 2 * k;  // tile row of the pair's first row
          if (a + 1 <= TR - 2) {
            const int ga = ybase + a;
            const T c0 = ysr[sc][a][lane], c1 = ysr[sc][a + 1][lane];
            T ym = ysr[sc][a - 1][lane], yp = ysr[sc][a + 2][lane];
            T zm0 = ysr[sl][a][lane], zm1 = ysr[sl][a + 1][lane];
            T zp0 = ysr[su][a][lane], zp1 = ysr[su][a + 1][lane];
            T xm0 = wshift<DPP_WAVE_SHR1>(c0), xp0 = wshift<DPP_WAVE_SHL1>(c0);
            T xm1 = wshift<DPP_WAVE_SHR1>(c1), xp1 = wshift<DPP_WAVE_SHL1>(c1);
            if (!PER) {
              if (xlo) {
                xm0 = -c0;
                xm1 = -c1;
              }
              if (xhi) {
                xp0 = -c0;
                xp1 = -c1;
              }
              if (ga == 0) ym = -c0;
              if (ga + 1 == ny - 1) yp = -c1;
              if (q == 0) {
                zm0 = -c0;
                zm1 = -c1;
              }
              if (q == nz - 1) {
                zp0 = -c0;
                zp1 = -c1;
              }
            }
            const T l0 = ((xm0 + xp0) - (T)2 * c0) * L.ihx2 + ((ym + c1) - (T)2 * c0) * L.ihy2 +
                         ((zm0 + zp0) - (T)2 * c0) * L.ihz2;
            const T l1 = ((xm1 + xp1) - (T)2 * c1) * L.ihx2 + ((c0 + yp) - (T)2 * c1) * L.ihy2 +
                         ((zm1 + zp1) - (T)2 * c1) * L.ihz2;
            const T r0 = BR[k][0] - l0, r1 = BR[k][1] - l1;
            const bool ok = xown && ga < ny;
            if (ok) rs2 += (double)r0 * (double)r0 + (double)r1 * (double)r1;
            const T yr = r0 + r1;
            if (q & 1) {
              const T zsum = acc[k] + yr;
              const T cv = (zsum + wshift<DPP_WAVE_SHL1>(zsum)) * (T)0.125;
              if (ok && !(gx & 1)) {
                bc[(long long)(q >> 1) * cnxyr + (long long)(ga >> 1) * cnxr + (gx >> 1)] = cv;
                rs1 += (double)cv;
              }
            } else {
              acc[k] = yr;
            }
          }
        }
      }
    }
  };

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
    if constexpr (CH) {
#pragma unroll
      for (int i = A1; i < NU - A1; ++i) VN[i] = row(v, ob, i);
    }
    // PRO: fine plane zl + 2 brings in a new coarse plane when odd: its loads
    // are issued here (into registers in float32, into LDS in float64) and it
    // is interpolated when UN is consumed
    const bool cnew = PRO && more && ((zl + 2) & 1);
    T csz = (T)1;
    if constexpr (PRO) {
      if (cnew) csz = cload(fdiv2(zl + 3), CRw);
    }
    // stage 1 at plane zl, rows A1 .. NU-1-A1
    {
      const int p = zl;
      const bool on = pin(p) && p >= z0 - (S - 1) - ZE && p <= z1 - 1 + (S - 1) + ZE;
      const bool pown = !RS && p >= z0 && p < z1;
      if (on) {
        if constexpr (!UZ) zfix(U0, U1, U2, p);
#pragma unroll
        for (int i = A1; i < NU - A1; ++i) {
          const T res = lap(U0, U1, U2, i, p) - Bq[0][i];
          T y;
          if (GS) {
            y = U1[i] + gscoef(co.c[0], i, p) * res;
            if ((xpar(i) ^ ((rodd >> i) & 1) ^ zodd(p)) != 0) y = U1[i];  // black cell: unchanged
          } else {
            if constexpr (CH) y = co.mu[0] * U1[i] + co.nu[0] * Vc[i] + co.c[0] * res;
            else y = U1[i] + co.c[0] * res;
          }
          if (part != nullptr && pown && i >= HY && i < HY + R && own(i) && ((rin >> i) & 1u))
            r2 += (double)res * (double)res;
          if constexpr (S == 1) YS[i] = y;
          else Yq[0][2][i] = y;
        }
        if constexpr (S > 1) gfix(Yq[0][2], 2 * A1, NU - 2 * A1);
      }
    }
    // stages 2 .. S at planes zl - j + 1, rows A1 j .. NU-1-A1 j
#pragma unroll
    for (int j = 2; j <= S; ++j) {
      const int p = zl - j + 1;
      const bool on = pin(p) && p >= z0 - (S - j) - ZE && p <= z1 - 1 + (S - j) + ZE;
      if (on) {
        zfix(Yq[j - 2][0], Yq[j - 2][1], Yq[j - 2][2], p);
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
        if (j < S) gfix(Yq[j < S ? j - 1 : 0][2], A1 * (j + 1), NU - A1 * (j + 1));
      }
    }
    // RS: the wavefront's rows of Y_S into the ring; b of the pairs' rows at
    // that plane into BB (BR: the plane below, whose residual the next
    // iteration takes)
    if constexpr (RS) {
      const int p = zl - S + 1;
      if (pin(p) && p >= z0 - 1 && p <= z1) {
#pragma unroll
        for (int i = HY; i < HY + R; ++i) ysr[p & 3][w * R + i - HY][lane] = YS[i];
      }
#pragma unroll
      for (int k = 0; k < MP; ++k) {
        BR[k][0] = BB[k][0];
        BR[k][1] = BB[k][1];
        BB[k][0] = Bq[S - 1][HY + 1 + 2 * k];
        BB[k][1] = Bq[S - 1][HY + 2 + 2 * k];
      }
    }
    // advance the queues; Dirichlet planes outside the box and rows outside it read as 0
    const bool un_ok = pin(zl + 2), bn_ok = pin(zl + 1);
    if constexpr (PRO) {
      if (cnew) {
#pragma unroll
        for (int i = 0; i < NU; ++i) EA[i] = EB[i];
        cfin(CRw, csz, EB);
      }
    }
#pragma unroll
    for (int i = 0; i < NU; ++i) {
      const bool rok = PER || ((rin >> i) & 1u);
      U0[i] = U1[i];
      U1[i] = U2[i];
      if constexpr (GO) U2[i] = UZ ? (T)0 : corr(UN[i], zl + 2, i);
      else U2[i] = (UZ || !un_ok || !rok) ? (T)0 : corr(UN[i], zl + 2, i);
#pragma unroll
      for (int j = NY - 1; j >= 0; --j) {
        Yq[j][0][i] = Yq[j][1][i];
        Yq[j][1][i] = Yq[j][2][i];
      }
#pragma unroll
      for (int j = S - 1; j > 0; --j) Bq[j][i] = Bq[j - 1][i];
      // GO: b and v are pointwise: rows and planes outside the box never
      // reach an in-box cell, so they need no zeroing
      Bq[0][i] = (GO || (bn_ok && rok)) ? BN[i] : (T)0;
      if constexpr (CH) Vc[i] = (GO || (bn_ok && rok)) ? VN[i] : (T)0;
    }
    if (more) exchange(U2, Bq[0], !UZ, true);
    if constexpr (!UZ) gfix(U2, A1, NU - A1);
    // RS: residual of plane zl - S, once the ring holds Y_S up to plane
    // zl - S + 1 (SHY: the exchange's barrier); the slot written next
    // iteration is none of the three it reads
    if constexpr (RS) {
      if (!SHY || !more) __syncthreads();
      resid_plane(zl - S);
    }
    // stores after the wait for the loads above, so that the next
    // iteration's wait does not also wait for these writes; NT: with
    // non-temporal hints
    __builtin_amdgcn_sched_barrier(0);
    {
      const int p = zl - S + 1;
      if (p >= z0 && p < z1) {
#pragma unroll
        for (int i = HY; i < HY + R; ++i)
          if (own(i) && ((rin >> i) & 1u) && (!RS || (w * R + i - HY >= 1 && w * R + i - HY <= TR - 2))) {
            T* dst = (T*)((char*)(out + oo + yoff[i]) + colb(i));
            if constexpr (NT) __builtin_nontemporal_store(YS[i], dst);
            else *dst = YS[i];
          }
      }
      // CH: Y_{S-1} of plane zl - S + 2 (the queue slot it moved to)
      if constexpr (CH && S >= 2) {
        if (p + 1 >= z0 && p + 1 < z1) {
#pragma unroll
          for (int i = HY; i < HY + R; ++i)
            if (own(i) && ((rin >> i) & 1u)) {
              T* dst = (T*)((char*)(out2 + oo2 + yoff[i]) + colb(i));
              if constexpr (NT) __builtin_nontemporal_store(Yq[S - 2][1][i], dst);
              else *dst = Yq[S - 2][1][i];
            }
        }
      }
    }
    oo = next_plane(oo, zl - S + 2);
    if constexpr (CH) oo2 = next_plane(oo2, zl - S + 3);
  }
  if constexpr (RS) {
    // (fine r^2, coarse sum) of the workgroup, reduced through the ring's LDS
    const double t2 = wave_sum_dpp(rs2), t1 = wave_sum_dpp(rs1);
    __syncthreads();
    double* rd = reinterpret_cast<double*>(&ysr[0][0][0]);
    if (lane == 0) {
      rd[2 * w] = t2;
      rd[2 * w + 1] = t1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a2 = 0.0, a1 = 0.0;
#pragma unroll
      for (int q = 0; q < WY; ++q) {
        a2 += rd[2 * q];
        a1 += rd[2 * q + 1];
      }
      part[2 * (size_t)blockIdx.x] = a2;
      part[2 * (size_t)blockIdx.x + 1] = a1;
    }
  } else if (part != nullptr) {
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

}  // namespace rkl
