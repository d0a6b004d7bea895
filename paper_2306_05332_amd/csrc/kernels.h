// Host-side launchers of the gfx950 kernels (see kernels.hip, coarse.hip, fused.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "rkl_device.h"

namespace rkl {

size_t stencil_blocks(int nx, int ny, int nz);  // blocks of the per-stage kernel
size_t resid_blocks(int nx, int ny, int nz);    // partial-sum pairs written by residual-type kernels
size_t ew_block_count(size_t n);                // partial-sum slots used by k_scale / k_sum

// Device-side state of the V-cycle convergence loop.
constexpr int CONV_HIST = 512;
struct ConvState {
  int stop;       // set once the loop has decided to stop; cycle kernels then return at once
  int status;     // rkl_status of the decision (0 = converged)
  int m;          // index of the next cycle-start state to test
  int result_m;   // cycle-start state the decision refers to (the answer)
  int stalled;    // status RKL_ENOCONV came from a stalled residual, not from max_cycles
  int pad_;
  double rel;     // last relative residual
  double mean;    // mean of the last tested residual (diagnostic)
  double last[4]; // last four relative residuals (divergence test)
  double hist[CONV_HIST];
};

template <typename T>
void launch_stage(const LevelView<T>& L, const T* yp, const T* ypp, const T* b, T* yout, double mu,
                  double nu, double c, int first, const int* stop, hipStream_t st);
// transfer.hip: part receives resid_blocks() pairs (sum r^2, sum r | sum of coarse values)
template <typename TU, typename TR>
void launch_residual(const LevelView<TU>& L, const TU* u, const TU* b, TR* r_out, double* part,
                     const int* stop, hipStream_t st, const Batch& bt = single_batch());
// u_out = u + e and r_out = b - M u_out in one pass (float64 u, float32 e;
// 3-D levels, one grid, u_out distinct from u); part as launch_residual
void launch_residual_add(const LevelView<double>& L, const double* u, const float* e, const double* b,
                         double* u_out, float* r_out, double* part, const int* stop, hipStream_t st);
template <typename T>
void launch_resid_restrict(const LevelView<T>& F, const T* u, const T* b, T* bc, double* part,
                           const int* stop, hipStream_t st, const Batch& bt = single_batch());
template <typename T>
void launch_prolong_add(int fnx, int fny, int fnz, int periodic, const T* e, T* fine, const int* stop,
                        hipStream_t st, const Batch& bt = single_batch());
template <typename T>
void launch_restrict(int fnx, int fny, int fnz, const T* fine, T* coarse, hipStream_t st);
void launch_reduce(const double* part, int nblk, int stride, int nq, double* out, const int* stop,
                   hipStream_t st, const Batch& bt = single_batch());
void launch_check(const double* part, int nblk, int stride, const double* res0sq, double tol, int max_cycles,
                  double count, ConvState* cs, hipStream_t st, const Batch& bt = single_batch());
// member m (bt.nb members): out + m * s0 = c * (tab[m] - sum[m * s1] / count)
// (sum nullptr: c * tab[m]); partials as launch_scale's at part + m * part_stride
void launch_scale_tab(const double* const* tab, double* out, size_t n, double c, const double* sum, double count,
                      double* part, hipStream_t st, const Batch& bt);
// launch_sum over the members tab[m] (partials at part + m * part_stride)
void launch_sum_tab(const double* const* tab, size_t n, double* part, hipStream_t st, const Batch& bt);
void launch_copy_tab(double* const* tab, const double* src, size_t n, hipStream_t st, const Batch& bt);
template <typename T>
void launch_fill(T* a, size_t n, T v, const int* stop, hipStream_t st, const Batch& bt = single_batch());
// out = c * (in - sum[0] / count) (sum nullptr: c * in); partials of out and
// out^2 into part[2 blk], part[2 blk + 1] for ew_block_count(n) blocks
void launch_scale(const double* in, double* out, size_t n, double c, const double* sum, double count, double* part,
                  hipStream_t st);
// dst = src - sum[0] / count, dst and src distinct
void launch_copy_sub_mean(double* dst, const double* src, size_t n, const double* sum, double count,
                          hipStream_t st);
template <typename T>
void launch_sub_mean_part(T* a, size_t n, const double* part, int nblk, int stride, int q, double count,
                          const int* stop, hipStream_t st, const Batch& bt = single_batch());
template <typename T>
void launch_sub_mean(T* a, size_t n, const double* sum, double count, const int* stop, hipStream_t st,
                     const Batch& bt = single_batch());
template <typename T>
void launch_sum(const T* a, size_t n, double* part, hipStream_t st,
                const Batch& bt = single_batch());  // ew_block_count(n) partials
// dst = src (distinct arrays) unless *stop is set
template <typename T>
void launch_copy(T* dst, const T* src, size_t n, const int* stop, hipStream_t st);
template <typename TE>
void launch_add_cast(double* u, const TE* e, size_t n, const int* stop, hipStream_t st,
                     const Batch& bt = single_batch());

// Coarsest-grid accelerated RKL solve in one workgroup (coarse.hip).
constexpr int COARSE_MAX_CELLS = 2048;
constexpr int COARSE_MAX_SCHED = 64;   // schedule entries cached in LDS (plans keep within this)
constexpr int COARSE_MAX_COEF = 512;   // stage rows cached in LDS
struct CoarseSchedule {
  const int* sched;     // device: stage count of schedule entry q
  const int* coff;      // device: first coefficient row of entry q
  const double* coef;   // device: rows (mu, nu, c) per stage
  int nsched;
};
template <typename T>
void launch_coarse_solve(const LevelView<T>& L, const T* b, const T* u_in, T* u, CoarseSchedule cs,
                         double tol, double ref_norm, int max_steps, int remove_mean, int* steps_out,
                         double* res_out, const int* stop, hipStream_t st);

// Fused s-stage tau-step, one HBM pass (fused.hip).  Returns false when the
// configuration is not supported (caller falls back to per-stage kernels).
struct StageCoef {
  double mu, nu, c;
};
constexpr int FUSED_MAX_S = 4;
template <typename T>
bool fused_tau_supported(const LevelView<T>& L, int s);
template <typename T>
size_t fused_tau_blocks(const LevelView<T>& L, int s);  // partial sums written when part != nullptr
// u == nullptr: the input iterate is zero
template <typename T>
bool launch_fused_tau(const LevelView<T>& L, const T* u, const T* b, T* out, int s,
                      const StageCoef* co, double* part, const int* stop, hipStream_t st,
                      const Batch& bt = single_batch());
// The fused tau-step of u + P e (prolongation and correction in its input;
// e: the next coarser level's correction, batch stride bt.s1), when the
// level's strip variant supports it; false: the caller prolongs separately.
template <typename T>
bool launch_fused_tau_pro(const LevelView<T>& L, const T* u, const T* e, const T* b, T* out, int s,
                          const StageCoef* co, const int* stop, hipStream_t st, const Batch& bt);
// The fused tau-step of u that also writes the next level's right-hand side
// bc = R(b - M Y_S) (batch stride bt.s1) and, per workgroup, the partial
// pair (sum of fine r^2, sum of coarse values) into part (batch stride
// bt.part_stride); returns the number of pairs written, 0 when the level has
// no such form (nothing launched: the caller relaxes and restricts
// separately).  strip_rs_parts_max bounds the pairs (times 2: doubles).
template <typename T>
int launch_fused_tau_rs(const LevelView<T>& L, const T* u, const T* b, T* out, T* bc, int s, const StageCoef* co,
                        double* part, const int* stop, hipStream_t st, const Batch& bt);
size_t strip_rs_parts_max(int nx, int ny, int nz);

// Stages j0 .. j0 + S - 1 of a longer tau-step in one pass (the strip
// kernel's chunk form): reads Y_{j0-1} = u (stencil), Y_{j0-2} = v
// (pointwise) and b, writes Y_{j0+S-1} to out and, for S >= 2, Y_{j0+S-2} to
// out2; co holds the S stages' coefficients.  tau_chunk_max: the largest S
// the level takes (0: no chunk form: 2-D or small levels).
template <typename T>
int tau_chunk_max(const LevelView<T>& L);
template <typename T>
void launch_tau_chunk(const LevelView<T>& L, const T* u, const T* v, const T* b, T* out, T* out2, int S,
                      const StageCoef* co, hipStream_t st);

// Fused tau-step variants: tile family and shape, plus the workgroup count
// the z-chunk length aims for.  A tuning table keyed by (level shape,
// boundary, precision, s) overrides the built-in choice.
enum : int {
  FV_HEUR = 0,
  FV_RING_64x8 = 1,
  FV_RING_64x4 = 2,
  FV_ZQ_64x32 = 3,
  FV_ZQ_64x16 = 4,
  FV_STRIP_8x4 = 5,   // strip kernel: R = 8 rows per lane, 4 wavefronts per workgroup
  FV_STRIP_8x1 = 6,   // R = 8, one wavefront per workgroup
  FV_STRIP_4x4 = 7,   // R = 4, 4 wavefronts per workgroup
  FV_STRIP2D_8 = 8,   // two-dimensional levels only: 8 x segments per lane, one wavefront per workgroup
  FV_STRIP2D_4 = 9,   // two-dimensional levels only: 4 x segments per lane
  FV_STRIP_5x1 = 10,  // strip kernel: R = 5 rows per lane (3 waves per SIMD in float64), one wavefront per workgroup
  FV_STRIPYX_8x4 = 11,  // R = 8, 4 wavefronts stacked in y sharing their halo rows through LDS
  FV_STRIPYX_4x8 = 12,  // R = 4, 8 wavefronts stacked in y sharing their halo rows through LDS
  FV_STRIPYX_8x8 = 13,  // R = 8, 8 wavefronts stacked in y sharing their halo rows through LDS
  FV_STRIPYX_2x8 = 14,  // R = 2, 8 wavefronts stacked in y sharing their halo rows through LDS
  FV_STRIPYX_2x16 = 15, // R = 2, 16 wavefronts stacked in y sharing their halo rows through LDS
  FV_COUNT = 16
};
// A two-dimensional level (nz = 1, ihz2 = 0) takes the FV_STRIP2D_* variants
// and no others; a 3-D level takes every variant but those.
inline bool variant_is_2d(int variant) { return variant == FV_STRIP2D_8 || variant == FV_STRIP2D_4; }
template <typename T>
inline bool level_is_2d(const LevelView<T>& L) { return L.nz == 1 && L.ihz2 == (T)0; }
struct FusedChoice {
  int variant;
  int target;
};
template <typename T>
bool fused_variant_ok(int variant, int s);
template <typename T>
FusedChoice fused_choice(const LevelView<T>& L, int s);
template <typename T>
size_t fused_tau_blocks_as(const LevelView<T>& L, FusedChoice c, int s);
// workgroups per z chunk of a strip variant on this level (0: not a strip
// variant); a target of per * c gives c chunks
template <typename T>
int fused_chunk_blocks(const LevelView<T>& L, int variant, int s);
template <typename T>
bool launch_fused_tau_as(const LevelView<T>& L, FusedChoice c, const T* u, const T* b, T* out, int s,
                         const StageCoef* co, double* part, const int* stop, hipStream_t st,
                         const Batch& bt = single_batch());
size_t fused_tau_blocks_max(int nx, int ny, int nz);  // over every variant and target

// Strip form of the fused tau-step (strip.hip): one wavefront per 64-column x
// strip of R = 8 or 4 rows, 4 or 1 wavefronts per workgroup stacked in y.
// The 2-D form marches y with R x segments per lane (flat = true: nx, ny, nz
// describe the transposed view, ny = 1 and nz = the 2-D row count).
// Workgroup layout of the strip kernel.  Three-dimensional one-wavefront
// variants pack the x remainder: when nx = txf * ox + rem, the remainder
// column block of pk interior strips (no row of them wraps or leaves the box)
// shares one wavefront, pk segments of rem + 2 s lanes side by side.  Per z
// chunk the workgroups are then: txf * gy full tiles, npk packed wavefronts
// (strips fi + k pk .. fi + k pk + pk - 1), and one remainder wavefront for each
// strip left over (strips below fi and from fi + npk pk on).  pk = 0: no packing
// (tiles tx = 0 .. gx - 1 over every strip).
struct StripMap {
  int txf, pk, npk, fi, per;
};
struct StripGrid {
  int ox, gx, gy, zc, gz, nblk;
  int per;  // workgroups per z chunk (nblk = per * gz)
  StripMap map;
};
StripGrid strip_grid(int s, int R, int WY, int nx, int ny, int nz, int target, bool flat = false, bool pack = true);
template <typename T, int S, int R, int WY>
void launch_strip(const LevelView<T>& L, int target, const T* u, const T* b, T* out, const FCoef<T, S>& fc,
                  double* part, const int* stop, const Batch& bt, hipStream_t st);
// WY > 1 wavefronts stacked in y that share their halo rows through LDS
template <typename T, int S, int R, int WY>
void launch_strip_yx(const LevelView<T>& L, int target, const T* u, const T* b, T* out, const FCoef<T, S>& fc,
                     double* part, const int* stop, const Batch& bt, hipStream_t st);
template <typename T, int S, int R, int WY>
void launch_strip2d(const LevelView<T>& L, int target, const T* u, const T* b, T* out, const FCoef<T, S>& fc,
                    double* part, const int* stop, const Batch& bt, hipStream_t st);
// The strip tau-step with prolongation and correction fused into its input
// (Sec. 2.1: the first post-smoothing relaxation of u + P e): reads u, the
// coarse correction e (batch stride bt.s1) and b, writes Y_S to out; u is not
// modified.  3-D levels of even extents, even R; no remainder packing.
// target <= 0 sizes the z chunks to one wave of resident workgroups.
template <typename T, int S, int R, int WY, bool SHY>
void launch_strip_pro(const LevelView<T>& L, int target, const T* u, const T* e, const T* b, T* out,
                      const FCoef<T, S>& fc, const int* stop, const Batch& bt, hipStream_t st);
template <typename T, int S, int R, int WY>
void launch_strip_ch(const LevelView<T>& L, int target, const T* u, const T* v, const T* b, T* out, T* out2,
                     const FCoef<T, S>& fc, const Batch& bt, hipStream_t st);
// The strip tau-step with the residual + restriction of its result fused in
// (strip_rs.hip); returns the workgroup count (partial pairs written).
// Stacked strips of R WY - 2 >= RS_MIN_ROWS output rows, even extents.
constexpr int RS_MIN_ROWS = 14;
StripGrid strip_grid_rs(int s, int R, int WY, int nx, int ny, int nz, int target);
template <typename T, int S, int R, int WY, bool SHY>
int launch_strip_rs(const LevelView<T>& L, int target, const T* u, const T* b, T* out, T* bc, const FCoef<T, S>& fc,
                    double* part, const int* stop, const Batch& bt, hipStream_t st);
template <typename T, int R, int WY, bool FLAT>
void launch_strip_gsrb(const LevelView<T>& L, int target, const T* u, const T* b, T* out, double omega_over_d,
                       double* part, const int* stop, const Batch& bt, hipStream_t st);

// One red-black Gauss-Seidel (omega = 1) or SOR iteration on M u = b
// (Sec. 2.2.4; App. B): red cells ((i + j + k) even) from the old values,
// then black cells from the new red values, u += (omega / D)(M u - b) with
// D = 2 sum h^-2, Dirichlet ghosts from the current values.  Out of place in
// one HBM pass when the level takes the strip kernel (returns true; u ==
// nullptr reads a zero iterate; part as for the fused tau-step), else false.
template <typename T>
bool launch_gsrb_fused(const LevelView<T>& L, const T* u, const T* b, T* out, double omega, double* part,
                       const int* stop, hipStream_t st, const Batch& bt = single_batch());
template <typename T>
size_t gsrb_blocks(const LevelView<T>& L);  // partial sums written by launch_gsrb_fused
// One colour per launch, any level size: uout = uin with the cells of
// `colour` updated from uin (two launches make one iteration).
template <typename T>
void launch_gsrb_half(const LevelView<T>& L, const T* uin, T* uout, const T* b, int colour, double omega,
                      const int* stop, hipStream_t st, const Batch& bt = single_batch());
// dst = src - sum over the Dirichlet faces of a cell of 2 g h_d^-2: after this
// the finest level needs only the homogeneous ghost -u (dst may be src).
void launch_fold_faces(int nx, int ny, int nz, double hx, double hy, double hz, const double* faces,
                       const double* src, double* dst, hipStream_t st);
// g = -grad(phi) by 4th-order differences (Sec. 3, eq. 4thorder_acceleration);
// Dirichlet second ghost layer by odd reflection about the face value.
void launch_gradient(int nx, int ny, int nz, double hx, double hy, double hz, int periodic, const double* faces,
                     const double* phi, double* gx, double* gy, double* gz, hipStream_t st);
// max |M u - b| over the level: per-block maxima in part, reduced into out[0]
template <typename T>
void launch_resid_absmax(const LevelView<T>& L, const T* u, const T* b, double* part, double* out, hipStream_t st);
void tune_install(int nx, int ny, int nz, int periodic, int dbl, int s, FusedChoice c);  // FV_HEUR erases
void tune_clear();
int tune_generation();
const char* fused_variant_name(int variant);

// Coarse tail of the V-cycle in one workgroup (tail.hip).
constexpr int TAIL_MAX_LEVELS = 6;
constexpr int TAIL_MAX_S = 8;
constexpr int TAIL_MAX_CELLS = 4096;          // cells of the top tail level
constexpr size_t TAIL_MAX_LDS = 144 * 1024;   // dynamic LDS for the tail arrays (static LDS: ~13 KB)
struct TailShape {
  int nlev;
  int nx[TAIL_MAX_LEVELS], ny[TAIL_MAX_LEVELS], nz[TAIL_MAX_LEVELS];
  double ihx2[TAIL_MAX_LEVELS], ihy2[TAIL_MAX_LEVELS], ihz2[TAIL_MAX_LEVELS];
};
template <typename T>
bool tail_fits(const TailShape& ts, int s);
// b_top: restricted right-hand side of the top tail level (mean not yet
// removed); u_top receives that level's correction.  smooth[l]: the s stage
// coefficients of tail level l.
void tail_prepare();
template <typename T>
void launch_tail(const TailShape& ts, const StageCoef* const* smooth, int s, int n_pre, int n_post, int periodic,
                 CoarseSchedule cs, double ctol, int cmax, const T* b_top, T* u_top, const int* stop,
                 hipStream_t st, const Batch& bt = single_batch(), int gs = 0);

}  // namespace rkl
