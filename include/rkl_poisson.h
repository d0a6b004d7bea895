/*
 * rkl_poisson.h -- C ABI of the MI355X (gfx950) RKL-multigrid Poisson solver.
 *
 * Solves  nabla^2 phi = 4 pi G rho  on a cell-centred box with the 7-point
 * Laplacian (Mandal, Mukherjee & Mignone 2023, "A self-gravity module for the
 * PLUTO code": Sec. 2.2.1 eq. discrete_laplace_3D), Dirichlet or periodic
 * boundaries (Sec. 2.3, eqs. solution_ghost, error_ghost, periodic), by a
 * correction-scheme multigrid V-cycle (Sec. 2.1) whose relaxation and
 * coarsest-grid solver are Runge-Kutta-Legendre super-time-steps of the
 * parabolic problem d phi/dt = nabla^2 phi - 4 pi G rho (Sec. 2.2.4,
 * App. A eq. RKL_intermediate_source).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Arrays are dense, row-major [k][j][i] with x fastest, nx*ny*nz elements.
 * - Pointers named "device" are HIP device (or managed) memory owned by the
 *   caller; "host" pointers are ordinary CPU memory owned by the caller.  The
 *   library never frees caller memory.  Work buffers are owned by the library
 *   in a plan cache keyed by (device, grid, options); rkl_release_all() frees
 *   them.
 * - Every call is ordered on the HIP stream passed as `hip_stream`
 *   (a hipStream_t; NULL = the default stream).  Calls that report a
 *   residual synchronise that stream to read it.
 * - Dirichlet boundary data `bc_faces` (device, float64) holds the boundary
 *   values at face centres, packed as
 *       x- (ny*nz, [k][j]), x+ (ny*nz), y- (nx*nz, [k][i]), y+ (nx*nz),
 *       z- (nx*ny, [j][i]), z+ (nx*ny);
 *   NULL means homogeneous data (g = 0).  It must be NULL for periodic grids.
 * - Errors are returned as rkl_status; nothing aborts or throws across the
 *   ABI.  rkl_last_error() gives a thread-local message for the last failure.
 *   On a failure after work started, phi holds the last complete iterate.
 * - Calls from several host threads are allowed; calls that share a plan
 *   (same device, grid and options) on different streams must not overlap.
 */
#ifndef RKL_POISSON_H
#define RKL_POISSON_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RKL_OK = 0,
    RKL_EINVAL = -1,      /* bad argument (sizes, spacing, options, NULL pointer) */
    RKL_ENOMEM = -2,      /* device allocation failed                             */
    RKL_ENOCONV = -3,     /* max_cycles reached before tol, or the residual       */
                          /* stalled above tol > 0 (no 10% gain in 8 cycles: tol  */
                          /* below the float64 rounding floor of M phi - f)       */
    RKL_EDIVERGED = -4,   /* residual grew in 3 consecutive cycles, to over       */
                          /* twice its best value                                 */
    RKL_ENONFINITE = -5,  /* NaN or Inf in the source or the residual             */
    RKL_EHIP = -6         /* a HIP runtime call failed                            */
} rkl_status;

typedef enum { RKL_BC_DIRICHLET = 0, RKL_BC_PERIODIC = 1 } rkl_bc;

typedef enum {
    RKL_FP64 = 0,   /* every sweep, transfer and norm in float64                    */
    RKL_MIXED = 1   /* float32 V-cycles inside a float64 defect-correction loop     */
} rkl_precision;

/* Finest-level geometry: active cell counts and spacings (Sec. 2.2.1).
 * Two dimensions: nz = 1 with hz = +infinity (HUGE_VAL).  Every z term of the
 * operator then carries 1/hz^2 = 0, which leaves the 5-point Laplacian of
 * eq. discrete_laplace_2D; the hierarchy halves x and y only, restriction
 * averages 4 children (eq. restriction_example_2D) and prolongation weighs
 * (9,3,3,1)/16 (eq. prolongation_example_2D).  Dirichlet face arrays keep
 * the six-face layout; the two z faces (ny*nx values each) carry no weight.
 * hz = inf with nz != 1 is RKL_EINVAL. */
typedef struct {
    int nx, ny, nz;
    double hx, hy, hz;
    int bc;            /* rkl_bc */
} rkl_grid;

/* V-cycle relaxation.  RKL_SMOOTH_RKL: one s-stage RKL tau-step per
 * relaxation (App. A eq. RKL_intermediate_source).  RKL_SMOOTH_GSRB: one
 * red-black Gauss-Seidel pass per relaxation, the paper's own smoother
 * (Sec. 2.2.4); the coarsest level is always solved by accelerated RKL. */
typedef enum { RKL_SMOOTH_RKL = 0, RKL_SMOOTH_GSRB = 1 } rkl_smoother;

/* Solver options.  rkl_default_opts() fills the defaults noted here. */
typedef struct {
    int s;               /* stages per smoothing tau-step (default 2; 0: the tuned stage count  */
                         /* of rkl_tune_set_s for the grid, else 2)                             */
    double tau_frac;     /* theta = tau / tau_max(s), in (0, 1] (default 0.9); tau_max from
                            eq. tau_max with |lambda_max| = 4 sum_d h_d^-2                        */
    int n_pre, n_post;   /* relaxations before / after the coarse correction (2, 1; Sec. 4.1)  */
    int min_coarse;      /* coarsen while every n/2 is even and >= min_coarse (default 4)      */
    double tol;          /* stop at ||M phi - f||_2 / ||M 0 - f||_2 <= tol (default 1e-10);     */
                         /* 0 runs exactly max_cycles cycles                                    */
    int max_cycles;      /* cap on V-cycles (outer iterations in RKL_MIXED) (default 100)       */
    int prec;            /* rkl_precision (default RKL_FP64)                                    */
    double four_pi_G;    /* f = four_pi_G * rho (default 4 pi, i.e. G = 1)                      */
    double coarse_tol;   /* coarsest solve: stop at ||M u - b|| <= coarse_tol ||b||; 0 picks
                            1e-13 (float64) or 1e-6 (float32)                                   */
    int coarse_max_steps;/* coarsest solve: cap on tau-steps (default 200)                      */
    int smoother;        /* rkl_smoother: relaxation of the V-cycle above the coarsest level    */
                         /* (default RKL_SMOOTH_RKL)                                            */
    int fuse;            /* transfer fusion on levels whose tau-step runs the strip kernel      */
                         /* (same arithmetic, one HBM pass less each), a bit mask:              */
                         /* bit 0: the prolongation + correction of Sec. 2.1 runs inside the    */
                         /* first post-smoothing tau-step; bit 1: the last pre-smoothing        */
                         /* tau-step also writes the restricted residual (steps 2a-2b).         */
                         /* 3 (default): both; 0: separate transfer kernels; other values:      */
                         /* RKL_EINVAL                                                          */
    int zero_start;      /* rkl_poisson_solve: 1 starts from phi = 0 whatever phi holds on      */
                         /* entry (a cold start: phi need not be initialised, and the first     */
                         /* relaxation reads no iterate); 0 (default) starts from phi's         */
                         /* contents; other values: RKL_EINVAL                                  */
} rkl_opts;

/* Solve statistics.  `history` (host, optional) receives the relative
 * residual before each cycle, up to history_cap entries. */
typedef struct {
    int cycles;          /* V-cycles (or outer refinements) performed                 */
    int levels;          /* multigrid levels used (1 = single-level RKL mode)         */
    double res0;         /* ||M 0 - f||_2                                             */
    double rel_res;      /* final ||M phi - f||_2 / res0                              */
    double *history;     /* host array or NULL                                        */
    int history_cap;
    int history_len;
    int status;          /* this solve's rkl_status (per member in batched calls)     */
} rkl_stats;

/* Fill `o` with the defaults listed in rkl_opts. */
void rkl_default_opts(rkl_opts *o);

/*
 * Full solve of nabla^2 phi = 4 pi G rho (eq. poisson_eqaution) to relative
 * residual opts->tol, by V-cycles from the initial guess in phi (zeros for a
 * cold start).  Sec. 2.1 (V-cycle), Sec. 4.1 (N_pre, N_post, stop metric).
 *   grid      host, finest-level geometry
 *   opts      host, may be NULL for defaults
 *   rho       device float64[nz*ny*nx], not modified
 *   bc_faces  device float64 packed faces (Dirichlet) or NULL
 *   phi       device float64[nz*ny*nx]: initial guess in, solution out;
 *             periodic solutions are returned with zero mean (the mean of
 *             rho is removed first, eq. source_modification)
 *   stats     host, optional
 * A grid that cannot be coarsened runs the accelerated single-level RKL
 * iteration of App. A.4 to tolerance (stats->levels == 1), in float64 for
 * either precision.
 */
rkl_status rkl_poisson_solve(const rkl_grid *grid, const rkl_opts *opts,
                             const double *rho, const double *bc_faces,
                             double *phi, rkl_stats *stats, void *hip_stream);

/*
 * One V-cycle (Sec. 2.1) on M phi = f at float64: f is the final right-hand
 * side (already 4 pi G rho, mean-free if periodic) and is used as given.
 *   f, phi      device float64[nz*ny*nx]; phi updated in place
 *   rel_res_out host, optional: ||M phi - f|| / ||M 0 - f|| after the cycle
 */
rkl_status mg_vcycle(const rkl_grid *grid, const rkl_opts *opts, const double *f,
                     const double *bc_faces, double *phi, double *rel_res_out,
                     void *hip_stream);

/*
 * n_steps RKL tau-steps of s stages on M phi = f at the finest level
 * (App. A eq. RKL_intermediate_source, tau = tau_frac * tau_max(s),
 * eq. tau_max).  f is used as given (no mean removal).  This is also the
 * single-level relaxation of App. B when n_steps is large.
 *   f, phi  device float64[nz*ny*nx]; phi updated in place
 */
rkl_status rkl_smooth(const rkl_grid *grid, int s, double tau_frac, int n_steps,
                      const double *f, const double *bc_faces, double *phi,
                      void *hip_stream);

/*
 * Residual r = f - M phi on the finest level (Sec. 2.1 eq. residual, with the
 * opposite sign) and its float64 L2 norm.
 *   r_out     device float64[n] or NULL (norm only)
 *   norm_out  host, optional
 */
rkl_status rkl_residual(const rkl_grid *grid, const double *f, const double *bc_faces,
                        const double *phi, double *r_out, double *norm_out,
                        void *hip_stream);

/*
 * Grid transfer building blocks of the V-cycle (float64, device arrays).
 * rkl_restrict: coarse = R(fine), the 8-point average of eq.
 *   restriction_example_3D; `grid` describes the FINE grid (even sizes).
 * rkl_prolong_add: fine += P(coarse) with the (27,9,9,9,3,3,3,1)/64 weights of
 *   eq. prolongation_example_3D and error-equation ghosts on the coarse grid
 *   (homogeneous Dirichlet or periodic, Sec. 2.3); `grid` describes the FINE grid.
 * On a two-dimensional grid (nz = 1, hz = inf) they are the 4-point average and
 * the (9,3,3,1)/16 weights of eqs. restriction_example_2D and
 * prolongation_example_2D, and the coarse grid has nz = 1 as well.
 */
rkl_status rkl_restrict(const rkl_grid *grid, const double *fine, double *coarse,
                        void *hip_stream);
rkl_status rkl_prolong_add(const rkl_grid *grid, const double *coarse, double *fine,
                           void *hip_stream);

/*
 * Coarsest-grid solve (App. A.4, accelerated RKL schedule) of M u = b with
 * homogeneous (Dirichlet) or periodic ghosts, from u = 0, until
 * ||M u - b|| <= coarse_tol ||b|| or coarse_max_steps tau-steps.
 *   b, u        device float64[n]
 *   steps_out   host, optional: tau-steps taken
 * Uses one workgroup with the level held in LDS when n <= 2048 cells.
 */
rkl_status rkl_coarse_solve(const rkl_grid *grid, const rkl_opts *opts, const double *b,
                            double *u, int *steps_out, void *hip_stream);

/*
 * Float32 twins of the level building blocks above: the kernels that the
 * RKL_MIXED path runs on the correction equation M e = r inside its float64
 * defect correction (the V-cycle of Sec. 2.1 with the RKL tau-steps of App. A
 * eq. RKL_intermediate_source, the transfers of eqs. restriction_example_3D and
 * prolongation_example_3D, the accelerated coarsest solve of App. A.4).  They
 * take the error equation's ghosts on every level: homogeneous Dirichlet
 * (ghost = -u, eq. error_ghost) or periodic wrap (eq. periodic); there is no
 * face-data argument.  Arrays are device float32[n] in the common layout; the
 * arithmetic is float32, norms and their partial sums float64.  Arguments,
 * errors and stream semantics are those of the float64 forms:
 *   rkl_smooth_f32       = rkl_smooth with bc_faces = NULL
 *   mg_vcycle_f32        = mg_vcycle with bc_faces = NULL (opts->prec is
 *                          ignored); rel_res_out: ||M phi - f|| / ||f||
 *   rkl_residual_f32     r = f - M phi (float32), ||r||_2 accumulated in float64
 *   rkl_restrict_f32, rkl_prolong_add_f32, rkl_coarse_solve_f32: as above
 *                          (coarse_tol 0 picks 1e-6 for float32)
 */
rkl_status rkl_smooth_f32(const rkl_grid *grid, int s, double tau_frac, int n_steps,
                          const float *f, float *phi, void *hip_stream);
rkl_status mg_vcycle_f32(const rkl_grid *grid, const rkl_opts *opts, const float *f, float *phi,
                         double *rel_res_out, void *hip_stream);
rkl_status rkl_residual_f32(const rkl_grid *grid, const float *f, const float *phi, float *r_out,
                            double *norm_out, void *hip_stream);
rkl_status rkl_restrict_f32(const rkl_grid *grid, const float *fine, float *coarse, void *hip_stream);
rkl_status rkl_prolong_add_f32(const rkl_grid *grid, const float *coarse, float *fine, void *hip_stream);
rkl_status rkl_coarse_solve_f32(const rkl_grid *grid, const rkl_opts *opts, const float *b, float *u,
                                int *steps_out, void *hip_stream);

/*
 * Batched solve of `nbatch` independent problems M phi_i = 4 pi G rho_i
 * (same equations, options and stopping rule as rkl_poisson_solve, Sec. 2.2
 * and 2.4; Dirichlet members take homogeneous faces).
 *   grids   host array of nbatch grids; sizes and boundary types may differ
 *   rho     host array of nbatch device pointers, float64[grid i's n] each
 *   phi     host array of nbatch device pointers (outputs, owned by caller)
 *   stats   host array of nbatch entries or NULL; each entry's history
 *           buffer (if any) receives that member's residual history
 * Members with identical grids form a class held in contiguous library-owned
 * buffers; every phase of a class's V-cycle is one launch over all members,
 * and each member has its own device-side convergence state, so converged
 * members drop out while the others continue.  The refinement loop
 * (float64 defect, V-cycle on the correction at the working precision,
 * float64 update) is captured once into a HIP graph and replayed until every
 * member has stopped.  A class whose hierarchy does not end in the
 * one-workgroup coarse tail is solved member by member with the single-solve
 * path.  Returns the first non-OK member status in class order (each member's
 * own outcome is in stats[i]); phi of periodic members is mean-free.  Calls
 * on one process are serialised.  Buffers persist until rkl_release_all.
 */
rkl_status rkl_poisson_solve_batched(const rkl_grid *grids, int nbatch, const rkl_opts *opts,
                                     const double *const *rho, double *const *phi,
                                     rkl_stats *stats, void *hip_stream);

/*
 * Number of kernel launches one finest-level tau-step of s stages takes on
 * this grid (1 when the fused single-pass tau-step kernel handles it, s when
 * it runs stage by stage), for precision prec (rkl_precision; RKL_MIXED
 * reports the float32 sweep).  Lets callers turn kernel timings into
 * bytes per launch.  Returns RKL_EINVAL (< 0) on bad arguments.
 */
int rkl_tau_step_launches(const rkl_grid *grid, int s, int prec);

/*
 * Tile tuning of the fused tau-step (the smoother of Sec. 2.2.3 run as one
 * HBM pass per tau-step).  A variant is a tile family and shape; `target` is
 * the workgroup count the z-chunking aims for.  Variants compute identical
 * values cell by cell; only the order of the float64 norm partials differs.
 * Three-dimensional one-wavefront strip variants (6 and 10) give the x
 * remainder of several interior strips to one shared wavefront, so their
 * workgroup count per z chunk is below tiles x strips.
 *   variant 0  built-in choice (in rkl_tune_set: erase the entry)
 *           1  LDS ring, 64 x 8 tiles        2  LDS ring, 64 x 4 tiles
 *           3  z-queue, 64 x 32 tiles        4  z-queue, 64 x 16 tiles
 *              (z-queue: s = 2 or 3 only)
 *           5  strip, 4 wavefronts of 64 columns x 8 rows per workgroup
 *           6  strip, 1 wavefront of 64 columns x 8 rows per workgroup
 *           7  strip, 4 wavefronts of 64 columns x 4 rows per workgroup
 *           8  2-D strip, 1 wavefront per workgroup, 8 segments of 64 columns
 *              per lane, marching in y
 *           9  2-D strip, as 8 with 4 segments per lane
 *          10  strip, 1 wavefront of 64 columns x 5 rows per workgroup
 *          11  strip, 4 wavefronts of 64 columns x 8 rows stacked in y, which
 *              take the halo rows they share from each other through LDS
 *              (u and b rows read once per workgroup instead of per wavefront)
 *          12  as 11 with 8 wavefronts of 4 rows
 *          13  as 11 with 8 wavefronts of 8 rows
 *          14  as 11 with 8 wavefronts of 2 rows (s <= 2)
 *          15  as 11 with 16 wavefronts of 2 rows (s <= 2)
 *          13  as 11 with 8 wavefronts of 8 rows
 *              (strip: s <= 2 in float64, s <= 3 in float32; variants 8 and 9
 *              are for two-dimensional levels, nz = 1 with hz = inf, and
 *              those levels take no other variant)
 * Entries are keyed by (nx, ny, nz, bc, prec, s) of one multigrid LEVEL
 * (prec RKL_FP64: float64 sweeps; RKL_MIXED: the float32 sweeps of the
 * mixed path) and take effect at the next solve.  The table is per process.
 */
typedef struct {
    int nx, ny, nz;      /* level shape                                      */
    int bc;              /* rkl_bc                                           */
    int prec;            /* rkl_precision                                    */
    int s;               /* stages per tau-step                              */
    int variant;         /* see above                                        */
    int target;          /* workgroups aimed for (>= 1)                      */
    double us;           /* rkl_autotune: mean launch time in microseconds   */
} rkl_tune_entry;

/* Install n entries (host array).  RKL_EINVAL for a malformed entry, a
 * variant not built for that (s, prec), or a 2-D variant on an entry with
 * nz != 1 (or a 3-D one with nz = 1); then nothing is installed. */
rkl_status rkl_tune_set(const rkl_tune_entry *entries, int n);
/* Drop every tile entry and every stage-count entry. */
rkl_status rkl_tune_clear(void);
/* The choice in effect for a level (variant 0 if no fused tau-step applies). */
rkl_status rkl_tune_get(const rkl_grid *level, int s, int prec, rkl_tune_entry *out);
/*
 * Time every variant and target on one level shape: reps launches each on
 * library-allocated scratch (freed before return), HIP events on hip_stream.
 * Targets: a fixed set from 64 to 4096 workgroups, and for strip variants
 * also one per distinct z-chunk length from 64 planes (2-D: rows) down to 1.
 * Installs the fastest; writes up to cap results sorted by time (host array)
 * and the number measured to *n_results.  Synchronises the stream.
 */
rkl_status rkl_autotune(const rkl_grid *level, int s, int prec, int reps, rkl_tune_entry *results,
                        int cap, int *n_results, void *hip_stream);
/* Stage count used when opts->s == 0 for this grid and precision (a timed
 * choice; without an entry s = 2).  s = 0 erases the entry. */
rkl_status rkl_tune_set_s(const rkl_grid *grid, int prec, int s);
/* Multigrid level shapes of `grid` (coarsening by 2 while every n/2 is an
 * even integer >= min_coarse, Sec. 2.2.2): returns the level count L (or a
 * negative rkl_status) and writes up to cap (nx, ny, nz) triples to nxyz. */
int rkl_level_shapes(const rkl_grid *grid, int min_coarse, int *nxyz, int cap);
/* Name of a variant ("ring64x8", ...; "heuristic" for 0 or unknown). */
const char *rkl_variant_name(int variant);

/*
 * n_iter red-black Gauss-Seidel iterations (omega = 1) or SOR iterations
 * (omega in (0, 2)) on M phi = f at one level (Sec. 2.2.4; App. B): red cells
 * ((i + j + k) even) from the old values, then black cells from the new red
 * values, each u += (omega / D_cell)(M u - f) with D_cell the operator's own
 * diagonal (2 sum h^-2, plus h_d^-2 for each Dirichlet face of the cell, whose
 * ghost is 2 g - u, or -u with bc_faces NULL), so omega = 1 solves each
 * cell's row exactly (the Jacobi splitting behind App. B's omega).
 * f, phi: device float64[n]; phi is updated in place.
 */
rkl_status rkl_gsrb_smooth(const rkl_grid *grid, double omega, int n_iter, const double *f,
                           const double *bc_faces, double *phi, void *hip_stream);

/*
 * Single-level relaxation of M phi = f to a maximum residual (App. B: the
 * comparison of RKL, Gauss-Seidel and SOR without multigrid).
 */
typedef enum { RKL_RELAX_RKL = 0, RKL_RELAX_GSRB = 1, RKL_RELAX_SOR = 2 } rkl_relax_method;
typedef struct {
    int method;          /* rkl_relax_method                                                  */
    int s;               /* RKL: 0 = accelerated schedule of App. A.4, > 0 = fixed stage count, */
                         /* -1 = the fixed count of App. A.3 (rkl_s_opt with kmax 6, digits 2) */
    double tau_frac;     /* RKL: theta = tau / tau_max (default 0.9)                          */
    double omega;        /* SOR: over-relaxation; 0 = App. B optimum 2/(1 + sqrt(1 - rho_J^2)),
                            rho_J = sum cos(pi/n_d) h_d^-2 / sum h_d^-2 (default 0)           */
    double tol_max;      /* stop when max |M phi - f| <= tol_max (default 1e-10)              */
    int max_iters;       /* cap on iterations: tau-steps or GS / SOR passes (default 100000)  */
    int check_every;     /* iterations between residual tests (default 1)                     */
} rkl_relax_opts;
void rkl_default_relax_opts(rkl_relax_opts *o);
/*
 * phi: device float64[n], initial guess in, result out; periodic grids have
 * the mean of phi removed after every iteration (f must be mean-free).
 * stats (optional): cycles = iterations, res0 = first tested residual,
 * rel_res = last tested max |M phi - f| (absolute), history = tested residuals,
 * status = RKL_OK, RKL_ENOCONV (max_iters) or RKL_ENONFINITE.
 */
rkl_status rkl_relax_solve(const rkl_grid *grid, const rkl_relax_opts *opts, const double *f,
                           const double *bc_faces, double *phi, rkl_stats *stats, void *hip_stream);

/*
 * Best fixed stage count of App. A.3 (eq. sopt_theory) for single-level RKL
 * relaxation on `grid` at tau = tau_frac * tau_max(s).  Mode k = 1 .. kmax
 * (bounded by n/2, n the smallest cell count) of the smoothest family --
 * Dirichlet: the diagonal mode (k,k,k), |lambda_k| = sum_d 4 sin^2(k pi /
 * 2 n_d) / h_d^2; periodic: the axis mode of least |lambda_k| =
 * min_d 4 sin^2(k pi / n_d) / h_d^2 -- is damped per tau-step by P_s(x_k),
 * x_k = 1 - tau_frac Delta t_par |lambda_k|, Delta t_par = 2 / (4 sum_d h_d^-2)
 * (eqs. eigenvalue_RKL, tau_max); rho(s) = max_k |P_s(x_k)| (eq.
 * spectral_rad_RKL); m_eff(s) = s * digits / (-log10 rho(s)) stages buy
 * `digits` orders of residual reduction (eq. iteration).  Returns the s in
 * [1, largest cell count] minimising m_eff (the first one on ties) or a
 * negative rkl_status; *m_eff_out (host, optional) receives m_eff(s_opt).
 * The paper's setting is kmax = 6, digits = 2: a cubic Dirichlet grid of N
 * cells per side at tau_frac = 1 has x_k = cos(k pi / N), the paper's 1-D
 * model, and N = 64 gives 56.  Host-only arithmetic (no GPU work).
 */
int rkl_s_opt(const rkl_grid *grid, double tau_frac, int kmax, double digits, double *m_eff_out);

/*
 * Gravitational acceleration g = -grad(phi) by the 4th-order differences of
 * Sec. 3 (eq. 4thorder_acceleration), e.g.
 *   g_x = -(4/3)(phi_{i+1} - phi_{i-1})/(2 dx) + (1/3)(phi_{i+2} - phi_{i-2})/(4 dx).
 * Two ghost layers: periodic wrap; Dirichlet odd reflection about the face
 * values of phi (phi_{-m} = 2 g - phi_{m-1}, m = 1, 2; bc_faces NULL: g = 0),
 * which needs every Dirichlet extent >= 2.  A two-dimensional grid (nz = 1,
 * hz = inf) gets gz = 0.
 *   phi        device float64[n]
 *   gx, gy, gz device float64[n] outputs (caller-owned)
 */
rkl_status rkl_gradient(const rkl_grid *grid, const double *phi, const double *bc_faces, double *gx,
                        double *gy, double *gz, void *hip_stream);

/*
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the residual
 * of rkl_residual without any allocation and without synchronising.
 *   r_out     device float64[n] or NULL: f - M phi, with the Dirichlet face
 *             data of bc_faces applied in the stencil (ghost 2 g - u); the
 *             values equal rkl_residual's (which folds the face data into a
 *             copy of f first) up to rounding, and bit for bit without faces
 *   norm_dev  DEVICE double or NULL: receives ||f - M phi||_2, computed on the
 *             GPU (stream-ordered; read it after synchronising the stream)
 * Other arguments as rkl_residual.  The workgroups' partial sums go to a fixed
 * 1 MiB array inside the library, one per GPU, held until the process ends;
 * a grid whose residual needs more than 65536 partial-sum pairs (3-D: beyond
 * about 1024^3 cells) is RKL_EINVAL, before any GPU work.  Every call on a GPU
 * uses that GPU's one array: calls that overlap in time on one GPU (other
 * streams or host threads) race and must be serialised by the caller.
 */
rkl_status rkl_residual_noalloc(const rkl_grid *grid, const double *f, const double *bc_faces,
                                const double *phi, double *r_out, double *norm_dev, void *hip_stream);

/* Thread-local message describing the last failure (never NULL). */
const char *rkl_last_error(void);

/* Free every cached plan and work buffer on every device. */
void rkl_release_all(void);

#ifdef __cplusplus
}
#endif

#endif /* RKL_POISSON_H */
