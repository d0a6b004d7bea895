"""CPU oracle for the RKL-multigrid Poisson solver -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct float64 numpy implementation of what the GPU
path computes, written from the paper (Mandal, Mukherjee & Mignone, "A
self-gravity module for the PLUTO code", ApJS 2023) and nothing else.  Only the
test-suite, the smoke check and the benchmark's CPU-baseline leg may import
it.  It shares no code with the GPU package and never imports it; the only
shared module is ``workloads`` (seeded input generators, no solver arithmetic).

Modules
-------
operators  cell-centred grid hierarchy, ghost cells, 7-point Laplacian,
           residual, 8-point restriction, 27/9/3/1 prolongation (Sec. 2.2, 2.3)
rkl        RKL1 coefficients and one s-stage tau-step with source (App. A,
           eq. RKL_intermediate_source), stability limit (eq. tau_max),
           spectral rules for s (eqs. spectral_rad_RKL, sopt_theory,
           sk_optimal) and the accelerated schedule (App. A.4)
multigrid  coarsest-grid RKL solve, correction-scheme V-cycle (Sec. 2.1),
           outer convergence loop, single-level RKL mode, mixed-precision
           defect correction, adjoint solve
exact      the exact discrete solution u* by independent routes: FFT with
           the discrete symbol (periodic), DST-II (Dirichlet), dense solve
smoothers  the paper's own GS-RB smoother and the single-level Jacobi / GS /
           SOR comparison iterations (Sec. 2.2.4, App. B)
gradient   4th-order finite-difference acceleration (eq. 4thorder_acceleration)

Every function is pinned by a CPU test against something other than itself
(closed forms, library routines, brute force, values printed in the paper);
see the pin table in the repository's design notes.
"""
from . import operators, rkl, multigrid, exact, smoothers, gradient  # noqa: F401
from .operators import Grid, Level, build_hierarchy, apply_M, residual, restrict, prolong  # noqa: F401
from .rkl import tau_step, rkl_coefficients  # noqa: F401
from .multigrid import Options, solve, vcycle, coarsest_solve, rkl_smooth  # noqa: F401
