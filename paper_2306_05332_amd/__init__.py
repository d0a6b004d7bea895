"""MI355X-native (gfx950) RKL-multigrid Poisson solver.

Solves nabla^2 phi = 4 pi G rho on cell-centred boxes (Dirichlet or periodic)
with a correction-scheme V-cycle whose smoother and coarsest-grid solver are
Runge-Kutta-Legendre super-time-steps (Mandal, Mukherjee & Mignone 2023).
All arithmetic runs in hand-written HIP kernels behind the C ABI of
``include/rkl_poisson.h``; this package is the thin Python binding.
"""
from ._lib import (RKLError, Options, Stats, coarse_solve, load_library, pack_faces,  # noqa: F401
                   prolong_add, release_all, residual, restrict, smooth, solve, solve_batched,
                   vcycle, tau_step_launches, kernel_info, EXPORTS, LIB_PATH, VARIANTS,
                   tune_set, tune_clear, tune_get, autotune_level, tune_set_s, level_shapes,
                   install_default_tuning, gsrb_smooth, relax_solve, gradient, s_opt, residual_noalloc,
                   RKL_OK, RKL_EINVAL, RKL_ENOMEM, RKL_ENOCONV, RKL_EDIVERGED, RKL_ENONFINITE, RKL_EHIP)
from .autograd import PoissonSolve, poisson_solve  # noqa: F401,E402
