"""Correction-scheme multigrid with RKL smoothing and an RKL coarsest solver (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper references (Mandal, Mukherjee & Mignone 2023):
* V-cycle: Sec. 2.1 (the do { ... } while listing) with N_pre = 2, N_post = 1
  (Sec. 4.1);
* error equation L e = -r and correction Psi <- Psi + e: Sec. 2.1, eqs.
  error_equation, new_guess;
* periodic compatibility: f <- f - mean(f) (Sec. 2.3, eq. source_modification)
  and the residual mean removed on every coarse level (Sec. 2.3, last paragraph);
* coarsest solver: the accelerated RKL iteration (App. A.4);
* convergence metric: L2 norm of the residual relative to the residual of
  Phi = 0 (Sec. 4.1, caption of the error figure);
* RKL as the relaxation (Sec. 2.2.4; App. A.2 eq. RKL_intermediate_source);
  the paper's own smoother, red-black Gauss-Seidel (Sec. 2.2.4), is the
  alternative ``smoother="gsrb"`` (one relaxation = one red + black pass);
* single-level relaxation to a maximum residual (App. B): accelerated RKL,
  GS-RB and SOR with the App. B over-relaxation parameter.

Readings of silent or garbled points (listed in the design notes):
* the coarse-level signs of the listing are made consistent by writing every
  level as M_l u_l = b_l with b_0 = f and b_{l+1} = -R(M_l u_l - b_l);
* one relaxation = one RKL tau-step of ``s`` stages with tau = theta tau_max;
* coarsest solve: accelerated schedule until ||M u - b|| <= coarse_tol ||b||
  (1e-13 in float64, 1e-6 in float32) or ``coarse_max_steps`` tau-steps;
* coarse-level ghosts used by prolongation are the error ghosts (homogeneous
  Dirichlet or periodic).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

from .operators import (DIRICHLET, PERIODIC, Grid, apply_M, build_hierarchy,
                        prolong, restrict)
from .rkl import accelerated_schedule, tau_step
from .smoothers import gsrb_sweep, sor_omega

STATUS_OK = 0
STATUS_ENOCONV = -3
STATUS_EDIVERGED = -4
STATUS_ENONFINITE = -5


@dataclass
class Options:
    """Solver options; defaults follow the paper where it states them."""

    s: int = 2                  # stages per smoothing tau-step
    theta: float = 0.9          # tau / tau_max(s)
    n_pre: int = 2              # Sec. 4.1
    n_post: int = 1             # Sec. 4.1
    min_coarse: int = 4
    tol: float = 1e-10          # relative L2 residual (Sec. 4.1)
    max_cycles: int = 100
    four_pi_G: float = 4.0 * math.pi   # G = 1 (Sec. 4.1)
    coarse_tol: float | None = None    # None: 1e-13 (float64) / 1e-6 (float32)
    coarse_max_steps: int = 200
    smoother: str = "rkl"       # "rkl": one s-stage tau-step; "gsrb": one red-black GS pass
    omega: float = 1.0          # GS-RB over-relaxation inside the V-cycle (1 = plain GS-RB)


@dataclass
class Stats:
    cycles: int = 0
    res0: float = 0.0
    rel_res: float = 0.0
    history: list = field(default_factory=list)
    status: int = STATUS_OK
    coarse_steps: list = field(default_factory=list)


def l2(x):
    """Plain Euclidean norm in float64 (the uniform-cell L2 norm of Sec. 4.1
    up to a constant factor that cancels in every ratio used here)."""
    x = np.asarray(x, dtype=np.float64)
    return math.sqrt(float(np.sum(x * x)))


def _coarse_tol(opts, dtype):
    if opts.coarse_tol is not None:
        return opts.coarse_tol
    return 1e-13 if np.dtype(dtype) == np.float64 else 1e-6


def rkl_accelerated(u, b, level, theta, faces=None, tol=1e-13, max_steps=200,
                    ref_norm=None, remove_mean=None):
    """Accelerated RKL iteration on one level (App. A.4).

    Takes tau-steps with the stage counts of ``accelerated_schedule`` (then its
    last entry repeated) while ||M u - b|| > tol * ref_norm, at most
    ``max_steps`` steps.  ``ref_norm`` defaults to ||b||.  For periodic levels
    the mean of u is removed after every step.  Returns (u, steps_taken,
    final_residual_norm).
    """
    sched = accelerated_schedule(level, theta)
    if ref_norm is None:
        ref_norm = l2(b)
    if remove_mean is None:
        remove_mean = level.bc == PERIODIC
    steps = 0
    while True:
        res = l2(apply_M(u, level.h, level.bc, faces) - b)
        if res <= tol * ref_norm or steps >= max_steps:
            return u, steps, res
        s = sched[min(steps, len(sched) - 1)]
        u = tau_step(u, b, s, theta, level, faces)
        if remove_mean:
            u = u - u.mean()
        steps += 1


def relax(u, b, level, opts, faces=None):
    """One relaxation of M u = b on ``level``: an RKL tau-step (s stages,
    tau = theta tau_max), or one red-black Gauss-Seidel pass (Sec. 2.2.4)."""
    if opts.smoother == "rkl":
        return tau_step(u, b, opts.s, opts.theta, level, faces)
    if opts.smoother == "gsrb":
        return gsrb_sweep(u, b, level.h, level.bc, faces, opts.omega)
    raise ValueError(f"unknown smoother {opts.smoother!r}")


def coarsest_solve(b, level, opts, stats=None):
    """Solve M_c u = b on the coarsest level from u = 0 (homogeneous ghosts)."""
    u = np.zeros_like(b)
    if l2(b) == 0.0:
        if stats is not None:
            stats.coarse_steps.append(0)
        return u
    u, steps, _ = rkl_accelerated(u, b, level, opts.theta, None,
                                  _coarse_tol(opts, b.dtype), opts.coarse_max_steps)
    if stats is not None:
        stats.coarse_steps.append(steps)
    return u


def vcycle(u0, f, levels, opts, faces=None, stats=None):
    """One correction-scheme V-cycle for M_0 u = f (Sec. 2.1).

    Level 0 uses the problem's ghosts (``faces`` for Dirichlet); every coarser
    level solves the error equation with homogeneous / periodic ghosts.
    """
    L = len(levels)
    bc = levels[0].bc
    u = [None] * L
    b = [None] * L
    u[0] = u0.copy()
    b[0] = f
    if L == 1:
        # single level: the relaxation is the whole cycle
        for _ in range(opts.n_pre + opts.n_post):
            u[0] = relax(u[0], b[0], levels[0], opts, faces)
        return u[0]
    for _ in range(opts.n_pre):
        u[0] = relax(u[0], b[0], levels[0], opts, faces)
    for l in range(1, L):
        lv = levels[l - 1]
        r = apply_M(u[l - 1], lv.h, bc, faces if l == 1 else None) - b[l - 1]
        b[l] = -restrict(r, lv.flat)
        if bc == PERIODIC:
            b[l] = b[l] - b[l].mean()
        u[l] = np.zeros_like(b[l])
        if l < L - 1:
            for _ in range(opts.n_pre):
                u[l] = relax(u[l], b[l], levels[l], opts, None)
        else:
            u[l] = coarsest_solve(b[l], levels[l], opts, stats)
    for l in range(L - 2, -1, -1):
        u[l] = u[l] + prolong(u[l + 1], bc, levels[l].flat)
        fl = faces if l == 0 else None
        for _ in range(opts.n_post):
            u[l] = relax(u[l], b[l], levels[l], opts, fl)
    return u[0]


def prepare_source(rho, grid, opts):
    """f = 4 pi G rho (eq. poisson_eqaution); periodic: f - mean(f) (eq. source_modification)."""
    f = opts.four_pi_G * np.asarray(rho, dtype=np.float64)
    if grid.bc == PERIODIC:
        f = f - f.mean()
    return f


def solve(rho, grid: Grid, opts: Options = None, faces=None, phi0=None):
    """Full solve of nabla^2 phi = 4 pi G rho to relative residual ``opts.tol``.

    Outer loop: V-cycles until ||M u - f|| / ||M 0 - f|| <= tol (Sec. 4.1);
    M 0 carries the Dirichlet boundary terms.  For grids that do not coarsen
    the accelerated single-level RKL iteration (App. A.4, App. B) runs to
    tolerance instead.  Periodic results are returned with zero mean.
    Returns (phi, Stats).
    """
    opts = opts or Options()
    levels = build_hierarchy(grid, opts.min_coarse)
    f = prepare_source(rho, grid, opts)
    fz = faces if grid.bc == DIRICHLET else None
    u = np.zeros(grid.shape) if phi0 is None else np.array(phi0, dtype=np.float64)
    stats = Stats()
    res0 = l2(apply_M(np.zeros(grid.shape), levels[0].h, grid.bc, fz) - f)
    stats.res0 = res0
    if res0 == 0.0:
        stats.rel_res = 0.0
        return np.zeros(grid.shape), stats
    if not np.all(np.isfinite(f)):
        stats.status = STATUS_ENONFINITE
        return u, stats
    if len(levels) == 1:
        u, steps, res = rkl_accelerated(u, f, levels[0], opts.theta, fz, opts.tol,
                                        opts.max_cycles, ref_norm=res0,
                                        remove_mean=False)
        stats.cycles = steps
        stats.rel_res = res / res0
        if stats.rel_res > opts.tol:
            stats.status = STATUS_ENOCONV
    else:
        grow = 0
        prev = math.inf
        while True:
            rel = l2(apply_M(u, levels[0].h, grid.bc, fz) - f) / res0
            stats.history.append(rel)
            stats.rel_res = rel
            if not math.isfinite(rel):
                stats.status = STATUS_ENONFINITE
                break
            if rel <= opts.tol:
                break
            grow = grow + 1 if rel > prev else 0
            if grow >= 3:
                stats.status = STATUS_EDIVERGED
                break
            if stats.cycles >= opts.max_cycles:
                stats.status = STATUS_ENOCONV
                break
            prev = rel
            u = vcycle(u, f, levels, opts, fz, stats)
            stats.cycles += 1
    if grid.bc == PERIODIC:
        u = u - u.mean()
    return u, stats


def relax_solve(f, grid: Grid, method, faces=None, tol_max=1e-10, max_iters=100000,
                s=0, theta=0.9, omega=None, check_every=1, phi0=None):
    """Single-level relaxation of M u = f (no multigrid), App. B.

    Iterates until the maximum residual max|M u - f| <= ``tol_max`` (tested
    before every ``check_every`` iterations) or ``max_iters`` iterations:
    * ``"rkl"``: RKL tau-steps; s = 0 walks the accelerated schedule of
      App. A.4 (then its last entry repeated), s > 0 keeps s fixed;
      tau = theta tau_max(s);
    * ``"gsrb"``: red-black Gauss-Seidel passes (omega = 1);
    * ``"sor"``: red-black SOR with omega from App. B (``sor_omega``) unless
      ``omega`` is given.
    Periodic grids have the mean of u removed after every iteration.
    Returns (u, iterations, final max residual, history of tested residuals).
    """
    lv = build_hierarchy(grid, 1 << 30)[0]
    fz = faces if grid.bc == DIRICHLET else None
    u = np.zeros(grid.shape) if phi0 is None else np.array(phi0, dtype=np.float64)
    if method == "sor" and omega is None:
        omega = sor_omega(grid.shape, lv.h)
    sched = accelerated_schedule(lv, theta) if (method == "rkl" and s == 0) else None
    it = 0
    hist = []
    while True:
        res = float(np.abs(apply_M(u, lv.h, grid.bc, fz) - f).max())
        hist.append(res)
        if res <= tol_max or it >= max_iters:
            return u, it, res, hist
        for _ in range(check_every):
            if it >= max_iters:
                break
            if method == "rkl":
                sk = sched[min(it, len(sched) - 1)] if sched is not None else s
                u = tau_step(u, f, sk, theta, lv, fz)
            elif method in ("gsrb", "sor"):
                u = gsrb_sweep(u, f, lv.h, grid.bc, fz, 1.0 if method == "gsrb" else omega)
            else:
                raise ValueError(f"unknown method {method!r}")
            if grid.bc == PERIODIC:
                u = u - u.mean()
            it += 1


def rkl_smooth(phi, f, grid: Grid, s, theta, n_steps, faces=None):
    """``n_steps`` RKL tau-steps of ``s`` stages on M phi = f at the finest level
    (no mean removal; f is used as given)."""
    lv = build_hierarchy(grid, 1 << 30)[0]
    u = np.array(phi, dtype=np.float64)
    for _ in range(n_steps):
        u = tau_step(u, f, s, theta, lv, faces if grid.bc == DIRICHLET else None)
    return u


def solve_mixed(rho, grid: Grid, opts: Options = None, faces=None, inner_cycles=1):
    """Mixed-precision defect correction (float32 V-cycles inside float64).

    Outer float64 loop: r = f - M u (with the level-0 boundary terms) and its
    float64 norm; the correction equation M e = r is solved approximately by
    ``inner_cycles`` float32 V-cycles from e = 0 with homogeneous level-0
    ghosts; u += e in float64.  Stops when the float64 relative residual is
    <= tol.  Returns (phi, Stats).
    """
    opts = opts or Options()
    levels = build_hierarchy(grid, opts.min_coarse)
    f = prepare_source(rho, grid, opts)
    fz = faces if grid.bc == DIRICHLET else None
    u = np.zeros(grid.shape)
    stats = Stats()
    res0 = l2(apply_M(u, levels[0].h, grid.bc, fz) - f)
    stats.res0 = res0
    if res0 == 0.0:
        return u, stats
    while True:
        r = f - apply_M(u, levels[0].h, grid.bc, fz)
        rel = l2(r) / res0
        stats.history.append(rel)
        stats.rel_res = rel
        if rel <= opts.tol:
            break
        if stats.cycles >= opts.max_cycles:
            stats.status = STATUS_ENOCONV
            break
        r32 = r.astype(np.float32)
        if grid.bc == PERIODIC:
            r32 = r32 - r32.mean(dtype=np.float32)
        e = np.zeros_like(r32)
        for _ in range(inner_cycles):
            e = vcycle(e, r32, levels, opts, None, stats)
        u = u + e.astype(np.float64)
        stats.cycles += 1
    if grid.bc == PERIODIC:
        u = u - u.mean()
    return u, stats


def adjoint_solve(w, grid: Grid, opts: Options = None):
    """Gradient of L = sum(w * phi) with respect to rho.

    phi = S(4 pi G rho) with S the (mean-projected, for periodic) inverse of
    the symmetric operator M with the problem's boundary terms; the boundary
    data does not depend on rho, so dL/drho = 4 pi G S^T w = 4 pi G S w:
    one more solve with source w, homogeneous ghosts and no 4 pi G scaling.
    """
    opts = opts or Options()
    o1 = replace(opts, four_pi_G=1.0)
    lam, st = solve(w, grid, o1, faces=None)
    return opts.four_pi_G * lam, st
