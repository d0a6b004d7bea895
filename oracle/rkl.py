"""Runge-Kutta-Legendre (RKL1) relaxation and its spectral rules (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper references (Mandal, Mukherjee & Mignone 2023, Appendix A):
* stability polynomial R_s = P_s(1 + w1 tau lambda), w1 = 2/(s^2+s)
  (eq. RKL1 stability poly);
* stage recurrence with a source term (eq. RKL_intermediate_source) with
  mu_j = (2j-1)/j, nu_j = (1-j)/j, mu~_j = mu_j w1;
* stability limit tau_max = Delta t_par (s^2+s)/2 with
  Delta t_par = 2/|lambda_max| (eq. tau_max, Sec. 2.2.4);
* spectral radius of the iteration matrix over the lowest modes
  (eq. spectral_rad_RKL) and the iteration count m >= d / (-log10 rho)
  (eq. iteration); the best fixed s minimises m_eff = s m (eq. sopt_theory);
* per-mode optimal stage count from the first zero of J0:
  s_k = Round(2.4048 N/(pi k) - 1/2) (eq. sk_optimal), and the accelerated
  schedule that walks k from N/2 down to 1 skipping repeated s (App. A.4).

Reading adopted for tau (the paper's tau = tau_max leaves the checkerboard mode
of a cell-centred grid undamped, since it maps to P_s(-1) = +-1): tau is a
fraction theta of tau_max, so that w1 tau = theta Delta t_par.
"""
from __future__ import annotations

import math

import numpy as np

from .operators import apply_M

BESSEL_J0_FIRST_ZERO = 2.4048  # the value printed with eq. sk_optimal


def rkl_coefficients(s: int):
    """(mu_j, nu_j, mu~_j) for j = 1..s of an s-stage RKL1 step (App. A).

    j = 1 uses mu_1 = 1, nu_1 = 0 (the first stage Y1 = Y0 + mu~_1 tau (M Y0 - f)).
    """
    w1 = 2.0 / (s * s + s)
    out = []
    for j in range(1, s + 1):
        mu = (2.0 * j - 1.0) / j
        nu = (1.0 - j) / j
        out.append((mu, nu, mu * w1))
    return out


def tau_for(s: int, theta: float, dt_par: float) -> float:
    """tau = theta * tau_max(s) with tau_max = Delta t_par (s^2+s)/2 (eq. tau_max)."""
    return theta * dt_par * (s * s + s) / 2.0


def tau_step(u, b, s, theta, level, faces=None):
    """One s-stage RKL tau-step for M u = b on ``level`` (eq. RKL_intermediate_source).

    Y_0 = u
    Y_1 = Y_0 + mu~_1 tau (M Y_0 - b)
    Y_j = mu_j Y_{j-1} + nu_j Y_{j-2} + mu~_j tau (M Y_{j-1} - b),  2 <= j <= s
    returns Y_s.  Ghosts are refreshed before every application of M.
    """
    tau = tau_for(s, theta, level.dt_par)
    coeffs = rkl_coefficients(s)
    y_prev2 = None
    y_prev = u
    for j, (mu, nu, mut) in enumerate(coeffs, start=1):
        Lm = apply_M(y_prev, level.h, level.bc, faces) - b
        if j == 1:
            y = y_prev + mut * tau * Lm
        else:
            y = mu * y_prev + nu * y_prev2 + mut * tau * Lm
        y_prev2, y_prev = y_prev, y
    return y_prev


# ---------------------------------------------------------------------------
# spectral rules (App. A.3, A.4)
# ---------------------------------------------------------------------------

def legendre(s: int, x):
    """P_s(x) by the three-term recursion (eq. LP_recursion)."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if s == 0:
        return p0
    p1 = x.copy()
    for j in range(2, s + 1):
        p0, p1 = p1, ((2.0 * j - 1.0) / j) * x * p1 - ((j - 1.0) / j) * p0
    return p1


def rkl_eigenvalue_1d(s: int, k, N: int):
    """lambda_{k,RKL}(s) = P_s(cos(k pi / N)) for the 1-D vertex-centred model
    operator at tau = tau_max (eq. eigenvalue_RKL)."""
    return legendre(s, np.cos(np.asarray(k, dtype=np.float64) * math.pi / N))


def spectral_radius_1d(s: int, N: int, kmax: int = 6):
    """rho(R) restricted to the lowest ``kmax`` modes (eq. spectral_rad_RKL with
    the paper's observation that k <= 6 sets the maximum)."""
    k = np.arange(1, min(kmax, N // 2) + 1)
    return float(np.max(np.abs(rkl_eigenvalue_1d(s, k, N))))


def m_eff_1d(s: int, N: int, d: float = 2.0, kmax: int = 6):
    """m_eff = s * m_RKL with m_RKL = d / (-log10 rho) (eqs. iteration, sopt_theory)."""
    rho = spectral_radius_1d(s, N, kmax)
    if rho <= 0.0:
        return 0.0
    if rho >= 1.0:
        return math.inf
    return s * d / (-math.log10(rho))


def s_opt_global_1d(N: int, d: float = 2.0, kmax: int = 6):
    """Best fixed stage count: argmin over s in [1, N] of m_eff (eq. sopt_theory)."""
    best_s, best = None, math.inf
    for s in range(1, N + 1):
        m = m_eff_1d(s, N, d, kmax)
        if m < best:
            best, best_s = m, s
    return best_s


def s_k_opt_1d(k: int, N: int) -> int:
    """Per-mode optimal s from the first zero of J0 (eq. sk_optimal):
    Round(2.4048 N / (pi k) - 1/2), Round(p) = floor(p + 1/2)."""
    p = BESSEL_J0_FIRST_ZERO / math.pi * (N / k) - 0.5
    return max(1, int(math.floor(p + 0.5)))


def s_k_from_x(x: float) -> int:
    """Generalised per-mode rule: the mode enters P_s at x = cos(theta_k), and
    the first zero of sqrt(theta/sin theta) J0((s+1/2) theta) gives
    s = Round(2.4048/theta - 1/2) (eqs. legendre_approx, sk_optimal)."""
    theta = math.acos(max(-1.0, min(1.0, x)))
    if theta <= 0.0:
        return 1 << 20
    p = BESSEL_J0_FIRST_ZERO / theta - 0.5
    return max(1, int(math.floor(p + 0.5)))


def mode_eigenvalue(level, k: int) -> float:
    """|lambda_k| of the smoothest family of modes on ``level`` (a positive number).

    Dirichlet (homogeneous error ghosts): the diagonal mode (k,k,k) with 1-D
    cell-centred eigenvalues 4 sin^2(k pi / (2 n_d)) / h_d^2 summed over axes.
    Periodic: the axis-aligned mode with the smallest eigenvalue,
    min_d 4 sin^2(k pi / n_d) / h_d^2.
    For a cubic Dirichlet grid at theta = 1 this reproduces the paper's 1-D
    x_k = cos(k pi / N).
    """
    nz, ny, nx = level.shape
    hx, hy, hz = level.h
    # a 2-D level (nz = 1, hz = inf: eq. discrete_laplace_2D) has no z modes
    ax = [(n, hh) for n, hh in zip((nx, ny, nz), (hx, hy, hz)) if math.isfinite(hh)]
    ns = tuple(a[0] for a in ax)
    hs = tuple(a[1] for a in ax)
    if level.bc == "periodic":
        return min(4.0 * math.sin(k * math.pi / n) ** 2 / (hh * hh) for n, hh in zip(ns, hs))
    return sum(4.0 * math.sin(k * math.pi / (2.0 * n)) ** 2 / (hh * hh) for n, hh in zip(ns, hs))


def s_opt_global(level, theta: float, d: float = 2.0, kmax: int = 6):
    """Best fixed stage count on a 3-D (or 2-D) level at tau = theta tau_max
    (eq. sopt_theory with the reading of the accelerated schedule): mode k of
    the smoothest family (``mode_eigenvalue``) enters the stage polynomial at
    x_k = 1 - theta Delta t_par |lambda_k|; rho(s) = max over k = 1 ..
    min(kmax, n/2) of |P_s(x_k)| (n the smallest cell count), and s_opt
    minimises m_eff = s d / (-log10 rho) over 1 <= s <= the largest cell
    count.  On a cubic Dirichlet grid at theta = 1, x_k = cos(k pi / N) and
    this is ``s_opt_global_1d``.  Returns (s_opt, m_eff(s_opt))."""
    ns = [nn for nn, hh in zip(level.shape[::-1], level.h) if math.isfinite(hh)]
    kk = np.arange(1, max(1, min(kmax, min(ns) // 2)) + 1)
    x = np.array([1.0 - theta * level.dt_par * mode_eigenvalue(level, int(k)) for k in kk])
    best_s, best = None, math.inf
    for s in range(1, max(ns) + 1):
        rho = float(np.max(np.abs(legendre(s, x))))
        if rho <= 0.0:
            m = 0.0
        elif rho >= 1.0:
            m = math.inf
        else:
            m = s * d / (-math.log10(rho))
        if m < best:
            best, best_s = m, s
    return best_s, best


def accelerated_schedule(level, theta: float):
    """Stage counts of the accelerated RKL iteration on ``level`` (App. A.4).

    k walks from n/2 down to 1 (n = smallest cell count of the level); for
    each k the mode's stability argument is x_k = 1 - theta Delta t_par |lambda_k|
    and s_k = Round(2.4048/arccos(x_k) - 1/2); a k whose s equals the previous
    one is skipped.  After the list ends the iteration repeats its last entry
    (s for k = 1).
    """
    n = min(nn for nn, hh in zip(level.shape[::-1], level.h) if math.isfinite(hh))
    k = max(1, n // 2)
    out = []
    s_old = 0
    while True:
        x = 1.0 - theta * level.dt_par * mode_eigenvalue(level, k)
        s = s_k_from_x(x)
        if s != s_old:
            out.append(s)
            s_old = s
        if k == 1:
            break
        k -= 1
    return out
