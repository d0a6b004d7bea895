"""The paper's own relaxations: Jacobi, red-black Gauss-Seidel and SOR (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper references (Mandal, Mukherjee & Mignone 2023):
* GS-RB smoother, two half-sweeps over the checkerboard colours: Sec. 2.2.4
  and its footnote;
* omega-Jacobi, SOR and the optimal over-relaxation parameter
  omega = 2 / (1 + sqrt(1 - rho_J^2)) with the Jacobi spectral radius of a
  Dirichlet box: App. B.

Reading of App. B: its Delta_t = 2 [sum h^-2]^-1 would make rho_J exceed 1 on
a uniform grid; the factor is taken as 1/2 (Delta_t = Delta t_par), which gives
the textbook rho_J = cos(pi/N) for a cube.

Ghost cells are refreshed before every half-sweep (lagged ghosts).
"""
from __future__ import annotations

import math

import numpy as np

from .operators import padded


def _nbr_sum(u, h, bc, faces):
    hx, hy, hz = h
    p = padded(u, bc, faces)
    return ((p[1:-1, 1:-1, :-2] + p[1:-1, 1:-1, 2:]) / (hx * hx)
            + (p[1:-1, :-2, 1:-1] + p[1:-1, 2:, 1:-1]) / (hy * hy)
            + (p[:-2, 1:-1, 1:-1] + p[2:, 1:-1, 1:-1]) / (hz * hz))


def _diag(h):
    hx, hy, hz = h
    return 2.0 * (1.0 / hx**2 + 1.0 / hy**2 + 1.0 / hz**2)


def jacobi_sweep(u, b, h, bc, faces=None, omega=1.0):
    """omega-Jacobi: u <- (1-omega) u + omega (sum_nbr/h^2 - b) / (2 sum h^-2)."""
    new = (_nbr_sum(u, h, bc, faces) - b) / _diag(h)
    return (1.0 - omega) * u + omega * new


def colour_mask(shape, colour):
    """True on cells with (i + j + k) % 2 == colour (0 = red, 1 = black)."""
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((i + j + k) % 2) == colour


def gsrb_sweep(u, b, h, bc, faces=None, omega=1.0):
    """One red-black Gauss-Seidel iteration (red half-sweep, then black).
    ``omega`` != 1 gives the SOR variant."""
    u = np.array(u, copy=True)
    for colour in (0, 1):
        m = colour_mask(u.shape, colour)
        new = (_nbr_sum(u, h, bc, faces) - b) / _diag(h)
        u[m] = (1.0 - omega) * u[m] + omega * new[m]
    return u


def rho_jacobi_dirichlet(shape, h):
    """Jacobi spectral radius of a Dirichlet box (App. B, with Delta_t = Delta t_par)."""
    nz, ny, nx = shape
    hx, hy, hz = h
    dt = 0.5 / (1.0 / hx**2 + 1.0 / hy**2 + 1.0 / hz**2)
    return 2.0 * dt * (math.cos(math.pi / nx) / hx**2 + math.cos(math.pi / ny) / hy**2
                       + math.cos(math.pi / nz) / hz**2)


def sor_omega(shape, h):
    """omega = 2 / (1 + sqrt(1 - rho_J^2)) (App. B)."""
    rj = rho_jacobi_dirichlet(shape, h)
    return 2.0 / (1.0 + math.sqrt(1.0 - rj * rj))
