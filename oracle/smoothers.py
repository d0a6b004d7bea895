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

Reading of the splitting: rho_J and the optimal omega of App. B are those of
the Jacobi splitting of the discrete operator itself, so every relaxation
divides the residual by the operator's own diagonal.  For a cell next to a
Dirichlet face that diagonal includes the ghost's -u term (ghost 2 g - u,
eq. solution_ghost, or -u, eq. error_ghost): D_cell = 2 sum h^-2 + h_d^-2 per
such face.  The update is u <- u + omega (M u - b) / D_cell with M u built from
the current values (ghosts refreshed before every half-sweep).
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


def cell_diagonal(shape, h, bc):
    """-(diagonal of M) per cell: 2 sum h^-2, plus h_d^-2 for each Dirichlet
    face the cell touches (the ghost's -u term)."""
    d = np.full(shape, _diag(h))
    if bc == "dirichlet":
        hx, hy, hz = h
        d[:, :, 0] += 1.0 / hx**2
        d[:, :, -1] += 1.0 / hx**2
        d[:, 0, :] += 1.0 / hy**2
        d[:, -1, :] += 1.0 / hy**2
        d[0, :, :] += 1.0 / hz**2
        d[-1, :, :] += 1.0 / hz**2
    return d


def _residual_M(u, b, h, bc, faces):
    """M u - b with the ghosts of the current u."""
    return _nbr_sum(u, h, bc, faces) - _diag(h) * u - b


def jacobi_sweep(u, b, h, bc, faces=None, omega=1.0):
    """omega-Jacobi: u <- u + omega (M u - b) / D_cell."""
    return u + omega * _residual_M(u, b, h, bc, faces) / cell_diagonal(u.shape, h, bc)


def colour_mask(shape, colour):
    """True on cells with (i + j + k) % 2 == colour (0 = red, 1 = black)."""
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((i + j + k) % 2) == colour


def gsrb_sweep(u, b, h, bc, faces=None, omega=1.0):
    """One red-black Gauss-Seidel iteration (red half-sweep, then black), each
    colour u <- u + omega (M u - b) / D_cell from the values before that half
    sweep.  ``omega`` != 1 gives the SOR variant."""
    u = np.array(u, copy=True)
    dc = cell_diagonal(u.shape, h, bc)
    for colour in (0, 1):
        m = colour_mask(u.shape, colour)
        r = _residual_M(u, b, h, bc, faces)
        u[m] = u[m] + omega * r[m] / dc[m]
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
