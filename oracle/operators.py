"""Cell-centred grid, ghost cells, Laplacian and grid-transfer operators (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper references (Mandal, Mukherjee & Mignone 2023):
* cell-centred discretisation: Sec. 2.2 (opening paragraph);
* 7-point Laplacian: Sec. 2.2.1, eq. discrete_laplace_3D;
* residual r = L Psi - f: Sec. 2.1, eq. residual;
* 8-point restriction: Sec. 2.2.2, eqs. restriction_equation_3D / _example_3D;
* cell-centred prolongation (27,9,9,9,3,3,3,1)/64: Sec. 2.2.3,
  eq. prolongation_example_3D;
* Dirichlet ghosts by linear extrapolation on the finest level: Sec. 2.3,
  eq. solution_ghost; homogeneous error ghosts on coarse levels: eq. error_ghost;
  periodic ghosts on all levels: eq. periodic.

Arrays are float64 numpy arrays of shape (nz, ny, nx) (x fastest).  Boundary
face arrays (Dirichlet, finest level only) are ordered x-, x+, y-, y+, z-, z+
with shapes (nz,ny), (nz,ny), (nz,nx), (nz,nx), (ny,nx), (ny,nx).

Two dimensions (eqs. discrete_laplace_2D, restriction_example_2D,
prolongation_example_2D) use the same arrays with nz = 1 and hz = inf: every
z term of the operator then carries the factor 1/hz^2 = 0, so the 7-point
operator is the 5-point one; the hierarchy coarsens x and y only, restriction
averages 4 children and prolongation weighs (9, 3, 3, 1)/16.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

DIRICHLET = "dirichlet"
PERIODIC = "periodic"


@dataclass(frozen=True)
class Grid:
    """Finest-level problem geometry: cell counts, spacings, boundary type."""

    nx: int
    ny: int
    nz: int
    hx: float
    hy: float
    hz: float
    bc: str

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def flat(self):
        """A 2-D problem: nz = 1 and hz = inf."""
        return self.nz == 1 and not np.isfinite(self.hz)


def grid2d(nx, ny, hx, hy, bc):
    """A 2-D grid in the (nz = 1, hz = inf) representation."""
    return Grid(nx, ny, 1, hx, hy, float("inf"), bc)


@dataclass
class Level:
    """One level of the hierarchy.  ``level`` is l (0 = finest)."""

    level: int
    shape: tuple  # (nz, ny, nx)
    h: tuple  # (hx, hy, hz)
    bc: str

    @property
    def flat(self):
        return self.shape[0] == 1 and not np.isfinite(self.h[2])

    @property
    def lam(self):
        """Lambda_l = 4 sum_d h_d^-2: the Gershgorin bound of |lambda_max(M_l)|
        (Sec. 2.2.4 eq. tau_max with the 3-D 7-point operator)."""
        hx, hy, hz = self.h
        return 4.0 * (1.0 / hx**2 + 1.0 / hy**2 + 1.0 / hz**2)

    @property
    def dt_par(self):
        """Explicit parabolic step Delta t_par = 2 / |lambda_max| (eq. tau_max)."""
        return 2.0 / self.lam


def build_hierarchy(grid: Grid, min_coarse: int = 4):
    """Level list from finest to coarsest.

    Coarsening halves every axis; it continues while every n_d/2 is an even
    integer that is at least ``min_coarse`` (the paper keeps N/2^(L-1) even,
    Sec. 4.1; the coarsest size floor follows the 32^3 -> 4^3 configuration).
    A grid that cannot be coarsened gives a single level.
    """
    levels = []
    shape = grid.shape
    h = (grid.hx, grid.hy, grid.hz)
    l = 0
    levels.append(Level(0, shape, h, grid.bc))
    flat = grid.flat
    def ok(n):
        return (n % 2 == 0) and ((n // 2) % 2 == 0) and (n // 2 >= min_coarse)
    while all(ok(n) for n in (shape[1:] if flat else shape)):
        shape = ((1,) if flat else (shape[0] // 2,)) + tuple(n // 2 for n in shape[1:])
        h = (2.0 * h[0], 2.0 * h[1], h[2] if flat else 2.0 * h[2])
        l += 1
        levels.append(Level(l, shape, h, grid.bc))
    return levels


def padded(u, bc, faces=None):
    """Copy of ``u`` with one ghost layer on every face.

    * periodic: wrap (eq. periodic), on every level;
    * Dirichlet with ``faces`` (finest level): ghost = 2 g - u_adj
      (eq. solution_ghost);
    * Dirichlet with ``faces is None`` (coarse levels, error equation):
      ghost = - u_adj (eq. error_ghost).
    Edge and corner ghosts are left at zero; the 7-point stencil never reads them.
    """
    nz, ny, nx = u.shape
    p = np.zeros((nz + 2, ny + 2, nx + 2), dtype=u.dtype)
    p[1:-1, 1:-1, 1:-1] = u
    if bc == PERIODIC:
        p[1:-1, 1:-1, 0] = u[:, :, -1]
        p[1:-1, 1:-1, -1] = u[:, :, 0]
        p[1:-1, 0, 1:-1] = u[:, -1, :]
        p[1:-1, -1, 1:-1] = u[:, 0, :]
        p[0, 1:-1, 1:-1] = u[-1, :, :]
        p[-1, 1:-1, 1:-1] = u[0, :, :]
        return p
    if bc != DIRICHLET:
        raise ValueError(f"unknown boundary type {bc!r}")
    if faces is None:
        gxm = gxp = gym = gyp = gzm = gzp = 0.0
    else:
        gxm, gxp, gym, gyp, gzm, gzp = faces
    p[1:-1, 1:-1, 0] = 2.0 * gxm - u[:, :, 0]
    p[1:-1, 1:-1, -1] = 2.0 * gxp - u[:, :, -1]
    p[1:-1, 0, 1:-1] = 2.0 * gym - u[:, 0, :]
    p[1:-1, -1, 1:-1] = 2.0 * gyp - u[:, -1, :]
    p[0, 1:-1, 1:-1] = 2.0 * gzm - u[0, :, :]
    p[-1, 1:-1, 1:-1] = 2.0 * gzp - u[-1, :, :]
    return p


def apply_M(u, h, bc, faces=None):
    """7-point discrete Laplacian with ghosts filled per ``padded`` (eq. discrete_laplace_3D).

    Returns sum_d (u_{-d} - 2u + u_{+d}) / h_d^2 on the active cells.  With
    Dirichlet ``faces`` the operator is affine: it includes the boundary terms.
    """
    hx, hy, hz = h
    p = padded(u, bc, faces)
    c = p[1:-1, 1:-1, 1:-1]
    lx = (p[1:-1, 1:-1, :-2] - 2.0 * c + p[1:-1, 1:-1, 2:]) / (hx * hx)
    ly = (p[1:-1, :-2, 1:-1] - 2.0 * c + p[1:-1, 2:, 1:-1]) / (hy * hy)
    lz = (p[:-2, 1:-1, 1:-1] - 2.0 * c + p[2:, 1:-1, 1:-1]) / (hz * hz)
    return lx + ly + lz


def residual(u, b, h, bc, faces=None):
    """r = M u - b (Sec. 2.1, eq. residual, with b in place of f)."""
    return apply_M(u, h, bc, faces) - b


def restrict(r, flat=False):
    """8-point average onto the coarse grid (eq. restriction_example_3D); in
    2-D (``flat``, nz = 1) the 4-point average of eq. restriction_example_2D."""
    nz, ny, nx = r.shape
    if flat:
        v = r.reshape(1, ny // 2, 2, nx // 2, 2)
        return v.sum(axis=(2, 4)) / 4.0
    v = r.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2)
    return v.sum(axis=(1, 3, 5)) / 8.0


def prolong(e, bc, flat=False):
    """Cell-centred trilinear prolongation (eq. prolongation_example_3D).

    Each fine cell takes 27/64 of its parent A, 9/64 of each of the three
    face-adjacent coarse cells on its side (B, D, E), 3/64 of the three
    edge-adjacent ones (C, F, H) and 1/64 of the corner one (G).  Coarse ghosts
    are those of the error equation: homogeneous Dirichlet (-e_adj) or
    periodic wrap (Sec. 2.3).  In 2-D (``flat``, nz = 1) the weights are
    (9, 3, 3, 1)/16 in x and y (eq. prolongation_example_2D).
    """
    if flat:
        return _prolong_2d(e, bc)
    p = padded(e, bc, None)
    # corner ghosts are needed by the corner weight G: fill them consistently
    # (periodic: wrap; Dirichlet: odd reflection through each face)
    p = _fill_edges_corners(p, bc)
    nz, ny, nx = e.shape
    out = np.zeros((2 * nz, 2 * ny, 2 * nx), dtype=e.dtype)
    w = {0: 3.0, 1: 1.0}  # 1-D weights: parent side 3/4, neighbour side 1/4
    for oz in (0, 1):
        for oy in (0, 1):
            for ox in (0, 1):
                # fine child (oz, oy, ox) of each coarse cell: its neighbours lie
                # on the -1 side for offset 0 and the +1 side for offset 1
                sz = -1 if oz == 0 else 1
                sy = -1 if oy == 0 else 1
                sx = -1 if ox == 0 else 1
                acc = np.zeros_like(e)
                for dz in (0, 1):
                    for dy in (0, 1):
                        for dx in (0, 1):
                            wt = w[dz] * w[dy] * w[dx] / 64.0
                            acc += wt * p[1 + dz * sz: 1 + dz * sz + nz,
                                          1 + dy * sy: 1 + dy * sy + ny,
                                          1 + dx * sx: 1 + dx * sx + nx]
                out[oz::2, oy::2, ox::2] = acc
    return out


def _prolong_2d(e, bc):
    """Bilinear cell-centred prolongation of a (1, ny, nx) array."""
    q = _fill_edges_corners(padded(e, bc, None), bc)[1]  # (ny + 2, nx + 2) plane with ghosts
    _, ny, nx = e.shape
    out = np.zeros((1, 2 * ny, 2 * nx), dtype=e.dtype)
    w = {0: 3.0, 1: 1.0}
    for oy in (0, 1):
        for ox in (0, 1):
            sy = -1 if oy == 0 else 1
            sx = -1 if ox == 0 else 1
            acc = np.zeros((ny, nx), dtype=e.dtype)
            for dy in (0, 1):
                for dx in (0, 1):
                    acc += (w[dy] * w[dx] / 16.0) * q[1 + dy * sy: 1 + dy * sy + ny, 1 + dx * sx: 1 + dx * sx + nx]
            out[0, oy::2, ox::2] = acc
    return out


def _fill_edges_corners(p, bc):
    """Fill the edge and corner ghosts of a padded coarse array.

    Periodic: wrap.  Dirichlet (homogeneous error): the ghost is the odd
    reflection through every boundary face it lies beyond, which is the
    linear extrapolation of eq. error_ghost applied axis by axis.
    """
    if bc == PERIODIC:
        inner = p[1:-1, 1:-1, 1:-1]
        return np.pad(inner, 1, mode="wrap")
    q = p.copy()
    # apply the reflection axis by axis on the already extended array so that
    # edges/corners become products of single-face reflections
    q[:, :, 0] = -q[:, :, 1]
    q[:, :, -1] = -q[:, :, -2]
    q[:, 0, :] = -q[:, 1, :]
    q[:, -1, :] = -q[:, -2, :]
    q[0, :, :] = -q[1, :, :]
    q[-1, :, :] = -q[-2, :, :]
    return q
