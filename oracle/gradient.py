"""4th-order gravitational acceleration g = -grad(phi) (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper reference: Sec. 3, eq. 4thorder_acceleration:
g_x = -(4/3) (phi_{i+1} - phi_{i-1}) / (2 dx) + (1/3) (phi_{i+2} - phi_{i-2}) / (4 dx),
and likewise along y and z.  Two ghost layers are needed: periodic boxes
wrap; Dirichlet boxes (reading: the paper does not say how its second ghost
layer is filled) reflect oddly about the face value g, phi_{-m} = 2 g -
phi_{m-1} for m = 1, 2 (the first layer is the solution ghost of eq.
solution_ghost; without face data g = 0), which reproduces linear fields
exactly.

Two dimensions (nz = 1, hz = inf) have no z derivative: g_z is zero.
"""
from __future__ import annotations

import numpy as np


def acceleration_periodic(phi, h):
    """(g_x, g_y, g_z) on a periodic grid, arrays shaped like ``phi``."""
    out = []
    # numpy axis 2 = x, 1 = y, 0 = z
    for axis, hh in ((2, h[0]), (1, h[1]), (0, h[2])):
        if axis == 0 and _flat(phi, h):
            out.append(np.zeros_like(phi))
            continue
        p1 = np.roll(phi, -1, axis=axis)
        m1 = np.roll(phi, 1, axis=axis)
        p2 = np.roll(phi, -2, axis=axis)
        m2 = np.roll(phi, 2, axis=axis)
        out.append(-(4.0 / 3.0) * (p1 - m1) / (2.0 * hh) + (1.0 / 3.0) * (p2 - m2) / (4.0 * hh))
    return tuple(out)


def _flat(phi, h):
    return phi.shape[0] == 1 and not np.isfinite(h[2])


def _pad2(phi, bc, faces, flat=False):
    """Copy of phi with two ghost layers per face (edges and corners unused)."""
    nz, ny, nx = phi.shape
    p = np.zeros((nz + 4, ny + 4, nx + 4))
    p[2:-2, 2:-2, 2:-2] = phi
    if bc == "periodic":
        p[2:-2, 2:-2, :] = np.pad(phi, ((0, 0), (0, 0), (2, 2)), mode="wrap")
        p[2:-2, :, 2:-2] = np.pad(phi, ((0, 0), (2, 2), (0, 0)), mode="wrap")
        p[:, 2:-2, 2:-2] = np.pad(phi, ((2, 2), (0, 0), (0, 0)), mode="wrap")
        return p
    g = faces if faces is not None else (0.0,) * 6
    for m in (1, 2):
        p[2:-2, 2:-2, 2 - m] = 2.0 * np.asarray(g[0]) - phi[:, :, m - 1]
        p[2:-2, 2:-2, nx + 1 + m] = 2.0 * np.asarray(g[1]) - phi[:, :, nx - m]
        p[2:-2, 2 - m, 2:-2] = 2.0 * np.asarray(g[2]) - phi[:, m - 1, :]
        p[2:-2, ny + 1 + m, 2:-2] = 2.0 * np.asarray(g[3]) - phi[:, ny - m, :]
        if not flat:
            p[2 - m, 2:-2, 2:-2] = 2.0 * np.asarray(g[4]) - phi[m - 1, :, :]
            p[nz + 1 + m, 2:-2, 2:-2] = 2.0 * np.asarray(g[5]) - phi[nz - m, :, :]
    return p


def acceleration(phi, h, bc="periodic", faces=None):
    """(g_x, g_y, g_z) by eq. 4thorder_acceleration with the two-layer ghosts
    described in the module docstring; ``faces`` = (x-, x+, y-, y+, z-, z+)
    face values of phi for Dirichlet boxes (None: homogeneous)."""
    phi = np.asarray(phi, dtype=np.float64)
    flat = _flat(phi, h)
    p = _pad2(phi, bc, faces, flat)
    c = p[2:-2, 2:-2, 2:-2]
    out = []
    for axis, hh in ((2, h[0]), (1, h[1]), (0, h[2])):
        if axis == 0 and flat:
            out.append(np.zeros_like(phi))
            continue

        def sh(d):
            sl = [slice(2, -2)] * 3
            n = p.shape[axis] - 4
            sl[axis] = slice(2 + d, 2 + d + n)
            return p[tuple(sl)]
        out.append(-(4.0 / 3.0) * (sh(1) - sh(-1)) / (2.0 * hh) + (1.0 / 3.0) * (sh(2) - sh(-2)) / (4.0 * hh))
    del c
    return tuple(out)
