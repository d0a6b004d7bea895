"""4th-order gravitational acceleration g = -grad(phi) (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper reference: Sec. 3, eq. 4thorder_acceleration:
g_x = -(4/3) (phi_{i+1} - phi_{i-1}) / (2 dx) + (1/3) (phi_{i+2} - phi_{i-2}) / (4 dx),
and likewise along y and z.  Two ghost layers are needed; this oracle
implements the periodic case (wrap), where every cell has its full stencil.
"""
from __future__ import annotations

import numpy as np


def acceleration_periodic(phi, h):
    """(g_x, g_y, g_z) on a periodic grid, arrays shaped like ``phi``."""
    out = []
    # numpy axis 2 = x, 1 = y, 0 = z
    for axis, hh in ((2, h[0]), (1, h[1]), (0, h[2])):
        p1 = np.roll(phi, -1, axis=axis)
        m1 = np.roll(phi, 1, axis=axis)
        p2 = np.roll(phi, -2, axis=axis)
        m2 = np.roll(phi, 2, axis=axis)
        out.append(-(4.0 / 3.0) * (p1 - m1) / (2.0 * hh) + (1.0 / 3.0) * (p2 - m2) / (4.0 * hh))
    return tuple(out)
