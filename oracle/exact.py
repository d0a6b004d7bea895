"""The exact discrete solution u* of M u = f by direct methods (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The RKL-multigrid iteration converges to the unique solution of the
cell-centred 7-point system (Sec. 2.2.1 eq. discrete_laplace_3D with the
ghosts of Sec. 2.3).  That solution has a plain definition, computed here by
routes that share nothing with the iteration:

* periodic (eq. periodic, source mean removed per eq. source_modification):
  FFT diagonalisation with the discrete symbol -sum_d 4 sin^2(pi k_d/n_d)/h_d^2,
  the k = 0 mode set to zero (zero-mean gauge);
* Dirichlet (eq. solution_ghost): the homogeneous operator (ghost = -u_adj) is
  diagonalised by the DST-II basis sin(pi k (i+1/2)/n) with eigenvalues
  -4 sin^2(pi k / (2n))/h^2; the boundary values enter as the right-hand-side
  terms 2 g / h_d^2 of the boundary cells;
* any boundary type, tiny grids: a dense matrix assembled cell by cell and
  numpy.linalg (lstsq with a zero-mean row for the singular periodic case).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft


def _symbol_periodic(shape, h):
    nz, ny, nx = shape
    hx, hy, hz = h
    kx = np.arange(nx // 2 + 1)
    ky = np.arange(ny)
    kz = np.arange(nz)
    sx = 4.0 * np.sin(math.pi * kx / nx) ** 2 / (hx * hx)
    sy = 4.0 * np.sin(math.pi * ky / ny) ** 2 / (hy * hy)
    sz = 4.0 * np.sin(math.pi * kz / nz) ** 2 / (hz * hz)
    return -(sz[:, None, None] + sy[None, :, None] + sx[None, None, :])


def solve_periodic_fft(f, h, workers=-1):
    """u* for the periodic problem: the mean of f is removed, u* has zero mean."""
    f = np.asarray(f, dtype=np.float64)
    fh = sfft.rfftn(f, workers=workers)
    sym = _symbol_periodic(f.shape, h)
    sym[0, 0, 0] = 1.0
    fh /= sym
    fh[0, 0, 0] = 0.0
    return sfft.irfftn(fh, s=f.shape, workers=workers)


def dirichlet_rhs(f, h, faces):
    """Right-hand side with the boundary terms moved over: f - B g, where the
    boundary cell of face d gains 2 g / h_d^2 from its ghost 2g - u_adj."""
    hx, hy, hz = h
    rhs = np.array(f, dtype=np.float64, copy=True)
    if faces is None:
        return rhs
    gxm, gxp, gym, gyp, gzm, gzp = faces
    rhs[:, :, 0] -= 2.0 * np.asarray(gxm) / (hx * hx)
    rhs[:, :, -1] -= 2.0 * np.asarray(gxp) / (hx * hx)
    rhs[:, 0, :] -= 2.0 * np.asarray(gym) / (hy * hy)
    rhs[:, -1, :] -= 2.0 * np.asarray(gyp) / (hy * hy)
    rhs[0, :, :] -= 2.0 * np.asarray(gzm) / (hz * hz)
    rhs[-1, :, :] -= 2.0 * np.asarray(gzp) / (hz * hz)
    return rhs


def solve_dirichlet_dst(f, h, faces=None, workers=-1):
    """u* for the Dirichlet problem by a 3-D DST-II diagonalisation."""
    rhs = dirichlet_rhs(f, h, faces)
    nz, ny, nx = rhs.shape
    hx, hy, hz = h
    c = sfft.dstn(rhs, type=2, workers=workers)
    lx = 4.0 * np.sin(math.pi * np.arange(1, nx + 1) / (2.0 * nx)) ** 2 / (hx * hx)
    ly = 4.0 * np.sin(math.pi * np.arange(1, ny + 1) / (2.0 * ny)) ** 2 / (hy * hy)
    lz = 4.0 * np.sin(math.pi * np.arange(1, nz + 1) / (2.0 * nz)) ** 2 / (hz * hz)
    c /= -(lz[:, None, None] + ly[None, :, None] + lx[None, None, :])
    return sfft.idstn(c, type=2, workers=workers)


def dense_matrix(shape, h, bc):
    """The homogeneous operator as a dense matrix, built one cell at a time.

    Row of cell (k, j, i): -2 sum_d h_d^-2 on the diagonal and h_d^-2 per face
    neighbour; periodic neighbours wrap; a Dirichlet neighbour outside the box
    is the ghost -u_adj, i.e. it subtracts h_d^-2 from the diagonal.
    """
    nz, ny, nx = shape
    hx, hy, hz = h
    N = nx * ny * nz
    A = np.zeros((N, N))

    def idx(k, j, i):
        return (k * ny + j) * nx + i

    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                row = idx(k, j, i)
                for (dk, dj, di, hh, n, pos) in ((0, 0, -1, hx, nx, i), (0, 0, 1, hx, nx, i),
                                                 (0, -1, 0, hy, ny, j), (0, 1, 0, hy, ny, j),
                                                 (-1, 0, 0, hz, nz, k), (1, 0, 0, hz, nz, k)):
                    w = 1.0 / (hh * hh)
                    A[row, row] -= 2.0 * w / 2.0  # half of the -2/h^2 per direction
                    q = pos + (di + dj + dk)
                    if 0 <= q < n:
                        A[row, idx(k + dk, j + dj, i + di)] += w
                    elif bc == "periodic":
                        A[row, idx((k + dk) % nz, (j + dj) % ny, (i + di) % nx)] += w
                    else:
                        A[row, row] -= w
    return A


def solve_dense(f, h, bc, faces=None):
    """u* from the dense matrix: Dirichlet by numpy.linalg.solve, periodic by
    least squares on the system augmented with the zero-mean row."""
    f = np.asarray(f, dtype=np.float64)
    shape = f.shape
    A = dense_matrix(shape, h, bc)
    if bc == "periodic":
        rhs = (f - f.mean()).ravel()
        Aa = np.vstack([A, np.ones((1, A.shape[1]))])
        ra = np.concatenate([rhs, [0.0]])
        u = np.linalg.lstsq(Aa, ra, rcond=None)[0]
    else:
        rhs = dirichlet_rhs(f, h, faces).ravel()
        u = np.linalg.solve(A, rhs)
    return u.reshape(shape)


def exact_solution(f, h, bc, faces=None, workers=-1):
    """u* by FFT (periodic) or DST-II (Dirichlet)."""
    if bc == "periodic":
        f = np.asarray(f, dtype=np.float64)
        return solve_periodic_fft(f - f.mean(), h, workers)
    return solve_dirichlet_dst(f, h, faces, workers)
