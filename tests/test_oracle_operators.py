"""Pins of the oracle's grid operators against closed forms, brute force and
library routines (not against the oracle itself)."""
import math

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

from oracle import exact
from oracle import operators as op


def _cc(n, h, lo=0.0):
    return lo + (np.arange(n) + 0.5) * h


def test_hierarchy_sizes():
    g = op.Grid(32, 32, 32, 1 / 16, 1 / 16, 1 / 16, "dirichlet")
    assert [l.shape[0] for l in op.build_hierarchy(g, 4)] == [32, 16, 8, 4]
    for n, want in ((256, [256, 128, 64, 32, 16, 8, 4]), (48, [48, 24, 12, 6]),
                    (96, [96, 48, 24, 12, 6]), (128, [128, 64, 32, 16, 8, 4]),
                    (10, [10]), (6, [6])):
        g = op.Grid(n, n, n, 1.0 / n, 1.0 / n, 1.0 / n, "periodic")
        lv = op.build_hierarchy(g, 4)
        assert [l.shape[0] for l in lv] == want
        assert all(abs(l.h[0] - 2 ** l.level / n) < 1e-15 for l in lv)


def test_laplacian_quadratic_dirichlet_closed_form():
    """u = x^2 with exact face data: M u = 2 inside; at the x-boundary cells the
    linear-extrapolation ghost 2g - u_adj misses the true ghost value by
    -h^2/2, so M u = 2 - 1/2 = 1.5 there (closed form)."""
    n = 8
    h = 1.0 / n
    x = _cc(n, h)
    u = np.broadcast_to(x[None, None, :] ** 2, (n, n, n)).copy()
    xf = (0.0, 1.0)
    faces = (np.full((n, n), xf[0] ** 2), np.full((n, n), xf[1] ** 2),
             u[:, 0, :].copy(), u[:, -1, :].copy(), u[0, :, :].copy(), u[-1, :, :].copy())
    Mu = op.apply_M(u, (h, h, h), "dirichlet", faces)
    # y and z faces carry the field's own value at the face (x^2 does not vary in y, z)
    want = np.full((n, n, n), 2.0)
    want[:, :, 0] = 1.5
    want[:, :, -1] = 1.5
    np.testing.assert_allclose(Mu, want, rtol=0, atol=1e-11)


@pytest.mark.parametrize("m", [(1, 0, 0), (2, 3, 1), (4, 4, 4), (0, 5, 7)])
def test_laplacian_periodic_fourier_eigenmode(m):
    """cos(2 pi (m . x)) is an eigenvector of the periodic 7-point operator with
    eigenvalue -sum_d 4 sin^2(pi m_d / n_d) / h_d^2."""
    nx, ny, nz = 8, 12, 10
    hx, hy, hz = 0.3, 0.2, 0.25
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    k = np.arange(nz)[:, None, None]
    mx, my, mz = m
    u = np.cos(2 * math.pi * (mx * i / nx + my * j / ny + mz * k / nz)) + 0 * (i + j + k)
    lam = -(4 * math.sin(math.pi * mx / nx) ** 2 / hx ** 2 + 4 * math.sin(math.pi * my / ny) ** 2 / hy ** 2
            + 4 * math.sin(math.pi * mz / nz) ** 2 / hz ** 2)
    np.testing.assert_allclose(op.apply_M(u, (hx, hy, hz), "periodic"), lam * u, atol=1e-10)


@pytest.mark.parametrize("m", [(1, 1, 1), (3, 1, 2), (8, 8, 8), (8, 1, 5)])
def test_laplacian_dirichlet_dst_eigenmode(m):
    """sin(pi m (i + 1/2) / n) per axis is an eigenvector of the homogeneous
    Dirichlet operator (ghost = -u_adj) with eigenvalue -sum 4 sin^2(pi m/2n)/h^2;
    m = n is the checkerboard with eigenvalue -Lambda."""
    n = 8
    h = (0.1, 0.15, 0.2)
    i = np.arange(n)
    mx, my, mz = m
    u = (np.sin(math.pi * mz * (i + 0.5) / n)[:, None, None]
         * np.sin(math.pi * my * (i + 0.5) / n)[None, :, None]
         * np.sin(math.pi * mx * (i + 0.5) / n)[None, None, :])
    lam = -sum(4 * math.sin(math.pi * mm / (2 * n)) ** 2 / hh ** 2 for mm, hh in zip(m, h))
    np.testing.assert_allclose(op.apply_M(u, h, "dirichlet"), lam * u, atol=1e-9)


@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
def test_laplacian_matches_cellwise_dense_matrix(bc):
    rng = np.random.default_rng(0)
    shape = (4, 6, 5)
    h = (0.3, 0.2, 0.7)
    A = exact.dense_matrix(shape, h, bc)
    u = rng.standard_normal(shape)
    np.testing.assert_allclose(op.apply_M(u, h, bc), (A @ u.ravel()).reshape(shape), atol=1e-11)
    # affine part of the Dirichlet operator: M u - A u = 2 g / h^2 on boundary cells
    if bc == "dirichlet":
        faces = tuple(rng.standard_normal(s) for s in
                      ((4, 6), (4, 6), (4, 5), (4, 5), (6, 5), (6, 5)))
        diff = op.apply_M(u, h, bc, faces) - op.apply_M(u, h, bc)
        want = np.zeros(shape)
        want[:, :, 0] += 2 * faces[0] / h[0] ** 2
        want[:, :, -1] += 2 * faces[1] / h[0] ** 2
        want[:, 0, :] += 2 * faces[2] / h[1] ** 2
        want[:, -1, :] += 2 * faces[3] / h[1] ** 2
        want[0, :, :] += 2 * faces[4] / h[2] ** 2
        want[-1, :, :] += 2 * faces[5] / h[2] ** 2
        np.testing.assert_allclose(diff, want, atol=1e-10)


def test_restriction_constants_linear_and_mean():
    rng = np.random.default_rng(1)
    n = 8
    h = 1.0 / n
    x = _cc(n, h)
    X = np.broadcast_to(x[None, None, :], (n, n, n))
    Z = np.broadcast_to(x[:, None, None], (n, n, n))
    lin = 3.0 * X - 2.0 * Z + 0.5
    xc = _cc(n // 2, 2 * h)
    want = (3.0 * xc[None, None, :] - 2.0 * xc[:, None, None] + 0.5) + 0 * np.zeros((4, 4, 4))
    np.testing.assert_allclose(op.restrict(lin), want, atol=1e-14)
    np.testing.assert_allclose(op.restrict(np.full((n, n, n), 7.0)), 7.0)
    r = rng.standard_normal((n, n, n))
    assert abs(op.restrict(r).mean() - r.mean()) < 1e-15
    # brute force on one coarse cell
    c = op.restrict(r)[1, 2, 3]
    assert abs(c - r[2:4, 4:6, 6:8].sum() / 8) < 1e-15


def _trilinear_reference(e, bc):
    """Prolongation by scipy's trilinear interpolation on a ghost-extended grid:
    periodic images, or odd reflection (the error vanishes on the boundary)."""
    nz, ny, nx = e.shape
    if bc == "periodic":
        ext = np.pad(e, 1, mode="wrap")
    else:
        ext = np.pad(e, 1, mode="constant")
        ext[:, :, 0] = -ext[:, :, 1]
        ext[:, :, -1] = -ext[:, :, -2]
        ext[:, 0, :] = -ext[:, 1, :]
        ext[:, -1, :] = -ext[:, -2, :]
        ext[0, :, :] = -ext[1, :, :]
        ext[-1, :, :] = -ext[-2, :, :]
    # coarse centres at index + 0.5 in coarse units, ghosts at -0.5 and n + 0.5
    zc = np.arange(-1, nz + 1) + 0.5
    yc = np.arange(-1, ny + 1) + 0.5
    xc = np.arange(-1, nx + 1) + 0.5
    interp = RegularGridInterpolator((zc, yc, xc), ext, method="linear")
    zf = (np.arange(2 * nz) + 0.5) / 2
    yf = (np.arange(2 * ny) + 0.5) / 2
    xf = (np.arange(2 * nx) + 0.5) / 2
    Zf, Yf, Xf = np.meshgrid(zf, yf, xf, indexing="ij")
    return interp(np.stack([Zf, Yf, Xf], axis=-1))


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_prolongation_is_trilinear_interpolation(bc):
    rng = np.random.default_rng(2)
    e = rng.standard_normal((4, 6, 5))
    np.testing.assert_allclose(op.prolong(e, bc), _trilinear_reference(e, bc), atol=1e-13)


def test_prolongation_weights_and_linear_fields():
    # the weights of one fine cell sum to 1: constants map to constants (periodic)
    np.testing.assert_allclose(op.prolong(np.full((4, 4, 4), 3.0), "periodic"), 3.0)
    # a single coarse unit impulse gives 27/64 on its children, 9/64, 3/64, 1/64 around
    e = np.zeros((4, 4, 4))
    e[1, 1, 1] = 1.0
    p = op.prolong(e, "periodic")
    assert abs(p[2, 2, 2] - 27 / 64) < 1e-15  # child (0,0,0) of the impulse
    assert abs(p[1, 2, 2] - 9 / 64) < 1e-15   # below: z-face neighbour's child
    assert abs(p[1, 1, 2] - 3 / 64) < 1e-15
    assert abs(p[1, 1, 1] - 1 / 64) < 1e-15
    assert abs(p.sum() - 8.0) < 1e-13  # each coarse value spreads a total weight of 8
