"""Pins of the oracle's two-dimensional problems (eqs. discrete_laplace_2D,
restriction_example_2D, prolongation_example_2D) against brute force, closed
forms and library routines.

A 2-D grid is a 3-D array with nz = 1 and hz = inf; the checks below build
their expected values in 2-D directly (hand loops, scipy interpolation and
sparse Kronecker sums), never from the 3-D operator.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.interpolate import RegularGridInterpolator

import workloads as W
from oracle import exact
from oracle import multigrid as mg
from oracle import operators as op
from oracle import rkl
from oracle import smoothers as sm

INF = float("inf")


def test_hierarchy_coarsens_x_and_y_only():
    g = op.grid2d(64, 32, 1 / 64, 1 / 32, "periodic")
    lv = op.build_hierarchy(g, 4)
    assert [l.shape for l in lv] == [(1, 32, 64), (1, 16, 32), (1, 8, 16), (1, 4, 8)]
    assert all(l.flat and math.isinf(l.h[2]) for l in lv)
    assert [l.h[0] for l in lv] == [2 ** l / 64 for l in range(4)]
    # Gershgorin bound of the 5-point operator: 4 (hx^-2 + hy^-2)
    assert lv[0].lam == 4.0 * (64 ** 2 + 32 ** 2)


def _five_point_loop(u, hx, hy, bc, g=None):
    """Eq. discrete_laplace_2D written out cell by cell; Dirichlet ghosts
    2 g - u with g the face value (g = None: homogeneous)."""
    ny, nx = u.shape
    out = np.zeros_like(u)
    for j in range(ny):
        for i in range(nx):
            def val(jj, ii, face):
                if 0 <= jj < ny and 0 <= ii < nx:
                    return u[jj, ii]
                if bc == "periodic":
                    return u[jj % ny, ii % nx]
                gv = 0.0 if g is None else g[face][jj if face < 2 else ii]
                return 2.0 * gv - u[j, i]
            out[j, i] = ((val(j, i - 1, 0) - 2 * u[j, i] + val(j, i + 1, 1)) / hx ** 2
                         + (val(j - 1, i, 2) - 2 * u[j, i] + val(j + 1, i, 3)) / hy ** 2)
    return out


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_five_point_operator_brute_force(bc):
    rng = np.random.default_rng(3)
    ny, nx, hx, hy = 7, 9, 0.3, 0.17
    u = rng.standard_normal((ny, nx))
    g = None
    faces = None
    if bc == "dirichlet":
        g = [rng.standard_normal(ny), rng.standard_normal(ny), rng.standard_normal(nx), rng.standard_normal(nx)]
        faces = (g[0][None, :], g[1][None, :], g[2][None, :], g[3][None, :],
                 rng.standard_normal((ny, nx)), rng.standard_normal((ny, nx)))  # z faces carry no weight
    Mu = op.apply_M(u[None], (hx, hy, INF), bc, faces)[0]
    np.testing.assert_allclose(Mu, _five_point_loop(u, hx, hy, bc, g), rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_five_point_eigenmodes(bc):
    """Periodic: cos(2 pi kx x) cos(2 pi ky y) with eigenvalue
    -(4 sin^2(pi kx/nx)/hx^2 + 4 sin^2(pi ky/ny)/hy^2); Dirichlet (homogeneous):
    sin(pi kx x) sin(pi ky y) on cell centres with 4 sin^2(pi k/(2n))/h^2."""
    nx, ny, kx, ky = 24, 16, 3, 2
    hx, hy = 1.0 / nx, 1.0 / ny
    x = (np.arange(nx) + 0.5) * hx
    y = (np.arange(ny) + 0.5) * hy
    if bc == "periodic":
        u = np.cos(2 * math.pi * kx * x)[None, :] * np.cos(2 * math.pi * ky * y)[:, None]
        lam = 4 * math.sin(math.pi * kx / nx) ** 2 / hx ** 2 + 4 * math.sin(math.pi * ky / ny) ** 2 / hy ** 2
    else:
        u = np.sin(math.pi * kx * x)[None, :] * np.sin(math.pi * ky * y)[:, None]
        lam = (4 * math.sin(math.pi * kx / (2 * nx)) ** 2 / hx ** 2
               + 4 * math.sin(math.pi * ky / (2 * ny)) ** 2 / hy ** 2)
    Mu = op.apply_M(u[None], (hx, hy, INF), bc, None)[0]
    np.testing.assert_allclose(Mu, -lam * u, atol=1e-10 * lam)


def test_restriction_four_point_average():
    """E = (e + f + g + h)/4 on each 2x2 block: brute force, conservation of the
    sum (times 4), exactness for a bilinear field."""
    rng = np.random.default_rng(5)
    r = rng.standard_normal((1, 12, 10))
    c = op.restrict(r, flat=True)
    assert c.shape == (1, 6, 5)
    for J in range(6):
        for I in range(5):
            want = (r[0, 2 * J, 2 * I] + r[0, 2 * J, 2 * I + 1] + r[0, 2 * J + 1, 2 * I] + r[0, 2 * J + 1, 2 * I + 1]) / 4
            assert abs(c[0, J, I] - want) < 1e-14
    assert abs(4 * c.sum() - r.sum()) < 1e-12
    h = 0.1
    x = (np.arange(10) + 0.5) * h
    y = (np.arange(12) + 0.5) * h
    f = 2.0 + 3.0 * x[None, :] - 1.5 * y[:, None]
    X = (np.arange(5) + 0.5) * 2 * h
    Y = (np.arange(6) + 0.5) * 2 * h
    np.testing.assert_allclose(op.restrict(f[None], flat=True)[0], 2.0 + 3.0 * X[None, :] - 1.5 * Y[:, None],
                               atol=1e-13)


def _pad_reference(e2, bc):
    """Ghost ring around a (ny, nx) coarse field built with numpy's own
    padding: periodic wrap, or the odd extension (-u) of a homogeneous
    Dirichlet boundary (corner ghosts then come out as +u)."""
    if bc == "periodic":
        return np.pad(e2, 1, mode="wrap")
    p = np.pad(e2, 1, mode="symmetric")
    p[0, :] *= -1
    p[-1, :] *= -1
    p[:, 0] *= -1
    p[:, -1] *= -1
    return p


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_prolongation_is_bilinear_interpolation(bc):
    """Eq. prolongation_example_2D: (9A + 3B + 3C + D)/16 at a fine centre is
    scipy's bilinear interpolation of the ghost-extended coarse field."""
    rng = np.random.default_rng(8)
    ny, nx = 6, 5
    H = 1.0
    e = rng.standard_normal((1, ny, nx))
    p = _pad_reference(e[0], bc)
    X = (np.arange(-1, nx + 1) + 0.5) * H
    Y = (np.arange(-1, ny + 1) + 0.5) * H
    interp = RegularGridInterpolator((Y, X), p, method="linear")
    xf = (np.arange(2 * nx) + 0.5) * H / 2
    yf = (np.arange(2 * ny) + 0.5) * H / 2
    YY, XX = np.meshgrid(yf, xf, indexing="ij")
    want = interp(np.stack([YY.ravel(), XX.ravel()], axis=1)).reshape(2 * ny, 2 * nx)
    got = op.prolong(e, bc, flat=True)
    assert got.shape == (1, 2 * ny, 2 * nx)
    np.testing.assert_allclose(got[0], want, atol=1e-13)


def _laplacian_2d_sparse(nx, ny, hx, hy, bc):
    """Kronecker sum of 1-D second differences (independent of the oracle)."""
    def d1(n, h):
        main = -2.0 * np.ones(n)
        if bc == "dirichlet":
            main[0] -= 1.0
            main[-1] -= 1.0
        m = sp.diags([np.ones(n - 1), main, np.ones(n - 1)], [-1, 0, 1], format="lil")
        if bc == "periodic":
            m[0, n - 1] += 1.0
            m[n - 1, 0] += 1.0
        return m.tocsr() / (h * h)
    return sp.kron(sp.identity(ny), d1(nx, hx)) + sp.kron(d1(ny, hy), sp.identity(nx))


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_exact_solvers_in_2d(bc):
    """The FFT / DST solvers on (1, ny, nx) against a sparse direct solve of the
    5-point system (Dirichlet with face data folded into the right-hand side
    by hand)."""
    rng = np.random.default_rng(11)
    ny, nx, hx, hy = 12, 20, 0.05, 0.08
    f = rng.standard_normal((ny, nx))
    A = _laplacian_2d_sparse(nx, ny, hx, hy, bc)
    faces = None
    if bc == "periodic":
        f -= f.mean()
        # pin the null space: solve with the zero-mean constraint appended
        n = nx * ny
        Ab = sp.vstack([sp.hstack([A, np.ones((n, 1))]), sp.hstack([np.ones((1, n)), sp.csr_matrix((1, 1))])])
        want = spla.spsolve(Ab.tocsc(), np.concatenate([f.ravel(), [0.0]]))[:n].reshape(ny, nx)
    else:
        g = [rng.standard_normal(ny), rng.standard_normal(ny), rng.standard_normal(nx), rng.standard_normal(nx)]
        rhs = f.copy()
        rhs[:, 0] -= 2 * g[0] / hx ** 2
        rhs[:, -1] -= 2 * g[1] / hx ** 2
        rhs[0, :] -= 2 * g[2] / hy ** 2
        rhs[-1, :] -= 2 * g[3] / hy ** 2
        want = spla.spsolve(A.tocsc(), rhs.ravel()).reshape(ny, nx)
        faces = (g[0][None, :], g[1][None, :], g[2][None, :], g[3][None, :], np.zeros((ny, nx)), np.zeros((ny, nx)))
    got = exact.exact_solution(f[None], (hx, hy, INF), bc, faces)[0]
    np.testing.assert_allclose(got, want, atol=1e-10 * np.abs(want).max())


def test_schedule_and_spectrum_ignore_z():
    """The accelerated schedule of a 2-D level walks k from n/2 with n the
    smaller of nx, ny (not nz = 1), and its stage counts reach Round(2.4048
    n/pi - 1/2) at k = 1 for theta = 1 on a square Dirichlet level (eq.
    sk_optimal with x_k = cos(k pi / n))."""
    n = 32
    g = op.grid2d(n, n, 1 / n, 1 / n, "dirichlet")
    lv = op.build_hierarchy(g, 4)[0]
    sched = rkl.accelerated_schedule(lv, 1.0)
    assert len(sched) > 3 and sched[0] == 1
    assert sched[-1] == rkl.s_k_opt_1d(1, n)
    # the diagonal (k, k) mode of the 5-point operator: x_k = cos(k pi / n)
    for k in (1, 3, 7):
        x = 1.0 - lv.dt_par * rkl.mode_eigenvalue(lv, k)
        assert abs(x - math.cos(k * math.pi / n)) < 1e-12
    gp = op.grid2d(48, 16, 1 / 48, 1 / 16, "periodic")
    lp = op.build_hierarchy(gp, 4)[0]
    assert abs(rkl.mode_eigenvalue(lp, 1) - min(4 * math.sin(math.pi / 48) ** 2 * 48 ** 2,
                                                4 * math.sin(math.pi / 16) ** 2 * 16 ** 2)) < 1e-9


def test_gsrb_sweep_2d_brute_force():
    """One red-black pass in 2-D against a cell-by-cell loop with the 5-point
    diagonal 2 (hx^-2 + hy^-2) plus h^-2 for each Dirichlet face."""
    rng = np.random.default_rng(2)
    ny, nx, hx, hy = 6, 8, 0.2, 0.3
    u = rng.standard_normal((ny, nx))
    b = rng.standard_normal((ny, nx))
    w = 1.3
    got = sm.gsrb_sweep(u[None], b[None], (hx, hy, INF), "dirichlet", None, w)[0]
    v = u.copy()
    for colour in (0, 1):
        old = v.copy()
        Mu = _five_point_loop(old, hx, hy, "dirichlet")
        for j in range(ny):
            for i in range(nx):
                if (i + j) % 2 != colour:
                    continue
                d = 2 / hx ** 2 + 2 / hy ** 2 + (1 / hx ** 2) * ((i == 0) + (i == nx - 1)) \
                    + (1 / hy ** 2) * ((j == 0) + (j == ny - 1))
                v[j, i] = old[j, i] + w * (Mu[j, i] - b[j, i]) / d
    np.testing.assert_allclose(got, v, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("smoother", ["rkl", "gsrb"])
def test_2d_multigrid_solve_reaches_exact(bc, smoother):
    p = W.problem_2d(64, 48, bc, seed=4)
    g = op.grid2d(p.shape[2], p.shape[1], p.h[0], p.h[1], bc)
    u, st = mg.solve(p.rho, g, mg.Options(tol=1e-10, smoother=smoother), faces=p.faces)
    assert st.status == mg.STATUS_OK and st.rel_res <= 1e-10 and st.cycles <= 14
    # per-cycle reduction of a working V-cycle on the 5-point operator
    rates = [b / a for a, b in zip(st.history, st.history[1:]) if a > 0]
    assert max(rates[1:]) < 0.2
    us = exact.exact_solution(4 * math.pi * p.rho, p.h, bc, p.faces)
    assert np.abs(u - us).max() / np.abs(us).max() < 1e-8


def test_acceleration_2d():
    """Eq. 4thorder_acceleration in 2-D: exact on a linear field with its face
    values (Dirichlet), fourth order on a periodic sine, g_z = 0."""
    from oracle import gradient
    nx, ny = 12, 10
    hx, hy = 0.1, 0.2
    x = (np.arange(nx) + 0.5) * hx
    y = (np.arange(ny) + 0.5) * hy
    phi = (1.0 + 2.0 * x[None, :] - 3.0 * y[:, None])[None]
    X1 = nx * hx
    Y1 = ny * hy
    faces = ((1.0 - 3.0 * y)[None, :], (1.0 + 2.0 * X1 - 3.0 * y)[None, :],
             (1.0 + 2.0 * x)[None, :], (1.0 + 2.0 * x - 3.0 * Y1)[None, :], np.zeros((ny, nx)), np.zeros((ny, nx)))
    gx, gy, gz = gradient.acceleration(phi, (hx, hy, INF), "dirichlet", faces)
    np.testing.assert_allclose(gx, -2.0, atol=1e-12)
    np.testing.assert_allclose(gy, 3.0, atol=1e-12)
    assert gz.shape == phi.shape and not gz.any()
    errs = []
    for n in (16, 32):
        xs = (np.arange(n) + 0.5) / n
        ph = (np.sin(2 * math.pi * xs)[None, :] * np.cos(2 * math.pi * xs)[:, None])[None]
        gx, gy, gz = gradient.acceleration(ph, (1 / n, 1 / n, INF), "periodic")
        want = -2 * math.pi * np.cos(2 * math.pi * xs)[None, :] * np.cos(2 * math.pi * xs)[:, None]
        errs.append(np.abs(gx[0] - want).max())
        assert not gz.any()
    assert 14.0 < errs[0] / errs[1] < 18.0


def test_smooth_disc_workload_second_order():
    """The smooth 2-D density's closed-form potential solves the continuous
    problem: the exact discrete solutions approach it at second order."""
    errs = []
    for n in (32, 64, 128):
        p = W.smooth_disc(n)
        us = exact.exact_solution(4 * math.pi * p.rho, p.h, "dirichlet", p.faces)
        errs.append(np.sqrt(np.mean((us - p.phi_exact) ** 2)))
    for a, b in zip(errs, errs[1:]):
        assert 3.6 < a / b < 4.4


def test_float64_residual_floor_of_the_2d_4096_field():
    """The benchmark's 2-D field (4096^2 periodic blobs, seed 6): its exact
    discrete solution u* (FFT), rounded to float64, has a relative residual
    ||M u* - f|| / ||f|| above 1e-10, which no float64 iteration can reliably
    beat; the floor grows about fourfold per doubling of n (eps Lambda
    ||u|| / ||f|| with Lambda = 8 n^2)."""
    floors = []
    for n in (1024, 2048, 4096):
        p = W.gaussian_blobs_2d(n, n, nblobs=32, seed=6)
        f = 4 * math.pi * (p.rho - p.rho.mean())
        us = exact.exact_solution(4 * math.pi * p.rho, p.h, "periodic")
        r = op.apply_M(us.reshape(1, n, n), (p.h[0], p.h[1], math.inf), "periodic").reshape(n, n) - f
        floors.append(np.linalg.norm(r) / np.linalg.norm(f))
    assert 1e-10 < floors[-1] < 3e-10
    for a, b in zip(floors, floors[1:]):
        assert 3.0 < b / a < 5.0
