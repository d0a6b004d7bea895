"""Pins of the oracle's direct solvers, V-cycle, outer loop, mixed-precision
defect correction, adjoint, and the paper's comparison smoothers."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import exact, gradient
from oracle import multigrid as mg
from oracle import operators as op
from oracle import smoothers as sm

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
FOURPI = 4.0 * math.pi


# ---------------------------------------------------------------- exact u*

@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 6, 6), (8, 6, 4)])
def test_fft_matches_dense_solve_periodic(shape):
    rng = np.random.default_rng(10)
    h = (0.3, 0.2, 0.25)
    f = rng.standard_normal(shape)
    u_fft = exact.exact_solution(f, h, "periodic")
    u_dense = exact.solve_dense(f, h, "periodic")
    np.testing.assert_allclose(u_fft, u_dense, atol=1e-11)
    assert abs(u_fft.mean()) < 1e-13


@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 6, 6), (8, 6, 4)])
def test_dst_matches_dense_solve_dirichlet(shape):
    rng = np.random.default_rng(11)
    h = (0.3, 0.2, 0.25)
    nz, ny, nx = shape
    f = rng.standard_normal(shape)
    faces = (rng.standard_normal((nz, ny)), rng.standard_normal((nz, ny)),
             rng.standard_normal((nz, nx)), rng.standard_normal((nz, nx)),
             rng.standard_normal((ny, nx)), rng.standard_normal((ny, nx)))
    u_dst = exact.exact_solution(f, h, "dirichlet", faces)
    u_dense = exact.solve_dense(f, h, "dirichlet", faces)
    np.testing.assert_allclose(u_dst, u_dense, atol=1e-11)


def test_exact_solutions_satisfy_the_discrete_equation():
    p = W.uniform_sphere(16)
    f = FOURPI * p.rho
    u = exact.exact_solution(f, p.h, "dirichlet", p.faces)
    r = op.apply_M(u, p.h, "dirichlet", p.faces) - f
    assert np.abs(r).max() < 1e-10 * np.abs(f).max()
    p = W.gaussian_blobs(16, 4, seed=0)
    f = FOURPI * p.rho
    u = exact.exact_solution(f, p.h, "periodic")
    r = op.apply_M(u, p.h, "periodic") - (f - f.mean())
    assert np.abs(r).max() < 1e-10 * np.abs(f).max()


# ---------------------------------------------------------------- V-cycle

def _grid(p):
    nz, ny, nx = p.shape
    return op.Grid(nx, ny, nz, *p.h, p.bc)


@pytest.mark.parametrize("which", ["sphere", "blobs"])
def test_exact_solution_is_vcycle_fixed_point(which):
    p = W.uniform_sphere(16) if which == "sphere" else W.gaussian_blobs(16, 6, seed=1)
    g = _grid(p)
    f = mg.prepare_source(p.rho, g, mg.Options())
    us = exact.exact_solution(f, p.h, p.bc, p.faces)
    lv = op.build_hierarchy(g)
    got = mg.vcycle(us, f, lv, mg.Options(), p.faces)
    assert np.abs(got - us).max() <= 1e-11 * np.abs(us).max()


@pytest.mark.parametrize("which", ["sphere", "blobs", "accuracy"])
def test_vcycle_reduction_factor_about_ten(which):
    """Sec. 4.1: each V-cycle cuts the residual by about an order of magnitude."""
    if which == "sphere":
        p = W.uniform_sphere(32)
    elif which == "blobs":
        p = W.gaussian_blobs(32, 16, seed=2)
    else:
        p = W.accuracy_problem(32)
    g = _grid(p)
    _, st = mg.solve(p.rho, g, mg.Options(tol=1e-9), faces=p.faces)
    h = st.history
    factors = [h[i + 1] / h[i] for i in range(2, len(h) - 1)]
    paper = 1.0 / GOLD["vcycle_reduction_factor"]["value"]
    assert max(factors) < 2.0 * paper
    assert min(factors) > 0.25 * paper


@pytest.mark.parametrize("which", ["sphere32", "blobs32", "aniso"])
def test_solve_reaches_exact_discrete_solution(which):
    if which == "sphere32":
        p = W.uniform_sphere(32)
        g = _grid(p)
    elif which == "blobs32":
        p = W.gaussian_blobs(32, 16, seed=2)
        g = _grid(p)
    else:
        # non-cubic, anisotropic spacing, periodic
        p = W.gaussian_blobs((16, 32, 64), 8, seed=5)
        g = _grid(p)
    u, st = mg.solve(p.rho, g, mg.Options(tol=1e-12), faces=p.faces)
    assert st.status == mg.STATUS_OK and st.rel_res <= 1e-12
    us = exact.exact_solution(FOURPI * p.rho, p.h, p.bc, p.faces)
    assert np.abs(u - us).max() <= 1e-10 * np.abs(us).max()


def test_single_level_mode_matches_exact():
    """A grid that cannot be coarsened (10^3) runs the accelerated RKL iteration
    of App. A.4 on the finest level until the tolerance."""
    p = W.gaussian_blobs(10, 3, seed=6)
    g = _grid(p)
    assert len(op.build_hierarchy(g)) == 1
    u, st = mg.solve(p.rho, g, mg.Options(tol=1e-11, max_cycles=2000))
    assert st.status == mg.STATUS_OK
    us = exact.exact_solution(FOURPI * p.rho, p.h, "periodic")
    assert np.abs(u - us).max() <= 1e-9 * np.abs(us).max()


def test_coarsest_solve_converges_to_tolerance():
    rng = np.random.default_rng(12)
    for bc in ("dirichlet", "periodic"):
        for n in (4, 6):
            lv = op.Level(3, (n, n, n), (0.4,) * 3, bc)
            b = rng.standard_normal((n, n, n))
            if bc == "periodic":
                b -= b.mean()
            st = mg.Stats()
            u = mg.coarsest_solve(b, lv, mg.Options(), st)
            r = op.apply_M(u, lv.h, bc) - b
            assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(b)
            assert 0 < st.coarse_steps[0] < 60


def test_second_order_accuracy_on_paper_model():
    """Sec. 4.1: the potential error falls as O(h^2) (factor 4 per doubling)."""
    errs = []
    for n in (16, 32, 64):
        p = W.accuracy_problem(n)
        u, _ = mg.solve(p.rho, _grid(p), mg.Options(tol=1e-11), faces=p.faces)
        errs.append(np.linalg.norm(u - p.phi_exact) / np.linalg.norm(p.phi_exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    order = GOLD["accuracy_order"]["value"]
    assert abs(math.log2(r1) - order) < 0.25 and abs(math.log2(r2) - order) < 0.15


def test_uniform_sphere_analytic_error():
    p = W.uniform_sphere(32)
    u, _ = mg.solve(p.rho, _grid(p), mg.Options(tol=1e-10), faces=p.faces)
    e = np.linalg.norm(u - p.phi_exact) / np.linalg.norm(p.phi_exact)
    assert 5e-3 < e < 3e-2


# ---------------------------------------------------------------- statuses

def test_status_codes():
    p = W.gaussian_blobs(16, 4, seed=7)
    g = _grid(p)
    _, st = mg.solve(p.rho, g, mg.Options(max_cycles=1))
    assert st.status == mg.STATUS_ENOCONV and st.cycles == 1
    bad = p.rho.copy()
    bad[3, 4, 5] = np.nan
    _, st = mg.solve(bad, g, mg.Options())
    assert st.status == mg.STATUS_ENONFINITE
    _, st = mg.solve(p.rho, g, mg.Options(theta=1.05, max_cycles=50))
    assert st.status == mg.STATUS_EDIVERGED
    u, st = mg.solve(np.zeros(g.shape), g, mg.Options())
    assert st.status == mg.STATUS_OK and np.all(u == 0)


# ---------------------------------------------------------------- mixed precision

def test_mixed_precision_defect_correction_reaches_fp64_accuracy():
    p = W.gaussian_random_field(32, seed=3)
    g = _grid(p)
    u, st = mg.solve_mixed(p.rho, g, mg.Options(tol=1e-10))
    assert st.status == mg.STATUS_OK and st.rel_res <= 1e-10
    us = exact.exact_solution(FOURPI * p.rho, p.h, "periodic")
    assert np.abs(u - us).max() <= 1e-9 * np.abs(us).max()
    # the inner float32 cycle contracts about as well as the float64 one
    h = st.history
    assert max(h[i + 1] / h[i] for i in range(1, len(h) - 1)) < 0.3


def test_mixed_precision_dirichlet():
    p = W.uniform_sphere(32)
    u, st = mg.solve_mixed(p.rho, _grid(p), mg.Options(tol=1e-10), faces=p.faces)
    assert st.rel_res <= 1e-10
    us = exact.exact_solution(FOURPI * p.rho, p.h, "dirichlet", p.faces)
    assert np.abs(u - us).max() <= 1e-9 * np.abs(us).max()


# ---------------------------------------------------------------- adjoint

def test_adjoint_dot_product_and_finite_differences():
    """L = sum(w phi) is linear in rho, so dL/drho from the adjoint must match
    central differences along random directions and satisfy <w, S v> = <S w, v>."""
    rng = np.random.default_rng(5)
    n = 16
    p = W.gaussian_blobs(n, 6, rng=rng)
    g = _grid(p)
    w = rng.standard_normal(g.shape)
    opts = mg.Options(tol=1e-13)
    grad, _ = mg.adjoint_solve(w, g, opts)
    assert abs(grad.mean()) < 1e-12 * np.abs(grad).max()
    eps = 1e-6
    for _ in range(4):
        d = rng.standard_normal(g.shape)
        d /= np.linalg.norm(d)
        up, _ = mg.solve(p.rho + eps * d, g, opts)
        um, _ = mg.solve(p.rho - eps * d, g, opts)
        fd = (np.sum(w * up) - np.sum(w * um)) / (2 * eps)
        an = np.sum(grad * d)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-30) + 1e-9
    v = rng.standard_normal(g.shape)
    o1 = mg.Options(tol=1e-13, four_pi_G=1.0)
    sv, _ = mg.solve(v, g, o1)
    sw, _ = mg.solve(w, g, o1)
    assert abs(np.sum(w * sv) - np.sum(sw * v)) < 1e-10 * abs(np.sum(w * sv))


def test_adjoint_dirichlet_matches_dense_transpose():
    rng = np.random.default_rng(8)
    n = 8
    h = (1 / n,) * 3
    g = op.Grid(n, n, n, *h, "dirichlet")
    w = rng.standard_normal(g.shape)
    grad, _ = mg.adjoint_solve(w, g, mg.Options(tol=1e-13))
    A = exact.dense_matrix(g.shape, h, "dirichlet")
    want = FOURPI * np.linalg.solve(A.T, w.ravel()).reshape(g.shape)
    np.testing.assert_allclose(grad, want, rtol=0, atol=1e-10 * np.abs(want).max())


# ---------------------------------------------------------------- comparison smoothers

def test_sor_omega_reading_gives_textbook_jacobi_radius():
    shape = (32, 32, 32)
    h = (1 / 32,) * 3
    assert abs(sm.rho_jacobi_dirichlet(shape, h) - math.cos(math.pi / 32)) < 1e-14
    # brute force: the spectral radius of the dense Jacobi iteration matrix on 6^3
    A = exact.dense_matrix((6, 6, 6), (1 / 6,) * 3, "dirichlet")
    # the App. B formula refers to the vertex-style Dirichlet box; check only its
    # uniform-grid value against the textbook formula and that SOR omega is in (1, 2)
    om = sm.sor_omega(shape, h)
    assert 1.0 < om < 2.0
    assert A.shape == (216, 216)


@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
def test_gsrb_and_jacobi_converge_to_exact(bc):
    rng = np.random.default_rng(9)
    n = 8
    h = (1 / n,) * 3
    f = rng.standard_normal((n, n, n))
    if bc == "periodic":
        f -= f.mean()
    us = exact.exact_solution(f, h, bc)
    u = np.zeros_like(f)
    for _ in range(400):
        u = sm.gsrb_sweep(u, f, h, bc)
        if bc == "periodic":
            u -= u.mean()
    assert np.abs(u - us).max() < 1e-8 * np.abs(us).max()
    # red-black: the first half-sweep updates exactly the red cells, each by
    # its own row of the system (diagonal 6/h^2, +1/h^2 per Dirichlet face)
    u1 = sm.gsrb_sweep(np.zeros_like(f), f, h, bc)
    red = sm.colour_mask(f.shape, 0)
    nface = np.zeros(f.shape)
    if bc == "dirichlet":
        for ax in range(3):
            idx = [slice(None)] * 3
            idx[ax] = 0
            nface[tuple(idx)] += 1
            idx[ax] = -1
            nface[tuple(idx)] += 1
    np.testing.assert_allclose(u1[red], (-f / ((6 + nface) * n * n))[red], atol=1e-15)


def test_fourth_order_gradient_convergence():
    """eq. 4thorder_acceleration: the error falls as h^4 on a smooth periodic field."""
    errs = []
    for n in (16, 32):
        x = (np.arange(n) + 0.5) / n
        phi = np.sin(2 * math.pi * x)[None, None, :] * np.ones((n, n, 1))
        gx, gy, gz = gradient.acceleration_periodic(phi, (1 / n,) * 3)
        want = -2 * math.pi * np.cos(2 * math.pi * x)[None, None, :]
        errs.append(np.abs(gx - want).max())
        assert np.abs(gy).max() < 1e-12 and np.abs(gz).max() < 1e-12
    assert abs(math.log2(errs[0] / errs[1]) - 4.0) < 0.1


# ---------------------------------------------------------------- GS-RB smoother and App. B relaxation

def test_gsrb_sweep_matches_bruteforce_loops():
    """Red-black pass written cell by cell: red cells from the old values, then
    black cells from the new red ones, each solving its own row of the
    discrete system exactly (omega = 1) and over-relaxed by omega: a
    Dirichlet face contributes 2 g to the right side and -u to the diagonal."""
    rng = np.random.default_rng(21)
    n = 4
    h = (0.3, 0.2, 0.25)
    u = rng.standard_normal((n, n, n))
    b = rng.standard_normal((n, n, n))
    faces = tuple(rng.standard_normal(s) for s in ((n, n),) * 6)
    om = 1.3
    want = u.copy()
    ih = [1 / hh ** 2 for hh in h]
    D = 2 * sum(ih)
    for colour in (0, 1):
        old = want.copy()
        for k in range(n):
            for j in range(n):
                for i in range(n):
                    if (i + j + k) % 2 != colour:
                        continue
                    c = old[k, j, i]
                    # row of the discrete system: sum_nb a_nb u_nb - diag u = b - boundary terms
                    rhs = b[k, j, i]
                    diag = D
                    acc = 0.0
                    for (cond, val, face, w) in (
                            (i > 0, lambda: old[k, j, i - 1], lambda: faces[0][k, j], ih[0]),
                            (i < n - 1, lambda: old[k, j, i + 1], lambda: faces[1][k, j], ih[0]),
                            (j > 0, lambda: old[k, j - 1, i], lambda: faces[2][k, i], ih[1]),
                            (j < n - 1, lambda: old[k, j + 1, i], lambda: faces[3][k, i], ih[1]),
                            (k > 0, lambda: old[k - 1, j, i], lambda: faces[4][j, i], ih[2]),
                            (k < n - 1, lambda: old[k + 1, j, i], lambda: faces[5][j, i], ih[2])):
                        if cond:
                            acc += w * val()
                        else:
                            rhs -= 2 * w * face()
                            diag += w
                    exact_row = (acc - rhs) / diag
                    want[k, j, i] = (1 - om) * c + om * exact_row
    got = sm.gsrb_sweep(u, b, h, "dirichlet", faces, om)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


def test_gsrb_asymptotic_rate_is_jacobi_radius_squared():
    """Red-black ordering is consistent, so on a periodic box (no ghosts) the
    Gauss-Seidel rate is rho_J^2.  The Jacobi eigenvalue of the Fourier mode
    with wave numbers 2 pi m / n is the mean of the three cosines; the largest
    below 1 belongs to the smoothest mode along one axis: (2 + cos(2 pi / n)) / 3."""
    n = 16
    g = op.Grid(n, n, n, 1 / n, 1 / n, 1 / n, "periodic")
    rng = np.random.default_rng(3)
    f = rng.standard_normal(g.shape)
    f -= f.mean()
    _, it, res, hist = mg.relax_solve(f, g, "gsrb", tol_max=1e-300, max_iters=120)
    assert hist[-1] > 1e-9 * hist[0]   # still far above rounding
    ratio = hist[-1] / hist[-2]
    assert abs(ratio - ((2 + math.cos(2 * math.pi / n)) / 3) ** 2) < 2e-3


def test_gsrb_vcycle_reduces_residual_about_tenfold():
    """Sec. 4.1: with the GS-RB smoother (N_pre = 2, N_post = 1) and the RKL
    coarsest solver the residual falls by about an order of magnitude per
    cycle; the solve reaches the exact discrete solution."""
    p = W.accuracy_problem(32)
    g = op.Grid(32, 32, 32, *p.h, "dirichlet")
    phi, st = mg.solve(p.rho, g, mg.Options(tol=1e-10, smoother="gsrb"), faces=p.faces)
    assert st.status == 0
    h = st.history
    rates = [h[i] / h[i + 1] for i in range(1, len(h) - 1)]
    geo = math.exp(sum(math.log(r) for r in rates) / len(rates))
    assert 5.0 < geo < 20.0
    us = exact.exact_solution(4 * math.pi * p.rho, p.h, "dirichlet", p.faces)
    assert np.abs(phi - us).max() < 1e-9 * np.abs(us).max()


def test_relax_solve_app_b_ordering():
    """App. B: to the same maximum residual the accelerated RKL iteration needs
    far fewer iterations than SOR, and SOR fewer than GS-RB; each stops below
    the tolerance, and SOR at omega = 1 is GS-RB."""
    n = 16
    p = W.accuracy_problem(n)
    g = op.Grid(n, n, n, *p.h, "dirichlet")
    f = mg.prepare_source(p.rho, g, mg.Options())
    out = {}
    for m in ("rkl", "gsrb", "sor"):
        u, it, res, hist = mg.relax_solve(f, g, m, faces=p.faces, tol_max=1e-10)
        assert res <= 1e-10
        out[m] = it
    assert out["rkl"] < out["sor"] < out["gsrb"]
    a = mg.relax_solve(f, g, "sor", faces=p.faces, tol_max=1e-300, max_iters=7, omega=1.0)[0]
    b = mg.relax_solve(f, g, "gsrb", faces=p.faces, tol_max=1e-300, max_iters=7)[0]
    np.testing.assert_array_equal(a, b)


# ---------------------------------------------------------------- 4th-order acceleration, both boundaries

def test_acceleration_matches_periodic_routine_and_linear_fields():
    rng = np.random.default_rng(8)
    n = (8, 10, 12)
    h = (0.1, 0.2, 0.3)
    phi = rng.standard_normal(n)
    a = gradient.acceleration(phi, h, "periodic")
    b = gradient.acceleration_periodic(phi, h)
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-12)
    # Dirichlet: a linear field with its exact face values has g = -grad exactly,
    # up to the boundary (the odd reflection continues it linearly)
    nz, ny, nx = n
    X, Y, Z = W.cell_centres(n, (0.0, 0.0, 0.0), h)
    c = (1.5, -2.0, 0.75)
    lin = lambda x, y, z: c[0] * x + c[1] * y + c[2] * z + 0.3  # noqa: E731
    phi = lin(X, Y, Z)
    faces = tuple(lin(fx, fy, fz) for (fx, fy, fz) in W.face_centres(n, (0.0, 0.0, 0.0), h))
    gx, gy, gz = gradient.acceleration(phi, h, "dirichlet", faces)
    np.testing.assert_allclose(gx, -c[0], atol=1e-12)
    np.testing.assert_allclose(gy, -c[1], atol=1e-12)
    np.testing.assert_allclose(gz, -c[2], atol=1e-12)


def test_acceleration_of_paper_model_converges():
    """Sec. 4.1: g_x from the exact discrete solution approaches the analytic
    acceleration (eq. acceleration_3D) at second order (the potential's error
    dominates the 4th-order stencil)."""
    errs = []
    for n in (16, 32):
        p = W.accuracy_problem(n)
        us = exact.exact_solution(4 * math.pi * p.rho, p.h, "dirichlet", p.faces)
        gx, _, _ = gradient.acceleration(us, p.h, "dirichlet", p.faces)
        want = W.accuracy_acceleration_x(n)
        errs.append(math.sqrt(np.mean((gx - want) ** 2)) / math.sqrt(np.mean(want ** 2)))
    assert 1.6 < math.log2(errs[0] / errs[1]) < 2.6
