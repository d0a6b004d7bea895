"""The paper's own smoother (red-black Gauss-Seidel, Sec. 2.2.4) and the
single-level comparison of App. B on the GPU, against the oracle.

GS-RB / SOR passes are checked cell by cell (1e-12 relative, float64); the
V-cycle with the GS-RB smoother against the oracle's V-cycle (1e-11); solves
against the exact discrete solution; the App. B relaxation driver against the
oracle's iteration counts (equal up to a tie at the tolerance) and iterates.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import exact
from oracle import multigrid as omg
from oracle import operators as oop
from oracle import smoothers as osm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
FOURPI = 4.0 * math.pi


def _lib():
    import paper_2306_05332_amd as R
    return R


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rand_faces(rng, shape):
    nz, ny, nx = shape
    return tuple(rng.standard_normal(s) for s in ((nz, ny), (nz, ny), (nz, nx), (nz, nx), (ny, nx), (ny, nx)))


# one-pass strip kernel for the first four (ragged, odd periodic sizes
# included), one-colour passes for the tiny one
# ragged in x, y and z; the last two have many strips and a narrow x remainder
GSHAPES = [(20, 11, 130), (16, 16, 16), (40, 24, 64), (72, 130, 160), (9, 6, 5), (11, 100, 136), (9, 60, 20)]


@pytest.mark.parametrize("shape", GSHAPES)
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("omega", [1.0, 1.6])
def test_gsrb_passes_match_oracle(shape, bc, omega):
    R = _lib()
    rng = np.random.default_rng(31)
    h = (0.11, 0.07, 0.13)
    u0 = rng.standard_normal(shape)
    f = rng.standard_normal(shape) * 50
    faces = rand_faces(rng, shape) if bc == "dirichlet" else None
    want = u0
    for _ in range(3):
        want = osm.gsrb_sweep(want, f, h, bc, faces, omega)
    print(f"shape={shape} bc={bc} omega={omega}", flush=True)
    phi = cu(u0)
    R.gsrb_smooth(cu(f), phi, h, bc, omega=omega, n_iter=3, faces=R.pack_faces(faces) if faces else None)
    assert relmax(phi.cpu().numpy(), want) < 1e-12


@pytest.mark.parametrize("variant", ["strip5x1", "strip4x4", "strip8x4"])
@pytest.mark.parametrize("shape", [(20, 11, 130), (40, 24, 64), (11, 100, 136), (9, 60, 20)])
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_gsrb_passes_forced_strip_match_oracle(variant, shape, bc):
    """The one-pass GS-RB / SOR kernel in each strip shape it takes from the
    level's tuned tile (the five-row strips, whose interior strips pack their
    x remainders into shared wavefronts at nx = 136, and the 4 x 4 and 8 x 4
    strips), against the oracle's sweeps."""
    R = _lib()
    nz, ny, nx = shape
    target = 128 if (nx + ny) % 2 else 2048
    try:
        R.tune_set([{"nx": nx, "ny": ny, "nz": nz, "bc": bc, "prec": "fp64", "s": 2, "variant": variant,
                     "target": target}])
        rng = np.random.default_rng(41)
        h = (0.11, 0.07, 0.13)
        u0 = rng.standard_normal(shape)
        f = rng.standard_normal(shape) * 50
        want = u0
        for _ in range(3):
            want = osm.gsrb_sweep(want, f, h, bc, None, 1.6)
        print(f"variant={variant} target={target} shape={shape} bc={bc}", flush=True)
        phi = cu(u0)
        R.gsrb_smooth(cu(f), phi, h, bc, omega=1.6, n_iter=3)
        assert relmax(phi.cpu().numpy(), want) < 1e-12
    finally:
        R.tune_clear()
        R.install_default_tuning()


def _problem(which):
    if which == "sphere32":
        return W.uniform_sphere(32)
    if which == "blobs32":
        return W.gaussian_blobs(32, 16, seed=2)
    if which == "aniso":
        return W.gaussian_blobs((16, 32, 64), 8, seed=5)
    return W.accuracy_problem(32)


def _grid(p):
    nz, ny, nx = p.shape
    return oop.Grid(nx, ny, nz, *p.h, p.bc)


@pytest.mark.parametrize("which", ["sphere32", "blobs32", "aniso", "accuracy32"])
def test_gsrb_vcycle_matches_oracle(which):
    R = _lib()
    p = _problem(which)
    g = _grid(p)
    f = omg.prepare_source(p.rho, g, omg.Options())
    lv = oop.build_hierarchy(g)
    oo = omg.Options(smoother="gsrb")
    rng = np.random.default_rng(1)
    u0 = rng.standard_normal(p.shape) * 0.01
    want = omg.vcycle(u0, f, lv, oo, p.faces)
    want2 = omg.vcycle(want, f, lv, oo, p.faces)
    phi = cu(u0)
    faces = R.pack_faces(p.faces) if p.faces else None
    o = R.Options(smoother="gsrb")
    R.vcycle(cu(f), phi, p.h, p.bc, faces=faces, opts=o)
    assert relmax(phi.cpu().numpy(), want) < 1e-11
    R.vcycle(cu(f), phi, p.h, p.bc, faces=faces, opts=o)
    assert relmax(phi.cpu().numpy(), want2) < 1e-11


@pytest.mark.parametrize("which", ["sphere32", "blobs32", "accuracy32"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_gsrb_solve_reaches_exact(which, prec):
    R = _lib()
    p = _problem(which)
    faces = R.pack_faces(p.faces) if p.faces else None
    phi, st = R.solve(cu(p.rho), p.h, p.bc, faces=faces, opts=R.Options(tol=1e-10, smoother="gsrb", prec=prec))
    assert st.status == 0 and st.rel_res <= 1e-10
    us = exact.exact_solution(FOURPI * p.rho, p.h, p.bc, p.faces)
    assert relmax(phi.cpu().numpy(), us) < 1e-9
    if prec == "fp64":
        _, ost = omg.solve(p.rho, _grid(p), omg.Options(tol=1e-10, smoother="gsrb"), faces=p.faces)
        assert abs(ost.cycles - st.cycles) <= 1
        np.testing.assert_allclose(st.history[:4], ost.history[:4], rtol=1e-8)


def test_gsrb_batched_reaches_exact():
    R = _lib()
    probs = W.batch_blob_problems(seed=12, total=6, sizes=(32, 64))
    phis, stats = R.solve_batched([cu(p.rho) for p in probs], [p.h for p in probs], "periodic",
                                  opts=R.Options(tol=1e-10, prec="mixed", smoother="gsrb"))
    for p, phi, st in zip(probs, phis, stats):
        assert st.status == 0
        us = exact.exact_solution(FOURPI * p.rho, p.h, "periodic")
        assert relmax(phi.cpu().numpy(), us) < 1e-9


@pytest.mark.parametrize("method", ["rkl", "gsrb", "sor"])
@pytest.mark.parametrize("n", [16, 20])
def test_relax_solve_matches_oracle(method, n):
    """App. B driver: same iteration count as the oracle (up to a tie at the
    tolerance) and the same iterate."""
    R = _lib()
    p = W.accuracy_problem(n)
    g = _grid(p)
    f = omg.prepare_source(p.rho, g, omg.Options())
    u, it, res, hist = omg.relax_solve(f, g, method, faces=p.faces, tol_max=1e-10)
    phi, st = R.relax_solve(cu(f), p.h, "dirichlet", method, faces=R.pack_faces(p.faces), tol_max=1e-10)
    print(f"{method} n={n}: oracle {it} iterations, gpu {st.cycles}", flush=True)
    assert st.status == 0 and st.rel_res <= 1e-10
    assert abs(st.cycles - it) <= 1
    np.testing.assert_allclose(st.history[:5], hist[:5], rtol=1e-9)
    if st.cycles == it:
        assert relmax(phi.cpu().numpy(), u) < 1e-9
    us = exact.exact_solution(FOURPI * p.rho, p.h, "dirichlet", p.faces)
    assert relmax(phi.cpu().numpy(), us) < 1e-8


def test_relax_solve_periodic_and_statuses():
    R = _lib()
    rng = np.random.default_rng(4)
    n = 16
    f = rng.standard_normal((n, n, n))
    f -= f.mean()
    h = (1 / n,) * 3
    g = oop.Grid(n, n, n, *h, "periodic")
    u, it, res, hist = omg.relax_solve(f, g, "gsrb", tol_max=1e-8, check_every=4)
    phi, st = R.relax_solve(cu(f), h, "periodic", "gsrb", tol_max=1e-8, check_every=4)
    assert st.status == 0 and abs(st.cycles - it) <= 4
    phi, st = R.relax_solve(cu(f), h, "periodic", "gsrb", tol_max=1e-14, max_iters=10, raise_on_error=False)
    assert st.status == R.RKL_ENOCONV and st.cycles == 10


@pytest.mark.parametrize("n", [16, 32])
def test_relax_solve_fixed_s_opt_matches_oracle(n):
    """Single-level RKL with the fixed stage count of App. A.3 (s = -1 asks the
    library for it): the s the library reports (rkl_s_opt) equals the oracle's
    level rule, and the relaxation matches the oracle's with that s (iteration
    count up to a tie at the tolerance, the iterate, u*)."""
    R = _lib()
    from oracle import rkl as orkl
    p = W.accuracy_problem(n)
    g = _grid(p)
    f = omg.prepare_source(p.rho, g, omg.Options())
    s, _ = R.s_opt(p.shape, p.h, "dirichlet", tau_frac=0.9)
    assert s == orkl.s_opt_global(oop.build_hierarchy(g, 1 << 30)[0], 0.9)[0]
    u, it, res, hist = omg.relax_solve(f, g, "rkl", faces=p.faces, tol_max=1e-10, s=s, theta=0.9)
    phi, st = R.relax_solve(cu(f), p.h, "dirichlet", "rkl", faces=R.pack_faces(p.faces), s=-1, tol_max=1e-10)
    print(f"s_opt n={n}: s={s}, oracle {it} tau-steps, gpu {st.cycles}", flush=True)
    assert st.status == 0 and st.rel_res <= 1e-10
    assert abs(st.cycles - it) <= 1
    np.testing.assert_allclose(st.history[:5], hist[:5], rtol=1e-9)
    if st.cycles == it:
        assert relmax(phi.cpu().numpy(), u) < 1e-9
    us = exact.exact_solution(FOURPI * p.rho, p.h, "dirichlet", p.faces)
    assert relmax(phi.cpu().numpy(), us) < 1e-8
