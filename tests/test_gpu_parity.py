"""GPU (HIP, gfx950) path vs the CPU oracle, element by element, through the C ABI.

Tolerances (float64): a tau-step, residual or transfer agrees with the oracle to
1e-12 of the field's max norm (a few ulp per stage; the kernels contract to FMA
and multiply by 1/h^2 where the oracle divides); a V-cycle to 1e-11; a solve
run to relative residual 1e-12 matches the exact discrete solution u* (FFT /
DST-II) to 1e-10 (max norm, relative).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import exact
from oracle import multigrid as omg
from oracle import operators as oop
from oracle import rkl as orkl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FOURPI = 4.0 * math.pi


def _lib():
    import paper_2306_05332_amd as R
    return R


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rand_faces(rng, shape):
    nz, ny, nx = shape
    return tuple(rng.standard_normal(s) for s in ((nz, ny), (nz, ny), (nz, nx), (nz, nx), (ny, nx), (ny, nx)))


# shapes (nz, ny, nx): several 64x4x8 / 64x8 tiles with ragged tails; the
# first, fourth and fifth run the fused tau-step kernel (the fifth with
# z-chunking), the others the per-stage kernels
SHAPES = [(20, 11, 130), (9, 6, 5), (16, 16, 16), (40, 24, 64), (64, 40, 96)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("s,theta", [(1, 1.0), (2, 0.9), (3, 0.85), (4, 0.9), (5, 0.9)])
def test_rkl_smooth_matches_oracle(shape, bc, s, theta):
    R = _lib()
    rng = np.random.default_rng(100 + s)
    h = (0.11, 0.07, 0.13)
    u0 = rng.standard_normal(shape)
    f = rng.standard_normal(shape) * 50
    faces = rand_faces(rng, shape) if bc == "dirichlet" else None
    nz, ny, nx = shape
    g = oop.Grid(nx, ny, nz, *h, bc)
    want = omg.rkl_smooth(u0, f, g, s, theta, 3, faces)
    phi = cu(u0)
    fused = R.tau_step_launches(shape, s, bc) == 1
    print(f"shape={shape} bc={bc} s={s} fused={fused}", flush=True)
    R.smooth(cu(f), phi, h, bc, s=s, tau_frac=theta, n_steps=3,
             faces=R.pack_faces(faces) if faces else None)
    assert relmax(host(phi), want) < 1e-12


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_rkl_smooth_large_tiles_match_oracle(bc):
    """(nz, ny, nx) = (72, 130, 160): large enough for the z-queue kernel (64 x 32
    tiles, 32-plane chunks) with ragged tiles in x, y and z."""
    R = _lib()
    rng = np.random.default_rng(5)
    shape = (72, 130, 160)
    h = (0.01, 0.012, 0.009)
    u0 = rng.standard_normal(shape)
    f = rng.standard_normal(shape) * 1e4
    faces = rand_faces(rng, shape) if bc == "dirichlet" else None
    nz, ny, nx = shape
    g = oop.Grid(nx, ny, nz, *h, bc)
    want = omg.rkl_smooth(u0, f, g, 2, 0.9, 2, faces)
    phi = cu(u0)
    R.smooth(cu(f), phi, h, bc, s=2, tau_frac=0.9, n_steps=2, faces=R.pack_faces(faces) if faces else None)
    assert relmax(host(phi), want) < 1e-12


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_residual_matches_oracle(bc):
    R = _lib()
    rng = np.random.default_rng(7)
    shape = (20, 11, 130)
    h = (0.11, 0.07, 0.13)
    u = rng.standard_normal(shape)
    f = rng.standard_normal(shape)
    faces = rand_faces(rng, shape) if bc == "dirichlet" else None
    want = f - oop.apply_M(u, h, bc, faces)
    r, nrm = R.residual(cu(f), cu(u), h, bc, faces=R.pack_faces(faces) if faces else None)
    assert relmax(host(r), want) < 1e-13
    assert abs(nrm - np.linalg.norm(want)) < 1e-12 * np.linalg.norm(want)


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("shape", [(4, 4, 4), (8, 6, 10), (16, 34, 132)])
def test_transfers_match_oracle(bc, shape):
    R = _lib()
    rng = np.random.default_rng(9)
    fine = rng.standard_normal(shape)
    got = host(R.restrict(cu(fine)))
    assert relmax(got, oop.restrict(fine)) < 1e-15
    coarse = rng.standard_normal(tuple(n // 2 for n in shape))
    base = rng.standard_normal(shape)
    out = cu(base)
    R.prolong_add(cu(coarse), out, bc)
    assert relmax(host(out), base + oop.prolong(coarse, bc)) < 1e-14


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("n", [4, 6, 8, 16])
def test_coarse_solve_matches_oracle(bc, n):
    """n <= 12 runs in one workgroup (LDS); 16^3 takes the multi-kernel path."""
    R = _lib()
    rng = np.random.default_rng(n)
    shape = (n, n, n)
    h = (0.3, 0.3, 0.3)
    b = rng.standard_normal(shape)
    if bc == "periodic":
        b -= b.mean()
    lv = oop.Level(3, shape, h, bc)
    st = omg.Stats()
    want = omg.coarsest_solve(b, lv, omg.Options(), st)
    u, steps = R.coarse_solve(cu(b), h, bc)
    assert relmax(host(u), want) < 1e-11
    if steps >= 0:
        assert abs(steps - st.coarse_steps[0]) <= 1


def _problem(which):
    if which == "sphere32":
        return W.uniform_sphere(32)
    if which == "blobs32":
        return W.gaussian_blobs(32, 16, seed=2)
    if which == "aniso":
        return W.gaussian_blobs((16, 32, 64), 8, seed=5)
    if which == "accuracy32":
        return W.accuracy_problem(32)
    raise ValueError(which)


def _grid(p):
    nz, ny, nx = p.shape
    return oop.Grid(nx, ny, nz, *p.h, p.bc)


@pytest.mark.parametrize("which", ["sphere32", "blobs32", "aniso"])
def test_vcycle_matches_oracle(which):
    R = _lib()
    p = _problem(which)
    g = _grid(p)
    f = omg.prepare_source(p.rho, g, omg.Options())
    lv = oop.build_hierarchy(g)
    rng = np.random.default_rng(1)
    u0 = rng.standard_normal(p.shape) * 0.01
    want = omg.vcycle(u0, f, lv, omg.Options(), p.faces)
    want2 = omg.vcycle(want, f, lv, omg.Options(), p.faces)
    phi = cu(u0)
    faces = R.pack_faces(p.faces) if p.faces else None
    R.vcycle(cu(f), phi, p.h, p.bc, faces=faces)
    assert relmax(host(phi), want) < 1e-11
    R.vcycle(cu(f), phi, p.h, p.bc, faces=faces)
    assert relmax(host(phi), want2) < 1e-11


@pytest.mark.parametrize("which", ["sphere32", "blobs32", "aniso", "accuracy32"])
def test_solve_reaches_exact_discrete_solution(which):
    R = _lib()
    p = _problem(which)
    faces = R.pack_faces(p.faces) if p.faces else None
    phi, st = R.solve(cu(p.rho), p.h, p.bc, faces=faces, opts=R.Options(tol=1e-12))
    assert st.rel_res <= 1e-12
    us = exact.exact_solution(FOURPI * p.rho, p.h, p.bc, p.faces)
    assert relmax(host(phi), us) < 1e-10
    # the oracle's own solve takes the same number of cycles (up to a tie at tol)
    _, ost = omg.solve(p.rho, _grid(p), omg.Options(tol=1e-12), faces=p.faces)
    assert abs(ost.cycles - st.cycles) <= 1
    np.testing.assert_allclose(st.history[:len(ost.history)][:5], ost.history[:5], rtol=1e-8)


def test_single_level_mode_matches_oracle():
    R = _lib()
    p = W.gaussian_blobs(10, 3, seed=6)
    o = R.Options(tol=1e-11, max_cycles=2000)
    phi, st = R.solve(cu(p.rho), p.h, "periodic", opts=o)
    assert st.levels == 1
    want, ost = omg.solve(p.rho, _grid(p), omg.Options(tol=1e-11, max_cycles=2000))
    assert abs(st.cycles - ost.cycles) <= 1
    assert relmax(host(phi), want) < 1e-9


def test_status_codes_on_gpu():
    R = _lib()
    p = W.gaussian_blobs(16, 4, seed=7)
    rho = cu(p.rho)
    _, st = R.solve(rho, p.h, "periodic", opts=R.Options(max_cycles=1), raise_on_error=False)
    assert st.status == -3 and st.cycles == 1
    bad = p.rho.copy()
    bad[3, 4, 5] = np.nan
    # multi-level solves learn ||f|| after their first cycles are queued: a
    # zero or non-finite one still decides the solve as before (phi = 0, or
    # the non-finite status), in both precisions and from a warm start
    for prec in ("fp64", "mixed"):
        _, st = R.solve(cu(bad), p.h, "periodic", opts=R.Options(prec=prec), raise_on_error=False)
        assert st.status == -5 and st.cycles == 0
        for phi0 in (None, rho * 0.5):
            phi, st = R.solve(torch.zeros_like(rho), p.h, "periodic", phi0=phi0, opts=R.Options(prec=prec))
            assert st.status == 0 and st.cycles == 0 and st.res0 == 0.0 and float(phi.abs().max()) == 0.0
    _, st = R.solve(rho, p.h, "periodic", opts=R.Options(tau_frac=1.05, max_cycles=50), raise_on_error=False)
    assert st.status == -4
    with pytest.raises(R.RKLError):
        R.solve(rho, p.h, "periodic", opts=R.Options(s=-1))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_zero_start_ignores_phi(prec, bc):
    """Options.zero_start (solve() sets it when no phi0 is given): the solve
    never reads phi on entry (the float64 path relaxes its first cycle from
    the zero iterate in the fused tau-step's zero-input form), so a phi full
    of NaN gives the solve from phi = 0 cycle for cycle; a solve that stops
    at its start state returns zeros."""
    import dataclasses
    R = _lib()
    p = W.gaussian_blobs(64, 8, seed=23) if bc == "periodic" else W.uniform_sphere(64)
    faces = R.pack_faces(p.faces) if p.faces else None
    rho = cu(p.rho)
    o = R.Options(tol=1e-10, prec=prec)
    nan = torch.full_like(rho, float("nan"))
    print(f"zero_start prec={prec} bc={bc}", flush=True)
    phi_a, st_a = R.solve(rho, p.h, bc, faces=faces, phi0=torch.zeros_like(rho), opts=o)
    phi_b, st_b = R.solve(rho, p.h, bc, faces=faces, phi0=nan, opts=dataclasses.replace(o, zero_start=True))
    phi_c, st_c = R.solve(rho, p.h, bc, faces=faces, opts=o)  # phi0 None: zero_start, uninitialised phi
    assert st_a.status == st_b.status == st_c.status == 0
    assert st_a.cycles == st_b.cycles == st_c.cycles
    np.testing.assert_allclose(st_b.history, st_a.history, rtol=1e-12)
    assert relmax(host(phi_b), host(phi_a)) < 1e-12 and relmax(host(phi_c), host(phi_a)) < 1e-12
    phi_d, st_d = R.solve(rho, p.h, bc, faces=faces, phi0=nan, opts=dataclasses.replace(o, zero_start=True, tol=1.5))
    assert st_d.status == 0 and st_d.cycles == 0 and float(phi_d.abs().max()) == 0.0


def test_warm_start_converges_in_fewer_cycles():
    R = _lib()
    p = W.gaussian_blobs(64, 16, seed=2)
    rho = cu(p.rho)
    phi, st = R.solve(rho, p.h, "periodic", opts=R.Options(tol=1e-8))
    phi2, st2 = R.solve(rho * 1.001, p.h, "periodic", phi0=phi * 1.001, opts=R.Options(tol=1e-8))
    assert st2.cycles < st.cycles


@pytest.mark.parametrize("n_post", [1, 2])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_no_pre_smoothing_returns_the_tested_state(n_post, prec):
    """n_pre = 0: the cycles start with a copy of the start state (no relaxation
    keeps it); cycles queued past the stopping one must leave the answer
    intact.  The returned phi has the reported residual (recomputed here by
    the library's residual) and matches u*."""
    R = _lib()
    p = W.gaussian_blobs(64, 8, seed=21)
    o = R.Options(tol=1e-10, n_pre=0, n_post=n_post, prec=prec, max_cycles=200)
    phi, st = R.solve(cu(p.rho), p.h, "periodic", opts=o)
    assert st.status == 0 and st.rel_res <= 1e-10
    f = FOURPI * (p.rho - p.rho.mean())
    _, nrm = R.residual(cu(f), phi, p.h, "periodic")
    assert nrm / np.linalg.norm(f) <= 1.0001e-10
    assert abs(nrm / np.linalg.norm(f) - st.rel_res) <= 1e-3 * st.rel_res
    us = exact.exact_solution(FOURPI * p.rho, p.h, "periodic")
    assert relmax(host(phi), us) < 1e-8


def test_batched_class_alternating_n_pre():
    """One grid class solved with n_pre = 2, then 0, then 2 again: each call
    matches the single solve with the same options cycle for cycle."""
    R = _lib()
    probs = [W.gaussian_blobs(32, 6, seed=30 + q) for q in range(3)]
    rhos = [cu(p.rho) for p in probs]
    for n_pre in (2, 0, 2):
        o = R.Options(tol=1e-10, n_pre=n_pre, n_post=1, max_cycles=200)
        phis, sts = R.solve_batched(rhos, [p.h for p in probs], "periodic", opts=o)
        for q, p in enumerate(probs):
            phi1, st1 = R.solve(rhos[q], p.h, "periodic", opts=o)
            print(f"n_pre={n_pre} member {q}: batched {sts[q].cycles} cycles, single {st1.cycles}", flush=True)
            assert sts[q].status == 0 and sts[q].cycles == st1.cycles
            assert relmax(host(phis[q]), host(phi1)) < 1e-12
