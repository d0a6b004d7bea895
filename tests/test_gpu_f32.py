"""Float32 building blocks of the mixed-precision path against the oracle run in
float32, cell by cell, through the float32 C-ABI twins (rkl_smooth_f32,
mg_vcycle_f32, rkl_residual_f32, rkl_restrict_f32, rkl_prolong_add_f32,
rkl_coarse_solve_f32).

The oracle's functions keep the dtype of their inputs, so float32 arrays make
them compute in numpy float32 arithmetic (the emulation of the mixed path's
inner V-cycle).  Both sides then round every operation to float32; they differ
in the order of additions, in FMA contraction (the GPU) and in multiplying by
1/h^2 (the GPU) where the oracle divides by h^2, i.e. by a few float32 ulp
(6e-8) per operation.  Bound: 1e-5 of the field's max norm per call.

The float32 entry points take the correction equation's ghosts on every level
(homogeneous Dirichlet, -u, or periodic wrap), so the oracle runs with no face
data.  The coarsest solve is compared at a fixed number of tau-steps
(coarse_tol far below float32 rounding): a residual test near its threshold
could otherwise stop the two sides one step apart.

The mixed solve as a whole (float64 defect correction around the float32
V-cycles) is compared with the oracle's solve_mixed on its residual history.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import multigrid as omg
from oracle import operators as oop
from oracle import rkl as orkl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def _lib():
    import paper_2306_05332_amd as R
    return R


def cu32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def cu64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def relmax(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def oracle_tau_steps(u0, f, shape, h, bc, s, theta, n):
    """n tau-steps of the oracle in float32 arithmetic"""
    lv = oop.Level(0, shape, h, bc)
    u = np.asarray(u0, dtype=np.float32)
    b = np.asarray(f, dtype=np.float32)
    for _ in range(n):
        u = orkl.tau_step(u, b, s, theta, lv, None)
    assert u.dtype == np.float32
    return u


@pytest.fixture(autouse=True)
def _restore_table():
    R = _lib()
    R.load_library()
    yield
    R.tune_clear()
    R.install_default_tuning()


# several tiles with ragged tails in x, y and z; the first, fourth and fifth take
# the fused tau-step, (9, 6, 5) the per-stage kernels
SHAPES = [(20, 11, 130), (9, 6, 5), (16, 16, 16), (40, 24, 64), (64, 40, 96)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("s,theta", [(1, 1.0), (2, 0.9), (3, 0.85), (4, 0.9), (5, 0.9)])
def test_smooth_f32_matches_oracle(shape, bc, s, theta):
    R = _lib()
    rng = np.random.default_rng(200 + s)
    h = (0.11, 0.07, 0.13)
    u0 = rng.standard_normal(shape)
    f = rng.standard_normal(shape) * 50
    want = oracle_tau_steps(u0, f, shape, h, bc, s, theta, 3)
    phi = cu32(u0)
    print(f"f32 smooth shape={shape} bc={bc} s={s} launches={R.tau_step_launches(shape, s, bc, 'mixed')}",
          flush=True)
    R.smooth(cu32(f), phi, h, bc, s=s, tau_frac=theta, n_steps=3)
    assert phi.dtype == torch.float32
    assert relmax(host(phi), want) < TOL32


VSHAPES = [(20, 11, 130), (16, 16, 16), (40, 24, 64), (72, 130, 160), (11, 100, 136), (9, 60, 20)]
# stage counts each 3-D variant is built for in float32
SUPPORT32 = {"ring64x8": (1, 2, 3, 4), "ring64x4": (1, 2, 3, 4), "zq64x32": (2, 3), "zq64x16": (2, 3),
             "strip8x4": (1, 2, 3), "strip8x1": (1, 2, 3), "strip4x4": (1, 2, 3), "strip5x1": (1, 2, 3),
             "stripyx8x4": (1, 2, 3), "stripyx4x8": (1, 2, 3), "stripyx8x8": (1, 2, 3), "stripyx2x8": (1, 2),
             "stripyx2x16": (1, 2)}


@pytest.mark.parametrize("variant", list(SUPPORT32))
@pytest.mark.parametrize("shape", VSHAPES)
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("s", [1, 2, 3, 4])
def test_forced_variant_f32_matches_oracle(variant, shape, bc, s):
    """Every float32 variant the tuner may install, forced through the tuning
    table (prec "mixed" keys the float32 sweeps), on ragged shapes; the last
    two shapes pack the x remainder of interior strips in the one-wavefront
    strip variants."""
    if s not in SUPPORT32[variant]:
        pytest.skip(f"{variant} is not built for float32 s = {s}")
    R = _lib()
    nz, ny, nx = shape
    target = 128 if (nx + ny) % 2 else 2048
    R.tune_set([{"nx": nx, "ny": ny, "nz": nz, "bc": bc, "prec": "mixed", "s": s, "variant": variant,
                 "target": target}])
    assert R.tune_get(shape, s, bc, "mixed")["variant"] == variant
    rng = np.random.default_rng(17 + s)
    h = (0.11, 0.07, 0.13)
    u0 = rng.standard_normal(shape)
    f = rng.standard_normal(shape) * 50
    want = oracle_tau_steps(u0, f, shape, h, bc, s, 0.9, 2)
    print(f"f32 variant={variant} target={target} shape={shape} bc={bc} s={s}", flush=True)
    phi = cu32(u0)
    R.smooth(cu32(f), phi, h, bc, s=s, tau_frac=0.9, n_steps=2)
    assert relmax(host(phi), want) < TOL32


@pytest.mark.parametrize("shape2", [(64, 200), (34, 130), (128, 96)])
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("s", [1, 2, 3])
def test_smooth_f32_two_dimensional(shape2, bc, s):
    """2-D levels (nz = 1, hz = inf): the float32 2-D strip kernel; three steps
    (a pair pass and a single one where pairs apply)."""
    R = _lib()
    rng = np.random.default_rng(30 + s)
    ny, nx = shape2
    h = (0.02, 0.03)
    u0 = rng.standard_normal(shape2)
    f = rng.standard_normal(shape2) * 50
    want = oracle_tau_steps(u0[None], f[None], (1, ny, nx), (h[0], h[1], math.inf), bc, s, 0.9, 3)[0]
    phi = cu32(u0)
    R.smooth(cu32(f), phi, h, bc, s=s, tau_frac=0.9, n_steps=3)
    assert relmax(host(phi), want) < TOL32


@pytest.mark.parametrize("shape", [(20, 11, 130), (9, 6, 5), (64, 40, 96)])
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_residual_f32_matches_oracle(shape, bc):
    R = _lib()
    rng = np.random.default_rng(7)
    h = (0.11, 0.07, 0.13)
    u = rng.standard_normal(shape).astype(np.float32)
    f = (rng.standard_normal(shape) * 100).astype(np.float32)
    want = f - oop.apply_M(u, h, bc, None)
    assert want.dtype == np.float32
    r, nrm = R.residual(cu32(f), cu32(u), h, bc)
    assert r.dtype == torch.float32
    assert relmax(host(r), want) < TOL32
    ref = np.linalg.norm(want.astype(np.float64))
    assert abs(nrm - ref) < TOL32 * ref


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("shape", [(4, 4, 4), (8, 6, 10), (16, 34, 132), (1, 34, 132)])
def test_transfers_f32_match_oracle(bc, shape):
    R = _lib()
    rng = np.random.default_rng(9)
    flat = shape[0] == 1
    fine = rng.standard_normal(shape).astype(np.float32)
    got = host(R.restrict(cu32(fine)))
    assert relmax(got, oop.restrict(fine, flat)) < 1e-6
    cshape = (1 if flat else shape[0] // 2, shape[1] // 2, shape[2] // 2)
    coarse = rng.standard_normal(cshape).astype(np.float32)
    base = rng.standard_normal(shape).astype(np.float32)
    out = cu32(base)
    R.prolong_add(cu32(coarse), out, bc)
    want = base + oop.prolong(coarse, bc, flat)
    assert want.dtype == np.float32
    assert relmax(host(out), want) < 1e-6


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("n", [4, 6, 8, 16])
def test_coarse_solve_f32_matches_oracle(bc, n):
    """n <= 12 runs in one workgroup; 16^3 takes the multi-kernel path.  A fixed
    count of 24 accelerated tau-steps on both sides."""
    R = _lib()
    rng = np.random.default_rng(40 + n)
    shape = (n, n, n)
    h = (0.3, 0.3, 0.3)
    b = rng.standard_normal(shape)
    if bc == "periodic":
        b -= b.mean()
    b = b.astype(np.float32)
    lv = oop.Level(3, shape, h, bc)
    steps = 24
    want, k, _ = omg.rkl_accelerated(np.zeros_like(b), b, lv, 0.9, None, tol=0.0, max_steps=steps)
    assert k == steps and want.dtype == np.float32
    u, got_steps = R.coarse_solve(cu32(b), h, bc, opts=R.Options(coarse_tol=1e-30, coarse_max_steps=steps))
    assert u.dtype == torch.float32
    if got_steps >= 0:
        assert got_steps == steps
    assert relmax(host(u), want) < TOL32


def _problem(which):
    if which == "sphere32":
        return W.uniform_sphere(32)
    if which == "blobs32":
        return W.gaussian_blobs(32, 16, seed=2)
    if which == "aniso":
        return W.gaussian_blobs((16, 32, 64), 8, seed=5)
    if which == "blobs64":
        return W.gaussian_blobs(64, 8, seed=9)
    raise ValueError(which)


def _grid(p):
    nz, ny, nx = p.shape
    return oop.Grid(nx, ny, nz, *p.h, p.bc)


@pytest.mark.parametrize("which", ["sphere32", "blobs32", "aniso", "blobs64"])
def test_vcycle_f32_matches_oracle(which):
    """Two float32 V-cycles (the tail levels, the transfers and the coarsest
    solve included) from a random start on the correction equation: the
    sphere's density with homogeneous Dirichlet ghosts, periodic blobs."""
    R = _lib()
    p = _problem(which)
    g = _grid(p)
    f = omg.prepare_source(p.rho, g, omg.Options()).astype(np.float32)
    lv = oop.build_hierarchy(g)
    rng = np.random.default_rng(1)
    u0 = (rng.standard_normal(p.shape) * 0.01).astype(np.float32)
    oo = omg.Options(coarse_tol=1e-30, coarse_max_steps=30)
    want = omg.vcycle(u0, f, lv, oo, None)
    want2 = omg.vcycle(want, f, lv, oo, None)
    assert want2.dtype == np.float32
    phi = cu32(u0)
    ro = R.Options(coarse_tol=1e-30, coarse_max_steps=30)
    rel = R.vcycle(cu32(f), phi, p.h, p.bc, opts=ro, want_residual=True)
    print(f"f32 vcycle {which}: rel_res after one cycle {rel:.3e}", flush=True)
    assert relmax(host(phi), want) < TOL32
    R.vcycle(cu32(f), phi, p.h, p.bc, opts=ro)
    assert relmax(host(phi), want2) < TOL32
    # the reported residual is that of the returned iterate (float32 residual,
    # float64 sums); float32 rounding of M u is ~ eps32 * Lambda |u|, which is
    # a few 1e-4 of a residual reduced tenfold, hence the 1e-2
    r1 = np.linalg.norm((f - oop.apply_M(want, p.h, p.bc, None)).astype(np.float64)) / np.linalg.norm(f)
    assert abs(rel - r1) < 1e-2 * r1


@pytest.mark.parametrize("which", ["sphere32", "blobs32", "blobs64"])
def test_mixed_solve_history_matches_oracle(which):
    """The whole mixed-precision solve (float64 residual and update around one
    float32 V-cycle per outer iteration) against the oracle's solve_mixed: the
    same number of outer iterations and the same relative residuals to 1e-4
    (float32 rounding moves them by ~1e-6: the oracle's own history with
    float64 inner cycles differs from its float32 one by < 1e-6 here)."""
    R = _lib()
    p = _problem(which)
    faces = R.pack_faces(p.faces) if p.faces else None
    phi, st = R.solve(cu64(p.rho), p.h, p.bc, faces=faces, opts=R.Options(tol=1e-10, prec="mixed"))
    want, ost = omg.solve_mixed(p.rho, _grid(p), omg.Options(tol=1e-10), faces=p.faces)
    print(f"mixed {which}: gpu {st.cycles} outer, oracle {ost.cycles}; "
          f"gpu {st.history[:4]} oracle {ost.history[:4]}", flush=True)
    assert st.status == 0 and ost.status == 0
    assert st.cycles == ost.cycles
    np.testing.assert_allclose(st.history, ost.history, rtol=1e-4)
    assert relmax(host(phi), want) < 1e-8
