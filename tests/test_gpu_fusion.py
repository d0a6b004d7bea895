"""Transfer fusion: V-cycles whose prolongation + correction runs inside the
first post-smoothing tau-step (Options.fuse bit 0; Sec. 2.1 steps 4-5
followed by the post-smoothing relaxation), and whose last pre-smoothing
tau-step also writes the restricted residual (bit 1; Sec. 2.1 steps 1-2b),
against the oracle's V-cycle, which relaxes, forms the residual, restricts,
prolongs and corrects as separate steps.

Every strip variant is forced through the tuning table onto the two finest
levels (the five-row strip has no fused form: in float64 it keeps the
separate prolongation, in float32 its levels take the fused four-row strips;
the float64 eight-row strips take the stacked two-row strips for the fused
step), on a grid that is ragged against every tile shape in x and y, with both
boundary types, float64 (mg_vcycle) and float32 (mg_vcycle_f32) and one or
two post-smoothing (or pre-smoothing) relaxations.  The restriction form
exists at s >= 2 for the stacked two-row strips (every float64 level, s = 2)
and, in float32, for the four-row strips (s = 2, 3), which a level takes unless
tuned for the two-row strips; s = 1 and float64 s = 3 restrict separately.  A
finest level with Dirichlet face data (mg_vcycle with faces) runs the LDS-ring
kernel and restricts separately; its next level takes the fused form.
Tolerances are those of the unfused
V-cycle tests: 1e-11 of the field's max norm in float64, 1e-5 in float32
(the float32 oracle runs in numpy float32; the coarsest solve takes a fixed
number of tau-steps so both sides stop at the same step).
"""
import functools
import math

import numpy as np
import pytest

from oracle import multigrid as omg
from oracle import operators as oop

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (nz, ny, nx): levels (40, 24, 136), (20, 12, 68), (10, 6, 34).  nx = 136 is
# 2 full x tiles + 16 columns for s = 2 (60-column tiles), ny = 24 is 1.5 or
# 0.75 workgroups of the 16- and 32-row variants
SHAPE = (40, 24, 136)
H = (0.11, 0.07, 0.13)
VARIANTS = ["strip8x4", "strip8x1", "strip4x4", "strip5x1", "stripyx8x4", "stripyx4x8", "stripyx8x8",
            "stripyx2x8", "stripyx2x16"]
S64 = {v: (1, 2) for v in VARIANTS}
S32 = {v: (1, 2, 3) for v in VARIANTS}
S32["stripyx2x8"] = S32["stripyx2x16"] = (1, 2)
TOL64, TOL32 = 1e-11, 1e-5
COARSE = dict(coarse_tol=1e-30, coarse_max_steps=40)


def _lib():
    import paper_2306_05332_amd as R
    return R


@pytest.fixture(autouse=True)
def _restore_table():
    R = _lib()
    R.load_library()
    yield
    R.tune_clear()
    R.install_default_tuning()


def relmax(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _inputs(bc, dtype):
    rng = np.random.default_rng(31)
    f = rng.standard_normal(SHAPE) * 40.0
    if bc == "periodic":
        f -= f.mean()
    u0 = rng.standard_normal(SHAPE) * 0.05
    faces = None
    if bc == "dirichlet" and dtype == np.float64:
        nz, ny, nx = SHAPE
        faces = tuple(rng.standard_normal(s) for s in ((nz, ny), (nz, ny), (nz, nx), (nz, nx), (ny, nx), (ny, nx)))
    return f.astype(dtype), u0.astype(dtype), faces


@functools.lru_cache(maxsize=None)
def _oracle(bc, s, n_post, dtype_name, n_pre=2):
    dtype = np.dtype(dtype_name).type
    f, u0, faces = _inputs(bc, dtype)
    nz, ny, nx = SHAPE
    lv = oop.build_hierarchy(oop.Grid(nx, ny, nz, *H, bc))
    o = omg.Options(s=s, n_pre=n_pre, n_post=n_post, **COARSE)
    return omg.vcycle(u0, f, lv, o, faces)


def _force(R, variant, s, bc, prec):
    shapes = R.level_shapes(SHAPE, bc=bc, h=H)
    R.tune_set([{"nx": nx, "ny": ny, "nz": nz, "bc": bc, "prec": prec, "s": s, "variant": variant, "target": 512}
                for (nz, ny, nx) in shapes[:2]])


def _run(R, bc, s, n_post, fuse, dtype, n_pre=2):
    f, u0, faces = _inputs(bc, dtype)
    phi = torch.from_numpy(u0.copy()).cuda()
    ft = torch.from_numpy(f).cuda()
    pf = R.pack_faces(faces) if faces is not None else None
    R.vcycle(ft, phi, H, bc, faces=pf, opts=R.Options(s=s, n_pre=n_pre, n_post=n_post, fuse=fuse, **COARSE))
    return phi.cpu().numpy()


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("s", [1, 2])
@pytest.mark.parametrize("n_post", [1, 2])
def test_fused_prolongation_vcycle_matches_oracle(variant, bc, s, n_post):
    R = _lib()
    if s not in S64[variant]:
        pytest.skip(f"{variant} is not built for float64 s = {s}")
    _force(R, variant, s, bc, "fp64")
    print(f"fp64 {variant} {bc} s={s} n_post={n_post}", flush=True)
    want = _oracle(bc, s, n_post, "float64")
    got = _run(R, bc, s, n_post, True, np.float64)
    assert relmax(got, want) < TOL64
    unfused = _run(R, bc, s, n_post, False, np.float64)
    assert relmax(unfused, want) < TOL64


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("s", [1, 2, 3])
def test_fused_prolongation_vcycle_f32_matches_oracle(variant, bc, s):
    R = _lib()
    if s not in S32[variant]:
        pytest.skip(f"{variant} is not built for float32 s = {s}")
    _force(R, variant, s, bc, "mixed")
    print(f"fp32 {variant} {bc} s={s}", flush=True)
    want = _oracle(bc, s, 1, "float32")
    got = _run(R, bc, s, 1, True, np.float32)
    assert relmax(got, want) < TOL32


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("s", [1, 2, 3])
@pytest.mark.parametrize("n_pre", [1, 2])
def test_fused_restriction_vcycle_matches_oracle(variant, bc, s, n_pre):
    """Each fusion alone (fuse = 1: prolongation, 2: restriction) and both
    (fuse = 3), float64: with n_pre = 1 only the finest level's single
    relaxation carries the restriction (a coarse level's only relaxation is
    the one from zero), with n_pre = 2 every level above the tail."""
    R = _lib()
    if s == 3 and variant != "stripyx4x8":
        pytest.skip("float64 s = 3 takes the stacked four-row strips (restricted separately)")
    if s != 3 and s not in S64[variant]:
        pytest.skip(f"{variant} is not built for float64 s = {s}")
    _force(R, variant, s, bc, "fp64")
    print(f"fp64 {variant} {bc} s={s} n_pre={n_pre}", flush=True)
    want = _oracle(bc, s, 1, "float64", n_pre)
    for fuse in (1, 2, 3):
        got = _run(R, bc, s, 1, fuse, np.float64, n_pre)
        assert relmax(got, want) < TOL64, fuse


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("s", [1, 2, 3])
def test_fused_restriction_vcycle_f32_matches_oracle(variant, bc, s):
    R = _lib()
    if s not in S32[variant]:
        pytest.skip(f"{variant} is not built for float32 s = {s}")
    _force(R, variant, s, bc, "mixed")
    print(f"fp32 {variant} {bc} s={s}", flush=True)
    want = _oracle(bc, s, 1, "float32")
    for fuse in (1, 2, 3):
        got = _run(R, bc, s, 1, fuse, np.float32)
        assert relmax(got, want) < TOL32, fuse


def test_fused_solve_takes_the_same_cycles():
    """A 128^3 periodic solve to 1e-10 with and without fusion: the same cycle
    count and residual history to rounding.  The two iterates differ by
    rounding (~1e-16 of |u|), which moves a relative residual by about
    eps |M| |u| / |f| ~ 1e-15 in absolute terms, hence atol = 1e-14."""
    import workloads as W
    R = _lib()
    R.install_default_tuning()
    p = W.gaussian_blobs(128, 16, seed=2)
    rho = torch.from_numpy(p.rho).cuda()
    out = {}
    for fuse in (True, False):
        for prec in ("fp64", "mixed"):
            phi, st = R.solve(rho, p.h, "periodic", opts=R.Options(tol=1e-10, prec=prec, fuse=fuse))
            out[fuse, prec] = (phi.cpu().numpy(), st)
    for prec in ("fp64", "mixed"):
        (a, sa), (b, sb) = out[True, prec], out[False, prec]
        assert sa.cycles == sb.cycles and sa.rel_res <= 1e-10
        np.testing.assert_allclose(sa.history, sb.history, rtol=1e-6, atol=1e-14)
        assert relmax(a, b) < 1e-10
