"""Every fused tau-step variant the tuner may pick, forced through the tuning
table, against the oracle's tau-steps; the tuner itself on the GPU; and the
stage count taken from the table when Options.s == 0."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import exact
from oracle import multigrid as omg
from oracle import operators as oop

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


@pytest.fixture(autouse=True)
def _restore_table():
    R = _lib()
    R.load_library()
    yield
    R.tune_clear()
    R.install_default_tuning()


# ragged in x, y and z for every tile shape; (72, 130, 160) spans several
# z-queue tiles in x and y.  The last two pack the x remainder of interior
# strips into shared wavefronts in the one-wavefront strip variants
# (nx = 136: 3 or 4 strips per wavefront, with unpacked interior strips left
# over; nx = 20: no full tile, 2 strips per wavefront)
VSHAPES = [(20, 11, 130), (16, 16, 16), (40, 24, 64), (72, 130, 160), (11, 100, 136), (9, 60, 20)]
VARIANTS = ["ring64x8", "ring64x4", "zq64x32", "zq64x16", "strip8x4", "strip8x1", "strip4x4", "strip5x1",
            "stripyx8x4", "stripyx4x8", "stripyx8x8", "stripyx2x8", "stripyx2x16"]
# stage counts each variant is built for: (float64, float32)
SUPPORT = {"ring64x8": ((1, 2, 3), (1, 2, 3, 4)), "ring64x4": ((1, 2, 3), (1, 2, 3, 4)),
           "zq64x32": ((2, 3), (2, 3)), "zq64x16": ((2, 3), (2, 3)),
           "strip8x4": ((1, 2), (1, 2, 3)), "strip8x1": ((1, 2), (1, 2, 3)), "strip4x4": ((1, 2), (1, 2, 3)),
           "strip5x1": ((1, 2), (1, 2, 3)), "stripyx8x4": ((1, 2), (1, 2, 3)), "stripyx4x8": ((1, 2, 3), (1, 2, 3)),
           "stripyx8x8": ((1, 2), (1, 2, 3)), "stripyx2x8": ((1, 2), (1, 2)), "stripyx2x16": ((1, 2), (1, 2))}


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("shape", VSHAPES)
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("s", [1, 2, 3])
def test_forced_variant_matches_oracle(variant, shape, bc, s):
    if s not in SUPPORT[variant][0]:
        pytest.skip(f"{variant} is not built for float64 s = {s}")
    R = _lib()
    nz, ny, nx = shape
    target = 128 if (nx + ny) % 2 else 2048
    R.tune_set([{"nx": nx, "ny": ny, "nz": nz, "bc": bc, "prec": "fp64", "s": s, "variant": variant,
                 "target": target}])
    assert R.tune_get(shape, s, bc, "fp64")["variant"] == variant
    rng = np.random.default_rng(7 + s)
    h = (0.11, 0.07, 0.13)
    u0 = rng.standard_normal(shape)
    f = rng.standard_normal(shape) * 50
    faces = rand_faces(rng, shape) if bc == "dirichlet" else None
    g = oop.Grid(nx, ny, nz, *h, bc)
    want = omg.rkl_smooth(u0, f, g, s, 0.9, 2, faces)
    print(f"variant={variant} target={target} shape={shape} bc={bc} s={s}", flush=True)
    phi = cu(u0)
    R.smooth(cu(f), phi, h, bc, s=s, tau_frac=0.9, n_steps=2, faces=R.pack_faces(faces) if faces else None)
    assert relmax(phi.cpu().numpy(), want) < 1e-12


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("s", [2, 3])
def test_forced_variant_float32_solve(variant, bc, s):
    """The float32 sweeps of the mixed path with each variant on every level
    that runs a fused tau-step: the solve still reaches u*, in the same number
    of outer iterations as with the built-in choice (all variants compute the
    same values up to float32 rounding).  Each outer iteration's float32
    V-cycle rounds differently per variant, which perturbs that iteration's
    contraction independently of the others, so the residual histories drift
    apart roughly linearly in the iteration count (about 1e-5 per iteration
    here); the per-iteration contraction factors h_k / h_(k-1) are compared."""
    if s not in SUPPORT[variant][1]:
        pytest.skip(f"{variant} is not built for float32 s = {s}")
    R = _lib()
    p = W.gaussian_blobs(64, 8, seed=9) if bc == "periodic" else W.uniform_sphere(64)
    rho = cu(p.rho)
    o = R.Options(tol=1e-10, prec="mixed", s=s)
    R.tune_clear()
    _, ref = R.solve(rho, p.h, bc, opts=o)
    R.tune_set([{"nx": n, "ny": n, "nz": n, "bc": bc, "prec": "mixed", "s": s, "variant": variant,
                 "target": 512} for n in (64, 32, 16)])
    phi, st = R.solve(rho, p.h, bc, opts=o)
    assert st.status == 0 and st.cycles == ref.cycles
    got, want = np.asarray(st.history), np.asarray(ref.history)
    np.testing.assert_allclose(got[1:] / got[:-1], want[1:] / want[:-1], rtol=1e-4)
    us = exact.exact_solution(4 * math.pi * p.rho, p.h, bc, None)
    assert relmax(phi.cpu().numpy(), us) < 1e-9


@pytest.mark.parametrize("variant", ["strip8x1", "strip5x1"])
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_packed_remainder_solve(variant, bc):
    """float64 solve with a one-wavefront strip variant on every fused level of
    a (48, 96, 136) hierarchy, whose two finest levels pack their x remainder
    (the convergence test reads the packed kernel's residual partials): the
    same cycles and residual history as the built-in choice, and u*."""
    R = _lib()
    shape = (48, 96, 136)
    h = (0.010, 0.012, 0.015)
    rng = np.random.default_rng(12)
    rho = rng.standard_normal(shape)
    o = R.Options(tol=1e-10, s=2)
    R.tune_clear()
    _, ref = R.solve(cu(rho), h, bc, opts=o)
    R.tune_set([{"nx": nx, "ny": ny, "nz": nz, "bc": bc, "prec": "fp64", "s": 2, "variant": variant,
                 "target": t} for (nz, ny, nx) in ((48, 96, 136), (24, 48, 68), (12, 24, 34)) for t in (1024,)])
    print(f"variant={variant} bc={bc} shape={shape}", flush=True)
    phi, st = R.solve(cu(rho), h, bc, opts=o)
    assert st.status == 0 and st.cycles == ref.cycles
    # same values up to rounding; near 1e-10 the residual's rounding is ~1e-6 of it
    np.testing.assert_allclose(st.history, ref.history, rtol=1e-4)
    us = exact.exact_solution(4 * math.pi * rho, h, bc, None)
    assert relmax(phi.cpu().numpy(), us) < 1e-9


def test_autotune_level_installs_fastest():
    R = _lib()
    shape = (64, 64, 64)
    res = R.autotune_level(shape, 2, "periodic", "fp64", reps=5)
    assert len(res) >= 4
    us = [r["us"] for r in res]
    assert us == sorted(us) and us[0] > 0.0
    got = R.tune_get(shape, 2, "periodic", "fp64")
    assert (got["variant"], got["target"]) == (res[0]["variant"], res[0]["target"])
    p = W.gaussian_blobs(64, 8, seed=10)
    phi, st = R.solve(cu(p.rho), p.h, "periodic", opts=R.Options(tol=1e-10))
    us_ = exact.exact_solution(4 * math.pi * p.rho, p.h, "periodic")
    assert st.status == 0 and relmax(phi.cpu().numpy(), us_) < 1e-9


def test_stage_count_from_table():
    R = _lib()
    p = W.gaussian_blobs(32, 6, seed=11)
    rho = cu(p.rho)
    R.tune_set_s((32, 32, 32), 3, "periodic", "fp64")
    phi0, st0 = R.solve(rho, p.h, "periodic", opts=R.Options(s=0, tol=1e-10))
    phi3, st3 = R.solve(rho, p.h, "periodic", opts=R.Options(s=3, tol=1e-10))
    assert st0.cycles == st3.cycles and st0.history == st3.history
    assert torch.equal(phi0, phi3)
    R.tune_set_s((32, 32, 32), 0, "periodic", "fp64")  # erase: default s = 2
    phi2, st2 = R.solve(rho, p.h, "periodic", opts=R.Options(s=0, tol=1e-10))
    _, st2b = R.solve(rho, p.h, "periodic", opts=R.Options(s=2, tol=1e-10))
    assert st2.history == st2b.history
