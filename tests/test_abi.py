"""The C-ABI library: it loads, exports every function the header declares,
and rejects bad arguments before touching the GPU (runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rkl_poisson.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


@pytest.fixture(scope="module")
def lib():
    from paper_2306_05332_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("librklpoisson.so is not built (python -m paper_2306_05332_amd.build)")
    return _lib.load_library()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for want in ("rkl_poisson_solve", "mg_vcycle", "rkl_smooth", "rkl_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_binding_exports_match_header():
    from paper_2306_05332_amd import _lib
    assert sorted(_lib.EXPORTS) == _declared_functions()


def test_default_options(lib):
    from paper_2306_05332_amd._lib import c_opts
    o = c_opts()
    lib.rkl_default_opts(ctypes.byref(o))
    assert (o.s, o.n_pre, o.n_post, o.min_coarse, o.max_cycles, o.prec, o.smoother, o.fuse) == (2, 2, 1, 4, 100, 0, 0,
                                                                                                 3)
    assert o.zero_start == 0
    assert abs(o.tau_frac - 0.9) < 1e-15 and abs(o.tol - 1e-10) < 1e-25
    assert abs(o.four_pi_G - 4 * 3.141592653589793) < 1e-14


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(hx=0.0), dict(hy=-1.0), dict(hz=float("nan")), dict(bc=7),
    dict(hz=float("inf")), dict(hx=float("inf"), nz=1), dict(hz=-float("inf"), nz=1),
])
def test_invalid_grid_rejected_without_gpu(lib, bad):
    from paper_2306_05332_amd._lib import c_grid
    g = dict(nx=8, ny=8, nz=8, hx=0.1, hy=0.1, hz=0.1, bc=1)
    g.update(bad)
    cg = c_grid(g["nx"], g["ny"], g["nz"], g["hx"], g["hy"], g["hz"], g["bc"])
    st = lib.rkl_poisson_solve(ctypes.byref(cg), None, ctypes.c_void_p(16), None, ctypes.c_void_p(16), None,
                               None)
    assert st == -1
    assert len(lib.rkl_last_error()) > 0


@pytest.mark.parametrize("bad", [dict(s=-1), dict(s=65), dict(tau_frac=0.0), dict(tau_frac=2.5),
                                 dict(n_pre=0, n_post=0), dict(min_coarse=1), dict(tol=-1.0),
                                 dict(max_cycles=-1), dict(prec=5), dict(smoother=2), dict(fuse=4),
                                 dict(fuse=-1), dict(zero_start=2), dict(zero_start=-1)])
def test_invalid_options_rejected_without_gpu(lib, bad):
    from paper_2306_05332_amd._lib import c_grid, c_opts
    o = c_opts()
    lib.rkl_default_opts(ctypes.byref(o))
    for k, v in bad.items():
        setattr(o, k, v)
    cg = c_grid(8, 8, 8, 0.1, 0.1, 0.1, 1)
    st = lib.rkl_poisson_solve(ctypes.byref(cg), ctypes.byref(o), ctypes.c_void_p(16), None,
                               ctypes.c_void_p(16), None, None)
    assert st == -1


def test_periodic_with_faces_and_null_arrays_rejected(lib):
    from paper_2306_05332_amd._lib import c_grid
    cg = c_grid(8, 8, 8, 0.1, 0.1, 0.1, 1)
    assert lib.rkl_poisson_solve(ctypes.byref(cg), None, ctypes.c_void_p(16), ctypes.c_void_p(16),
                                 ctypes.c_void_p(16), None, None) == -1
    assert lib.rkl_poisson_solve(ctypes.byref(cg), None, None, None, ctypes.c_void_p(16), None, None) == -1
    assert lib.rkl_smooth(ctypes.byref(cg), 2, 0.9, -1, ctypes.c_void_p(16), None, ctypes.c_void_p(16),
                          None) == -1
    cg_odd = c_grid(7, 8, 8, 0.1, 0.1, 0.1, 1)
    assert lib.rkl_restrict(ctypes.byref(cg_odd), ctypes.c_void_p(16), ctypes.c_void_p(16), None) == -1


def test_product_path_has_no_cpu_fallback():
    """The binding imports no oracle module and raises if the library is absent."""
    import paper_2306_05332_amd._lib as L
    src = open(L.__file__).read()
    assert "oracle" not in src and "numpy" not in src
    with pytest.raises(ImportError):
        L._lib_saved = L._lib
        try:
            L._lib = None
            L.load_library("/nonexistent/librklpoisson.so")
        finally:
            L._lib = L._lib_saved


# ---------------------------------------------------------------- tuning table (host only)
def test_level_shapes_follow_the_coarsening_rule(lib):
    """Level shapes from the library equal the oracle's hierarchy (coarsen by 2
    while every n/2 is an even integer >= min_coarse)."""
    from oracle import operators as oop
    from paper_2306_05332_amd import _lib
    for shape in [(256, 256, 256), (48, 48, 48), (20, 20, 20), (5, 6, 9), (32, 64, 128), (96, 40, 24)]:
        nz, ny, nx = shape
        want = [lv.shape for lv in oop.build_hierarchy(oop.Grid(nx, ny, nz, 1.0, 1.0, 1.0, "periodic"), 4)]
        assert _lib.level_shapes(shape, 4) == want, shape
    assert _lib.level_shapes((256, 256, 256))[-1] == (4, 4, 4)
    assert len(_lib.level_shapes((256, 256, 256))) == 7


def test_level_shapes_two_dimensional(lib):
    """nz = 1 with hz = inf halves x and y only, like the oracle's 2-D
    hierarchy; with a finite hz the single plane stops the coarsening."""
    from oracle import operators as oop
    from paper_2306_05332_amd import _lib
    for ny, nx in [(48, 64), (4096, 4096), (80, 96), (6, 10), (768, 1024)]:
        want = [lv.shape for lv in oop.build_hierarchy(oop.grid2d(nx, ny, 1.0, 1.0, "periodic"), 4)]
        assert _lib.level_shapes((ny, nx)) == want
        assert _lib.level_shapes((1, ny, nx), h=(1.0, 1.0)) == want
        assert _lib.level_shapes((1, ny, nx)) == [(1, ny, nx)]
    assert _lib.level_shapes((48, 64))[-1] == (1, 6, 8)


def test_tuning_table_install_query_erase(lib):
    from paper_2306_05332_amd import _lib
    _lib.tune_clear()
    try:
        shape = (256, 256, 256)
        assert _lib.tune_get(shape, 2, "periodic", "fp64")["variant"] == "strip8x4"
        assert _lib.tune_get(shape, 3, "periodic", "fp64")["variant"] == "zq64x32"
        assert _lib.tune_get((16, 16, 16), 3, "periodic", "fp64")["variant"] == "ring64x4"
        assert _lib.tune_get((8, 8, 8), 2, "periodic", "fp64")["variant"] == "heuristic"  # no fused step
        e = {"nx": 256, "ny": 256, "nz": 256, "bc": "periodic", "prec": "fp64", "s": 2, "variant": "ring64x4",
             "target": 512}
        _lib.tune_set([e])
        got = _lib.tune_get(shape, 2, "periodic", "fp64")
        assert (got["variant"], got["target"]) == ("ring64x4", 512)
        # other keys untouched
        assert _lib.tune_get(shape, 2, "dirichlet", "fp64")["variant"] == "strip4x4"
        assert _lib.tune_get(shape, 2, "periodic", "mixed")["variant"] == "strip4x4"
        _lib.tune_set([dict(e, variant=0)])
        assert _lib.tune_get(shape, 2, "periodic", "fp64")["variant"] == "strip8x4"
        # a variant not built for the (s, precision) pair is refused, and nothing is installed
        with pytest.raises(_lib.RKLError):
            _lib.tune_set([dict(e, variant="ring64x8"), dict(e, s=1, variant="zq64x16")])
        assert _lib.tune_get(shape, 2, "periodic", "fp64")["variant"] == "strip8x4"
        with pytest.raises(_lib.RKLError):
            _lib.tune_set([dict(e, target=0)])
    finally:
        _lib.tune_clear()
        _lib.install_default_tuning()


def test_tuning_json_round_trip(lib, tmp_path):
    from paper_2306_05332_amd import _lib, autotune
    _lib.tune_clear()
    try:
        tiles = [{"nx": 128, "ny": 128, "nz": 128, "bc": "periodic", "prec": "mixed", "s": 2, "variant": "zq64x16",
                  "target": 1024, "us": 12.5}]
        path = str(tmp_path / "t.json")
        autotune.save(path, tiles, [{"nx": 64, "ny": 64, "nz": 64, "bc": "periodic", "prec": "fp64", "s": 3}])
        assert autotune.load(path) == 2
        got = _lib.tune_get((128, 128, 128), 2, "periodic", "mixed")
        assert (got["variant"], got["target"]) == ("zq64x16", 1024)
    finally:
        _lib.tune_clear()
        _lib.install_default_tuning()


def test_stored_table_is_valid(lib):
    """The committed table installs (every variant it names is built)."""
    from paper_2306_05332_amd import autotune
    if not os.path.exists(autotune.DEFAULT_TABLE):
        pytest.skip("no stored tuning table")
    assert autotune.load() > 0


def test_strip2d_variants_only_on_two_dimensional_levels(lib):
    from paper_2306_05332_amd import _lib
    try:
        _lib.tune_set([{"nx": 64, "ny": 32, "nz": 1, "bc": "periodic", "prec": "fp64", "s": 2,
                        "variant": "strip2d4", "target": 256}])
        got = _lib.tune_get((32, 64), 2, "periodic", "fp64")
        assert (got["variant"], got["target"]) == ("strip2d4", 256)
        for bad in ({"nz": 8, "variant": "strip2d8"}, {"nz": 1, "variant": "strip8x4"},
                    {"nz": 1, "variant": "strip2d8", "s": 5}):
            e = {"nx": 64, "ny": 32, "bc": "periodic", "prec": "fp64", "s": 2, "target": 256}
            e.update(bad)
            with pytest.raises(_lib.RKLError):
                _lib.tune_set([e])
        # float32 sweeps take s = 3 on 2-D levels
        _lib.tune_set([{"nx": 64, "ny": 32, "nz": 1, "bc": "dirichlet", "prec": "mixed", "s": 3,
                        "variant": "strip2d8", "target": 128}])
        assert _lib.tune_get((32, 64), 3, "dirichlet", "mixed")["variant"] == "strip2d8"
        assert _lib.tau_step_launches((32, 64), 2, "periodic") == 1
        assert _lib.tau_step_launches((32, 64), 4, "periodic") == 1  # 2-D levels fuse up to 4 stages
        assert _lib.tau_step_launches((32, 64), 5, "periodic") == 5
        assert _lib.tau_step_launches((1, 32, 64), 2, "periodic") == 2  # finite hz: a 3-D single plane
    finally:
        _lib.tune_clear()
        _lib.install_default_tuning()


def test_s_opt_rule_through_the_abi(lib):
    """App. A.3 through rkl_s_opt (host arithmetic, no GPU): 56 for the paper's
    N = 64 model (cubic Dirichlet grid, tau = tau_max, six modes, two digits);
    equal to the oracle's 1-D argmin for N = 16 .. 128 and to the oracle's
    level form at theta = 0.9 on periodic, anisotropic and 2-D grids."""
    import math

    from oracle import operators as op
    from oracle import rkl as orkl
    from paper_2306_05332_amd import _lib
    s, m = _lib.s_opt((64, 64, 64), 1.0 / 64, "dirichlet", tau_frac=1.0)
    assert s == 56
    assert abs(m - orkl.m_eff_1d(56, 64)) <= 1e-9 * m
    for N in (16, 24, 32, 48, 64, 96, 128):
        assert _lib.s_opt((N, N, N), 1.0 / N, "dirichlet", tau_frac=1.0)[0] == orkl.s_opt_global_1d(N), N
    cases = [((32, 32, 32), (1 / 32,) * 3, "periodic"), ((16, 32, 64), (0.01, 0.012, 0.015), "dirichlet"),
             ((24, 40, 56), (0.02, 0.02, 0.03), "periodic"), ((64, 96), (0.01, 0.02), "dirichlet")]
    for shape, h, bc in cases:
        lshape = shape if len(shape) == 3 else (1,) + shape
        lh = h if len(h) == 3 else (h[0], h[1], math.inf)
        want, wm = orkl.s_opt_global(op.Level(0, lshape, lh, bc), 0.9)
        got, gm = _lib.s_opt(shape, h, bc, tau_frac=0.9)
        assert got == want and abs(gm - wm) <= 1e-9 * wm, (shape, bc, got, want)


def test_s_opt_rejects_bad_arguments(lib):
    from paper_2306_05332_amd._lib import c_grid
    g = c_grid(8, 8, 8, 0.1, 0.1, 0.1, 0)
    assert lib.rkl_s_opt(ctypes.byref(g), 0.0, 6, 2.0, None) == -1
    assert lib.rkl_s_opt(ctypes.byref(g), 0.9, 0, 2.0, None) == -1
    assert lib.rkl_s_opt(ctypes.byref(g), 0.9, 6, -1.0, None) == -1
