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
    assert (o.s, o.n_pre, o.n_post, o.min_coarse, o.max_cycles, o.prec) == (2, 2, 1, 4, 100, 0)
    assert abs(o.tau_frac - 0.9) < 1e-15 and abs(o.tol - 1e-10) < 1e-25
    assert abs(o.four_pi_G - 4 * 3.141592653589793) < 1e-14


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(hx=0.0), dict(hy=-1.0), dict(hz=float("nan")), dict(bc=7),
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


@pytest.mark.parametrize("bad", [dict(s=0), dict(s=65), dict(tau_frac=0.0), dict(tau_frac=2.5),
                                 dict(n_pre=0, n_post=0), dict(min_coarse=1), dict(tol=-1.0),
                                 dict(max_cycles=-1), dict(prec=5)])
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
