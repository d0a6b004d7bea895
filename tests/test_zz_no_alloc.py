"""rkl_residual_noalloc (the residual entry point for callers that cannot
allocate) against rkl_residual, through the C ABI: the same kernels with the
partial sums in the library's fixed device array.  Two calls in a row, the
second on a smaller grid (the array keeps the first call's contents); 3-D
periodic (same arithmetic: bit-equal), 3-D Dirichlet with face data (applied
in the stencil instead of folded into f: equal to 1e-13), 2-D; and the size
limit, rejected before any GPU work."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    import paper_2306_05332_amd as R
    return R


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rand_faces(rng, shape):
    nz, ny, nx = shape
    return tuple(rng.standard_normal(s) for s in ((nz, ny), (nz, ny), (nz, nx), (nz, nx), (ny, nx), (ny, nx)))


def _pair(R, shape, h, bc, rng, faces=False):
    u = rng.standard_normal(shape)
    f = rng.standard_normal(shape) * 100
    fc = R.pack_faces(rand_faces(rng, shape if len(shape) == 3 else (1,) + shape)) if faces else None
    r_ref, n_ref = R.residual(cu(f), cu(u), h, bc, faces=fc)
    r, n = R.residual_noalloc(cu(f), cu(u), h, bc, faces=fc)
    return r_ref, n_ref, r, float(n.item())


@pytest.mark.parametrize("order", ["big_then_small", "dirichlet_then_2d"])
def test_noalloc_residual_matches_rkl_residual(order):
    R = _lib()
    rng = np.random.default_rng(3)
    if order == "big_then_small":
        cases = [((96, 80, 200), (0.01, 0.012, 0.015), "periodic", False),
                 ((20, 11, 130), (0.11, 0.07, 0.13), "periodic", False)]
    else:
        cases = [((64, 40, 96), (0.02, 0.03, 0.025), "dirichlet", True),
                 ((34, 130), (0.02, 0.03), "dirichlet", True),
                 ((8, 6, 10), (0.2, 0.3, 0.25), "periodic", False)]
    for shape, h, bc, faces in cases:
        print(f"noalloc residual shape={shape} bc={bc} faces={faces}", flush=True)
        r_ref, n_ref, r, n = _pair(R, shape, h, bc, rng, faces)
        if faces:
            assert float((r - r_ref).abs().max()) <= 1e-13 * float(r_ref.abs().max())
            assert abs(n - n_ref) <= 1e-13 * n_ref
        else:
            assert torch.equal(r, r_ref)
            assert n == n_ref


def test_noalloc_residual_rejects_oversize_grid_before_gpu_work():
    R = _lib()
    lib = R.load_library()
    from paper_2306_05332_amd._lib import c_grid
    g = c_grid(2048, 2048, 1024, 1.0, 1.0, 1.0, 1)
    dummy = torch.zeros(1, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(dummy.data_ptr())
    st = lib.rkl_residual_noalloc(ctypes.byref(g), p, None, p, None, None, None)
    assert st == R.RKL_EINVAL
    assert b"partial-sum pairs" in lib.rkl_last_error()
