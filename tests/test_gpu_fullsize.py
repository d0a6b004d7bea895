"""Full-size GPU cases (the benchmark's configurations) against the exact
discrete solution, which the CPU computes by FFT (periodic) or DST-II
(Dirichlet) for any size; the oracle's V-cycle would take minutes here.

Bounds: float64 solve at relative residual 1e-12 -> 1e-10 relative max-norm
error vs u*; timed float64 / mixed solves at 1e-10 -> reported error, bound
1e-9 (stated: the residual-to-error amplification observed on these fields is
below 10, and the float64 outer residual fixes the attainable accuracy for the
mixed path too).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import exact

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
FOURPI = 4.0 * math.pi


def _lib():
    import paper_2306_05332_amd as R
    return R


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def relmax(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_blobs_256_fp64_matches_fft():
    R = _lib()
    p = W.gaussian_blobs(256, 16, seed=2)
    us = exact.exact_solution(FOURPI * p.rho, p.h, "periodic")
    rho = cu(p.rho)
    phi, st = R.solve(rho, p.h, "periodic", opts=R.Options(tol=1e-12))
    assert st.status == 0 and st.rel_res <= 1e-12
    err = relmax(phi.cpu().numpy(), us)
    print(f"256^3 fp64 tol 1e-12: cycles={st.cycles} err={err:.3e}")
    assert err < 1e-10
    phi, st = R.solve(rho, p.h, "periodic", opts=R.Options(tol=1e-10))
    err = relmax(phi.cpu().numpy(), us)
    print(f"256^3 fp64 tol 1e-10: cycles={st.cycles} err={err:.3e}")
    assert err < 1e-9
    phi, st = R.solve(rho, p.h, "periodic", opts=R.Options(tol=1e-10, prec="mixed"))
    err = relmax(phi.cpu().numpy(), us)
    print(f"256^3 mixed tol 1e-10: cycles={st.cycles} err={err:.3e}")
    assert st.status == 0 and err < 1e-9


def test_grf_512_mixed_matches_fft():
    R = _lib()
    p = W.gaussian_random_field(512, seed=3)
    rho = cu(p.rho)
    phi, st = R.solve(rho, p.h, "periodic", opts=R.Options(tol=1e-10, prec="mixed"))
    assert st.status == 0 and st.rel_res <= 1e-10
    got = phi.cpu().numpy()
    del phi, rho
    us = exact.exact_solution(FOURPI * p.rho, p.h, "periodic")
    err = relmax(got, us)
    print(f"512^3 mixed tol 1e-10: cycles={st.cycles} err={err:.3e}")
    assert err < 1e-9


def test_sphere_32_dirichlet_fp64_matches_dst_and_analytic():
    R = _lib()
    p = W.uniform_sphere(32)
    phi, st = R.solve(cu(p.rho), p.h, "dirichlet", faces=R.pack_faces(p.faces), opts=R.Options(tol=1e-10))
    got = phi.cpu().numpy()
    us = exact.exact_solution(FOURPI * p.rho, p.h, "dirichlet", p.faces)
    assert relmax(got, us) < 1e-9
    e = np.linalg.norm(got - p.phi_exact) / np.linalg.norm(p.phi_exact)
    assert 5e-3 < e < 3e-2
