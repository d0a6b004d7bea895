"""Large-s tau-steps run as chunks of two stages (the strip kernel's chunk
form: each pass reads Y_{j-1}, Y_{j-2} and b and writes its last two
stages) against the oracle's stage-by-stage RKL recurrence (App. A eq.
RKL_intermediate_source), through the single-level relaxation driver
(rkl_relax_solve, App. B) on grids that are ragged against the 60 x 16 strip
tiles.

Fixed stage counts cover even and odd s (an odd s ends in a one-stage
chunk); s = 0 walks the accelerated schedule of App. A.4.  Both sides run
exactly `steps` tau-steps (tol_max = 0) and the iterates are compared to
1e-10 of their max norm: each of the ~50-100 stages adds a few ulp of
reordering and FMA contraction.
"""
import numpy as np
import pytest

from oracle import multigrid as omg
from oracle import operators as oop

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPES = [(20, 36, 70), (16, 9, 130)]


def _lib():
    import paper_2306_05332_amd as R
    return R


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("s,steps", [(5, 8), (6, 8), (7, 6), (12, 4), (0, 6)])
def test_chunked_tau_steps_match_oracle(shape, bc, s, steps):
    R = _lib()
    nz, ny, nx = shape
    h = (0.05, 0.04, 0.06)
    rng = np.random.default_rng(17 + s)
    f = rng.standard_normal(shape) * 100.0
    if bc == "periodic":
        f -= f.mean()
    faces = None
    if bc == "dirichlet":
        faces = tuple(rng.standard_normal(q) for q in ((nz, ny), (nz, ny), (nz, nx), (nz, nx), (ny, nx), (ny, nx)))
    g = oop.Grid(nx, ny, nz, *h, bc)
    u, it, _, _ = omg.relax_solve(f, g, "rkl", faces=faces, tol_max=0.0, max_iters=steps, s=s, theta=0.9)
    assert it == steps
    phi, st = R.relax_solve(torch.from_numpy(f).cuda(), h, bc, "rkl", faces=R.pack_faces(faces) if faces else None,
                            s=s, tol_max=0.0, max_iters=steps, raise_on_error=False)
    print(f"{shape} {bc} s={s}: {st.cycles} tau-steps, max residual {st.rel_res:.3e}", flush=True)
    assert st.cycles == steps
    assert relmax(phi.cpu().numpy(), u) < 1e-10
