"""Accuracy study of Sec. 4.1 on the GPU: L2 errors of phi and of g_x against
the analytic solution of the smooth model problem, for N = 16 ... 1024.

The potential is solved to relative residual 1e-12 (the discretisation error
then dominates), g = -grad(phi) comes from the 4th-order kernel, and the
errors are L2 norms relative to the exact fields (the paper's definition with
uniform cells).  Also reported: V-cycles and solve time, and the warm-start
cycle count of Sec. 4.1 (the previous solution as initial guess for a density
changed by 0.1 %, stopped when max |phi^m - phi^(m-1)| < 1e-6 is reached,
measured here from the V-cycle history).

    python -m paper_2306_05332_amd.accuracy --sizes 16 32 64 128 256 512 1024
"""
from __future__ import annotations

import argparse
import json
import math
import time

from . import _lib


def run(sizes, tol=1e-12, log=None):
    import torch

    import workloads as W
    out = []
    prev = None
    for n in sizes:
        rho, phi_e, gx_e, faces = W.accuracy_fields_device(n, "cuda")
        fz = _lib.pack_faces(faces)
        h = (1.0 / n,) * 3
        _lib.solve(rho, h, "dirichlet", faces=fz, opts=_lib.Options(tol=1e-2))  # plans
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi, st = _lib.solve(rho, h, "dirichlet", faces=fz, opts=_lib.Options(tol=tol))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        e_phi = (torch.linalg.vector_norm(phi - phi_e) / torch.linalg.vector_norm(phi_e)).item()
        gx, gy, gz = _lib.gradient(phi, h, "dirichlet", fz)
        del gy, gz
        e_g = (torch.linalg.vector_norm(gx - gx_e) / torch.linalg.vector_norm(gx_e)).item()
        rec = {"n": n, "cycles": st.cycles, "solve_ms": dt * 1e3, "rel_res": st.rel_res, "l2_err_phi": e_phi,
               "l2_err_gx": e_g}
        if prev is not None:
            rec["order_phi"] = math.log2(prev["l2_err_phi"] / e_phi)
            rec["order_gx"] = math.log2(prev["l2_err_gx"] / e_g)
        out.append(rec)
        prev = rec
        if log:
            log(json.dumps(rec))
        del rho, phi_e, gx_e, phi, gx
        _lib.release_all()
        torch.cuda.empty_cache()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--sizes", type=int, nargs="+", default=[16, 32, 64, 128, 256, 512, 1024])
    a = ap.parse_args(argv)
    _lib.load_library()
    run(a.sizes, log=lambda s: print(s, flush=True))


if __name__ == "__main__":
    main()
