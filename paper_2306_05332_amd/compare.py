"""Single-level comparison of RKL, Gauss-Seidel and SOR (App. B) on the GPU.

The paper times the three relaxations, without multigrid, on its 3-D
accuracy problem (Sec. 4.1: rho = rho0 (1 - r^2/r0^2)^2 inside r0 = 0.25,
Dirichlet data from the exact potential) at 128^3 until the maximum residual
falls below 1e-10; SOR uses omega = 2 / (1 + sqrt(1 - rho_J^2)).  This tool
runs the same three iterations through ``rkl_relax_solve`` and reports
iterations, wall time and the final maximum residual; the V-cycle solve of
the same problem is timed alongside for context.

    python -m paper_2306_05332_amd.compare --n 128
"""
from __future__ import annotations

import argparse
import json
import math
import time

from . import _lib


def accuracy_inputs(n):
    """Density, spacing and face data of the accuracy problem (seedless, closed form)."""
    import workloads as W
    return W.accuracy_problem(n)


def run(n=128, tol_max=1e-10, methods=("rkl", "sor", "gsrb"), check_every=None, max_iters=400000, log=None):
    import torch
    p = accuracy_inputs(n)
    f = torch.from_numpy(4.0 * math.pi * p.rho).cuda()
    faces = _lib.pack_faces(p.faces)
    out = []
    for m in methods:
        ce = check_every or (1 if m == "rkl" else 20)
        # warm-up: one whole solve, so that plans, kernels and every tau-step
        # length of the schedule have run once before the timed one
        _lib.relax_solve(f, p.h, "dirichlet", m, faces=faces, tol_max=tol_max, max_iters=max_iters,
                         check_every=ce, history_cap=8, raise_on_error=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi, st = _lib.relax_solve(f, p.h, "dirichlet", m, faces=faces, tol_max=tol_max, max_iters=max_iters,
                                   check_every=ce, history_cap=8, raise_on_error=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rec = {"method": m, "iterations": st.cycles, "seconds": dt, "max_residual": st.rel_res,
               "status": st.status, "check_every": ce}
        out.append(rec)
        if log:
            log(json.dumps(rec))
    rho = torch.from_numpy(p.rho).cuda()
    _lib.solve(rho, p.h, "dirichlet", faces=faces, opts=_lib.Options(tol=1e-12))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi, st = _lib.solve(rho, p.h, "dirichlet", faces=faces, opts=_lib.Options(tol=1e-12))
    torch.cuda.synchronize()
    rec = {"method": "multigrid (RKL smoother)", "iterations": st.cycles, "seconds": time.perf_counter() - t0,
           "relative_l2_residual": st.rel_res}
    out.append(rec)
    if log:
        log(json.dumps(rec))
    return out


def summarize_trace(d, top=10):
    """Per-kernel summary of a ``rocprofv3 --kernel-trace`` directory of this
    tool's run: calls, total and mean duration, largest first."""
    import csv
    import glob
    files = glob.glob(f"{d}/**/*kernel_trace.csv", recursive=True)
    if not files:
        raise SystemExit(f"no kernel trace under {d}")
    agg = {}
    for r in csv.DictReader(open(files[0])):
        dt = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        a = agg.setdefault(r["Kernel_Name"], [0, 0.0])
        a[0] += 1
        a[1] += dt
    lines = ["Kernel trace of the App. B single-level relaxations (128^3 accuracy problem, Dirichlet,",
             "max residual <= 1e-10; RKL accelerated schedule with two-stage chunk passes, then SOR)",
             "command (from the repository root, TMPDIR=/tmp):",
             "  rocprofv3 --kernel-trace --output-format csv -d <DIR> -o relax -- python3 -m paper_2306_05332_amd.compare "
             "--methods rkl sor",
             "  python3 -m paper_2306_05332_amd.compare --summarize-trace <DIR>",
             "", "   calls  total_ms   avg_us  name"]
    for k, (c, s) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        lines.append(f"{c:8d} {s / 1e3:9.3f} {s / c:8.2f}  {k[:100]}")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--methods", nargs="+", default=["rkl", "sor", "gsrb"], choices=["rkl", "sor", "gsrb"])
    ap.add_argument("--summarize-trace", metavar="TRACE_DIR", help="print a summary of a kernel trace and exit")
    a = ap.parse_args(argv)
    if a.summarize_trace:
        print(summarize_trace(a.summarize_trace))
        return
    _lib.load_library()
    res = run(a.n, a.tol, methods=tuple(a.methods), log=lambda s: print(s, flush=True))
    base = next(r for r in res if r["method"] == "rkl")["seconds"]
    for r in res:
        print(f"{r['method']:>26}: {r['iterations']:>8} iterations  {r['seconds'] * 1e3:10.2f} ms"
              f"  ({r['seconds'] / base:6.2f} x RKL)", flush=True)


if __name__ == "__main__":
    main()
