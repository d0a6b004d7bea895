"""Tile autotuner for the fused tau-step, and the stage-count choice.

For every multigrid level shape of the grids asked for, the library times
each fused tau-step variant (LDS-ring or z-queue kernel, tile shape) and each
workgroup target with HIP events (``rkl_autotune``) and keeps the fastest.
Optionally it also times whole solves for several stage counts s and records
the fastest for ``Options(s=0)``.  Results are stored as JSON; the package
installs ``tuning/gfx950.json`` when the library is loaded (set
``RKL_TUNING=none`` to skip, or ``RKL_TUNING=<path>`` for another table).

    python -m paper_2306_05332_amd.autotune --sizes 256 128 --out table.json
"""
from __future__ import annotations

import argparse
import json
import os
import time

from . import _lib

DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "gfx950.json")


def tune_levels(shapes, s_list=(2,), bcs=("periodic",), precs=("fp64", "mixed"), reps=20, min_coarse=4,
                min_cells=16 ** 3, log=None):
    """Tune every distinct level shape of the given grids; returns the winning
    entries, each with the built-in choice's time beside it.  A shape
    (ny, nx) is a two-dimensional grid (its levels (1, ny_l, nx_l) with
    hz = inf; s = 4 there also covers a fused pair of s = 2 tau-steps)."""
    out, seen = [], set()
    for shape in shapes:
        h = (1.0, 1.0) if len(shape) == 2 else 1.0
        for bc in bcs:
            for lv in _lib.level_shapes(shape, min_coarse, bc):
                if lv[0] * lv[1] * lv[2] < min_cells:
                    continue
                for prec in precs:
                    for s in s_list:
                        key = (lv, bc, prec, s)
                        if key in seen or _lib.tau_step_launches(lv, s, bc, prec, h) != 1:
                            continue
                        seen.add(key)
                        _lib.tune_set([{"nx": lv[2], "ny": lv[1], "nz": lv[0], "bc": bc, "prec": prec, "s": s,
                                        "variant": 0, "target": 0}])
                        heur = _lib.tune_get(lv, s, bc, prec, h)
                        res = _lib.autotune_level(lv, s, bc, prec, reps, h)
                        best = dict(res[0])
                        hv = [r["us"] for r in res if r["variant"] == heur["variant"] and r["target"] == heur["target"]]
                        best["heuristic"] = f'{heur["variant"]}/{heur["target"]}'
                        best["heuristic_us"] = hv[0] if hv else None
                        best["candidates"] = len(res)
                        out.append(best)
                        if log:
                            log(f"{lv} {bc} {prec} s={s}: {best['variant']}/{best['target']} {best['us']:.1f} us "
                                f"(built-in {best['heuristic']} {best['heuristic_us']})")
    return out


def tune_stage_count(shape, bc="periodic", prec="fp64", s_list=(1, 2, 3), tol=1e-10, seed=0, reps=3, log=None):
    """Time full solves of a seeded blob field for each s; returns (best s, {s: ms})."""
    import torch

    import workloads as W
    n = shape[0]
    if not (shape[0] == shape[1] == shape[2]):
        raise ValueError("stage-count tuning uses cubic grids")
    p = W.gaussian_blobs(n, 16, seed=seed) if bc == "periodic" else W.uniform_sphere(n)
    rho = torch.from_numpy(p.rho).cuda()
    times = {}
    for s in s_list:
        o = _lib.Options(s=s, tol=tol, prec=prec, tau_frac=0.9)
        _lib.solve(rho, p.h, bc, opts=o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _lib.solve(rho, p.h, bc, opts=o)
        torch.cuda.synchronize()
        times[s] = 1e3 * (time.perf_counter() - t0) / reps
        if log:
            log(f"{shape} {bc} {prec} s={s}: {times[s]:.2f} ms")
    best = min(times, key=times.get)
    _lib.tune_set_s(shape, best, bc, prec)
    return best, times


def save(path, tiles, stage_counts=(), device=None):
    doc = {"device": device or "gfx950", "tiles": list(tiles), "stage_counts": list(stage_counts)}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(doc, fh, indent=1)


def load(path=DEFAULT_TABLE):
    """Install a stored table; returns the number of entries installed."""
    with open(path) as fh:
        doc = json.load(fh)
    tiles = doc.get("tiles", [])
    if tiles:
        _lib.tune_set(tiles)
    for e in doc.get("stage_counts", []):
        _lib.tune_set_s((e["nz"], e["ny"], e["nx"]), e["s"], e["bc"], e["prec"])
    return len(tiles) + len(doc.get("stage_counts", []))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--sizes", type=int, nargs="+", default=[512, 256, 128, 96, 64, 48, 32])
    ap.add_argument("--s", type=int, nargs="+", default=[2, 3])
    ap.add_argument("--bcs", nargs="+", default=["periodic", "dirichlet"])
    ap.add_argument("--precs", nargs="+", default=["fp64", "mixed"])
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--sizes2d", type=int, nargs="*", default=[4096, 2048],
                    help="square two-dimensional grids (levels down to 64^2)")
    ap.add_argument("--s2d", type=int, nargs="+", default=[2, 4], help="stage counts for 2-D levels (4: pairs)")
    ap.add_argument("--stage-count-sizes", type=int, nargs="*", default=[256, 128])
    ap.add_argument("--out", default=DEFAULT_TABLE)
    a = ap.parse_args(argv)
    import torch
    _lib.load_library()
    _lib.tune_clear()
    log = lambda m: print(m, flush=True)  # noqa: E731
    tiles = tune_levels([(n, n, n) for n in a.sizes], tuple(a.s), tuple(a.bcs), tuple(a.precs), a.reps, log=log)
    tiles += tune_levels([(n, n) for n in a.sizes2d], tuple(a.s2d), tuple(a.bcs), tuple(a.precs), a.reps,
                         log=log)
    stage = []
    for n in a.stage_count_sizes:
        for prec in a.precs:
            best, times = tune_stage_count((n, n, n), "periodic", prec, s_list=(1, 2, 3), log=log)
            stage.append({"nx": n, "ny": n, "nz": n, "bc": "periodic", "prec": prec, "s": best,
                          "ms": {str(k): v for k, v in times.items()}})
    save(a.out, tiles, stage, device=torch.cuda.get_device_properties(0).gcnArchName)
    print(f"wrote {len(tiles)} tile entries and {len(stage)} stage counts to {a.out}", flush=True)


if __name__ == "__main__":
    main()
