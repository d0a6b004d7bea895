"""Benchmark: RKL-multigrid Poisson solve on one MI355X.

Workload (one "step"): a cold-start float64 solve of nabla^2 phi = 4 pi rho on
a 256^3 periodic box [0,1]^3, rho = 16 seeded Gaussian blobs (seed 2, widths
U[0.02,0.08], lognormal amplitudes, mean removed), to relative residual 1e-10
with the default V-cycle (s = 2, theta = 0.9, N_pre = 2, N_post = 1, down to 4^3).

Printed on one JSON line:
  value        finest-level cell-updates/s: 256^3 x (RKL stages applied on the
               finest level per solve) / wall time per solve
  roofline     the finest-level RKL sweep kernel, timed with HIP events on the
               solver's stream: algorithmic bytes per launch / mean duration
               against the 8 TB/s HBM peak
  cpu_baseline the CPU oracle (numpy, float64) on a bounded sample of the same
               workload: two V-cycles from a cold start
Also: time to 1e-10 for the float64 and mixed-precision paths, cycles, and the
max-norm error of each against the exact discrete solution (FFT).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-updates/s and time-to-1e-10 residual at 256^3 (mixed vs FP64); HBM GB/s %"
HBM_PEAK_GBS = 8000.0
N = 256
TOL = 1e-10


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep-steps", type=int, default=40, help="tau-steps in the kernel timing region")
    return ap.parse_args()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (this solver's path is single-GPU); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2306_05332_amd as R
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    R.load_library()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)

    prob = W.gaussian_blobs(N, 16, seed=2)
    rho = torch.from_numpy(prob.rho).to(dev)
    h = prob.h
    opts = R.Options(tol=TOL)
    opts_mixed = R.Options(tol=TOL, prec="mixed")
    n3 = N ** 3

    def solve(o):
        return R.solve(rho, h, "periodic", opts=o)

    # ---------------- warmup (plans, first-touch)
    for _ in range(args.warmup):
        phi, st = solve(opts)
        phim, stm = solve(opts_mixed)
    torch.cuda.synchronize()

    # ---------------- timed region: K float64 solves
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        phi, st = solve(opts)
    torch.cuda.synchronize()
    t_fp64 = (time.perf_counter() - t0) / args.steps
    print(f"# fp64 solve: {t_fp64 * 1e3:.3f} ms, cycles={st.cycles}, rel_res={st.rel_res:.3e}", flush=True)

    # mixed precision, same field, same stop rule
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        phim, stm = solve(opts_mixed)
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / args.steps
    print(f"# mixed solve: {t_mixed * 1e3:.3f} ms, outer={stm.cycles}, rel_res={stm.rel_res:.3e}", flush=True)

    # ---------------- dominant kernel: finest-level RKL sweep, HIP events on the solver's stream
    f = (4.0 * math.pi) * (rho - rho.mean())
    u = torch.zeros_like(rho)
    R.smooth(f, u, h, "periodic", s=opts.s, tau_frac=opts.tau_frac, n_steps=2)  # warm
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ksteps = args.sweep_steps
    ev0.record(stream)
    R.smooth(f, u, h, "periodic", s=opts.s, tau_frac=opts.tau_frac, n_steps=ksteps)
    ev1.record(stream)
    torch.cuda.synchronize()
    sweep_ms = ev0.elapsed_time(ev1)
    info = R.kernel_info(tuple(rho.shape), opts.s, "periodic", "fp64")
    launches = ksteps * info["launches_per_tau"]
    t_launch_s = sweep_ms * 1e-3 / launches
    achieved = info["bytes_per_launch"] / t_launch_s / 1e9

    # ---------------- accuracy vs the exact discrete solution (CPU FFT)
    from oracle import exact
    us = exact.exact_solution(4.0 * math.pi * prob.rho, h, "periodic")
    den = np.abs(us).max()
    err64 = float(np.abs(phi.cpu().numpy() - us).max() / den)
    errm = float(np.abs(phim.cpu().numpy() - us).max() / den)

    stages0 = st.cycles * (opts.n_pre + opts.n_post) * opts.s
    value = n3 * stages0 / t_fp64

    # ---------------- CPU oracle baseline (bounded sample: 2 V-cycles)
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import multigrid as omg
        from oracle import operators as oop
        g = oop.Grid(N, N, N, *h, "periodic")
        fo = omg.prepare_source(prob.rho, g, omg.Options())
        lv = oop.build_hierarchy(g)
        uo = np.zeros(g.shape)
        ncyc = 2
        t0 = time.perf_counter()
        for _ in range(ncyc):
            uo = omg.vcycle(uo, fo, lv, omg.Options())
        tc = time.perf_counter() - t0
        cpu = {"value": n3 * ncyc * (opts.n_pre + opts.n_post) * opts.s / tc, "unit": "cell-updates/s",
               "cores": 1, "kind": "oracle",
               "sample": f"{ncyc} V-cycles of the numpy float64 oracle on the same 256^3 field from a cold "
                         f"start ({tc:.1f} s; {cpu_model()}, {os.cpu_count()} host threads visible, numpy "
                         f"elementwise ops single-threaded)",
               "seconds_per_vcycle": tc / ncyc,
               "est_time_to_tol_s": tc / ncyc * st.cycles}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_fp64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "fp64 periodic 256^3 Poisson solve to relative residual 1e-10, cold start; "
                               "rho = 16 seeded Gaussian blobs (seed 2), mean removed",
                   "n": N, "bc": "periodic", "tol": TOL, "s": opts.s, "tau_frac": opts.tau_frac,
                   "n_pre": opts.n_pre, "n_post": opts.n_post, "coarsest": 4},
        "time_to_tol_ms": {"fp64": t_fp64 * 1e3, "mixed": t_mixed * 1e3},
        "cycles": {"fp64": st.cycles, "mixed": stm.cycles},
        "rel_res": {"fp64": st.rel_res, "mixed": stm.rel_res},
        "max_rel_err_vs_exact": {"fp64": err64, "mixed": errm},
        "vcycle_cell_updates_per_s": n3 * st.cycles / t_fp64,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": info["kernel"], "bytes_per_launch": info["bytes_per_launch"],
                     "mean_launch_us": t_launch_s * 1e6, "launches_timed": launches},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
