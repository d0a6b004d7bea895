"""Benchmark: RKL-multigrid Poisson solve on one MI355X.

Workload (one "step"): a cold-start float64 solve of nabla^2 phi = 4 pi rho on
a 256^3 periodic box [0,1]^3, rho = 16 seeded Gaussian blobs (seed 2, widths
U[0.02,0.08], lognormal amplitudes, mean removed), to relative residual 1e-10
with the default V-cycle (s = 2, theta = 0.9, N_pre = 2, N_post = 1, down to 4^3).

Printed on one JSON line:
  value        finest-level cell-updates/s: 256^3 x (RKL stages applied on the
               finest level per solve) / wall time per solve
  roofline     the finest-level fused tau-step kernel, timed with HIP events on
               the solver's stream over 40 back-to-back launches: algorithmic
               bytes per launch (u and b read, Y_s written: 3 words per cell) /
               mean duration, against the 8 TB/s HBM peak; `traffic` is the
               HBM bytes per launch that rocprofv3 counted (FETCH_SIZE +
               WRITE_SIZE, each scaled by the same counter on a plain copy of
               known size), read from the committed counter summary when it was
               taken on the current kernel sources, else null
  cpu_baseline the CPU oracle (numpy, float64) on a bounded sample of the same
               workload: V-cycles from a cold start
Also: time to 1e-10 for the float64 and mixed-precision paths, cycles, the
max-norm error of each against the exact discrete solution (FFT), the batched
96-grid workload, the adjoint (forward + backward) of 8 x 128^3 solves, the 2-D
4096^2 solves, the uniform sphere with Dirichlet faces at 32^3 and 256^3, and
the 512^3 k^-3 random field solved in mixed precision and in float64 to 1e-10
(its error against the FFT solution).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
       python bench.py --pmc-probe                 (program run under rocprofv3 --pmc)
       python bench.py --summarize-pmc FETCH_DIR WRITE_DIR   (counter summary text)
       python bench.py --summarize-trace TRACE_DIR          (kernel-trace summary text)
       python bench.py --bc-probe                  (the same tau-step on both boundary types)
       python bench.py --summarize-bc-pmc DIR [DIR ...]     (its instruction counters)
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
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
SWEEP_STEPS = 40
COPY_BYTES = 256 * 1024 * 1024  # plain copy used to scale the HBM counters
PMC_SUMMARY = os.path.join(ROOT, "profiles", "fused_tau_256_fp64_pmc.txt")
KERNEL_SOURCES = ["paper_2306_05332_amd/csrc/fused.hip", "paper_2306_05332_amd/csrc/strip.hip",
                  "paper_2306_05332_amd/csrc/strip_body.h", "paper_2306_05332_amd/csrc/kernels.h",
                  "paper_2306_05332_amd/csrc/rkl_device.h", "paper_2306_05332_amd/tuning/gfx950.json"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and adjoint workloads")
    ap.add_argument("--cpu-cycles", type=int, default=6, help="oracle V-cycles in the CPU baseline sample")
    ap.add_argument("--pmc-probe", action="store_true")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-trace", metavar="TRACE_DIR")
    ap.add_argument("--only-two-d", action="store_true", help="run only the 2-D workload; print its JSON")
    ap.add_argument("--cfg3", action="store_true",
                    help="run only the 512^3 k^-3 random-field comparison (float64 vs mixed); print its JSON")
    ap.add_argument("--summarize-trace-2d", metavar="TRACE_DIR")
    ap.add_argument("--summarize-trace-cfg3", metavar="TRACE_DIR",
                    help="per-solve kernel times of a kernel trace of the --cfg3 run")
    ap.add_argument("--bc-probe", action="store_true",
                    help="six 256^3 float64 tau-steps of the stacked two-row strips, periodic then Dirichlet")
    ap.add_argument("--summarize-bc-pmc", nargs="+", metavar="DIR")
    return ap.parse_args()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def sources_digest():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        p = os.path.join(ROOT, rel)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def kernel_symbol(R, shape, s, prec="fp64"):
    """Demangled name prefix of the finest-level periodic tau-step kernel in
    effect (strip kernels: up to the last template argument, the store-hint
    flag, which the launcher picks from the level's size)."""
    tname = "double" if prec == "fp64" else "float"
    v = R.tune_get(shape, s, "periodic", prec)["variant"]
    strip = {"strip8x4": (8, 4), "strip8x1": (8, 1), "strip4x4": (4, 4), "strip5x1": (5, 1)}
    shy = {"stripyx8x4": (8, 4), "stripyx4x8": (4, 8), "stripyx8x8": (8, 8), "stripyx2x8": (2, 8),
           "stripyx2x16": (2, 16)}
    flat = {"strip2d8": 8, "strip2d4": 4}
    if v in strip:
        return f"rkl::k_tau_strip<{tname}, {s}, {strip[v][0]}, {strip[v][1]}, true, false, false, false, "
    if v in shy:
        return f"rkl::k_tau_strip_yx<{tname}, {s}, {shy[v][0]}, {shy[v][1]}, true, false, false, "
    if v in flat:
        r = flat[v] if (prec != "fp64" or s <= 2) else 4
        return f"rkl::k_tau_strip<{tname}, {s}, {r}, 1, true, false, false, true, "
    return {"ring64x8": f"rkl::k_fused_tau<{tname}, {s}, 64, 8>",
            "ring64x4": f"rkl::k_fused_tau<{tname}, {s}, 64, 4>",
            "zq64x32": f"rkl::k_tau_zq<{tname}, {s}, 64, 32, 512, 1, 0>",
            "zq64x16": f"rkl::k_tau_zq<{tname}, {s}, 64, 16, 256, 1, 0>"}.get(v, f"rkl::k_stage<{tname}>")


def sweep_inputs(torch, W, dev):
    prob = W.gaussian_blobs(N, 16, seed=2)
    rho = torch.from_numpy(prob.rho).to(dev)
    f = (4.0 * math.pi) * (rho - rho.mean())
    return prob, rho, f


def read_traffic():
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources and tuning table."""
    if not os.path.exists(PMC_SUMMARY):
        return None, "no counter summary"
    kv = {}
    for line in open(PMC_SUMMARY):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("sources_sha256_16") != sources_digest():
        return None, "kernel sources changed since the counters were taken"
    try:
        return float(kv["traffic_bytes_per_launch"]), "counters on the current sources"
    except (KeyError, ValueError):
        return None, "malformed counter summary"


# ---------------------------------------------------------------- profiler helpers
def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _find(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits[0]


def summarize_pmc(fetch_dir, write_dir):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the copy and of the
    finest-level tau-step kernel -> scaled HBM bytes per launch."""
    import paper_2306_05332_amd as R
    R.load_library()
    ksym = kernel_symbol(R, (N, N, N), 2)

    def per_kernel(d, counter):
        rows = [r for r in _rows(_find(d, "counter_collection.csv")) if r.get("Counter_Name") == counter]
        copy = [float(r["Counter_Value"]) for r in rows if "copy" in r["Kernel_Name"].lower()
                and int(r.get("Grid_Size", r.get("Grid_Size_X", "0")) or 0) > 0]
        kern = [float(r["Counter_Value"]) for r in rows if ksym in r["Kernel_Name"]]
        return copy, kern

    cf, kf = per_kernel(fetch_dir, "FETCH_SIZE")
    cw, kw = per_kernel(write_dir, "WRITE_SIZE")
    if not (cf and kf and cw and kw):
        raise SystemExit("counter rows for the copy or the tau-step kernel are missing")
    kib = COPY_BYTES / 1024.0
    sf = kib / max(cf)          # known bytes / counted, read side
    sw = kib / max(cw)          # write side
    fetch = sorted(kf)[len(kf) // 2] * 1024.0 * sf
    write = sorted(kw)[len(kw) // 2] * 1024.0 * sw
    alg = 3 * 8 * N ** 3
    lines = [
        "HBM traffic of the finest-level fused tau-step kernel, 256^3 float64, s = 2",
        "commands (run from /tmp with TMPDIR=/tmp; <repo> is the repository root):",
        "  rocprofv3 --pmc FETCH_SIZE --output-format csv -d <FETCH_DIR> -o pmc -- python3 <repo>/bench.py --pmc-probe",
        "  rocprofv3 --pmc WRITE_SIZE --output-format csv -d <WRITE_DIR> -o pmc -- python3 <repo>/bench.py --pmc-probe",
        "  python3 <repo>/bench.py --summarize-pmc <FETCH_DIR> <WRITE_DIR>",
        f"kernel: {ksym}",
        f"copy_bytes: {COPY_BYTES}",
        f"copy_fetch_kib_per_dispatch: {max(cf):.1f}",
        f"copy_write_kib_per_dispatch: {max(cw):.1f}",
        f"fetch_scale: {sf:.4f}",
        f"write_scale: {sw:.4f}",
        f"kernel_dispatches_counted: {len(kf)} fetch, {len(kw)} write",
        f"kernel_fetch_kib_median: {sorted(kf)[len(kf) // 2]:.1f}",
        f"kernel_write_kib_median: {sorted(kw)[len(kw) // 2]:.1f}",
        f"fetch_bytes_per_launch: {fetch:.0f}",
        f"write_bytes_per_launch: {write:.0f}",
        f"traffic_bytes_per_launch: {fetch + write:.0f}",
        f"algorithmic_bytes_per_launch: {alg}",
        f"traffic_over_algorithmic: {(fetch + write) / alg:.3f}",
        f"sources_sha256_16: {sources_digest()}",
    ]
    print("\n".join(lines))


def summarize_trace(d):
    """rocprofv3 --kernel-trace --stats of the bench command: the top kernels
    by total time, and the finest-level tau-step kernel's mean duration over
    its 256^3 launches and over the 40-launch sweep that bench.py times."""
    import paper_2306_05332_amd as R
    R.load_library()
    ksym = kernel_symbol(R, (N, N, N), 2)
    stats = _rows(_find(d, "kernel_stats.csv"))
    trace = _rows(_find(d, "kernel_trace.csv"))
    out = ["Kernel trace of the bench command",
           "command (from /tmp, TMPDIR=/tmp):",
           "  rocprofv3 --kernel-trace --stats --output-format csv -d <DIR> -o bench -- "
           "python3 <repo>/bench.py --no-cpu-baseline --no-extras --steps 3 --warmup 1",
           "  python3 <repo>/bench.py --summarize-trace <DIR>",
           "", "top kernels (rocprofv3 kernel_stats):",
           f"  {'calls':>6} {'total_ms':>9} {'avg_us':>8} {'pct':>6}  name"]
    for r in stats[:14]:
        name = r["Name"].split("(")[0].replace("void ", "")
        out.append(f"  {int(r['Calls']):>6} {float(r['TotalDurationNs']) / 1e6:>9.3f} "
                   f"{float(r['AverageNs']) / 1e3:>8.2f} {float(r['Percentage']):>6.2f}  {name}")
    mine = [r for r in trace if ksym in r["Kernel_Name"]]
    dur = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in mine]
    # the timed sweep: the last SWEEP_STEPS dispatches of the longest run of
    # consecutive dispatches of this kernel (2 untimed warm-up launches precede it)
    order = sorted(trace, key=lambda r: int(r["Start_Timestamp"]))
    best, cur = [], []
    for r in order:
        if ksym in r["Kernel_Name"]:
            cur.append(r)
            if len(cur) > len(best):
                best = list(cur)
        else:
            cur = []
    best = best[-SWEEP_STEPS:]
    sw = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in best]
    span = (int(best[-1]["End_Timestamp"]) - int(best[0]["Start_Timestamp"])) / 1e3 / len(best)
    out += ["", f"finest-level tau-step kernel: {ksym}",
            f"  all launches of this kernel (any level): {len(dur)}, mean {sum(dur) / len(dur):.2f} us",
            f"  timed sweep at 256^3: {len(sw)} launches, mean duration {sum(sw) / len(sw):.2f} us "
            f"(min {min(sw):.2f}, max {max(sw):.2f}); first start to last end / launches {span:.2f} us",
            f"  algorithmic bytes per launch: {3 * 8 * N ** 3} -> "
            f"{3 * 8 * N ** 3 / (sum(sw) / len(sw)) / 1e3:.1f} GB/s over the sweep"]
    print("\n".join(out))


def summarize_trace_cfg3(d, top=10):
    """Kernel trace of the --cfg3 run: per-solve kernel times of its four
    cases (512^3 random field float64 / mixed, then 256^3 blobs float64 /
    mixed, four solves each, the first of each case untimed).  A solve's
    window opens at its source scaling pass (k_scale); the second and third
    solves of a case are averaged (the fourth is followed by the copy of phi
    to the host and the next case's set-up).  Kernels are grouped by name."""
    trace = sorted(_rows(_find(d, "kernel_trace.csv")), key=lambda r: int(r["Start_Timestamp"]))
    starts = [i for i, r in enumerate(trace) if "k_scale(" in r["Kernel_Name"]]
    cases = ["512^3 k^-3 random field, float64", "512^3 k^-3 random field, mixed",
             "256^3 blobs, float64", "256^3 blobs, mixed"]
    out = ["Kernel trace of the 512^3 / 256^3 mixed-against-float64 comparison (bench.py --cfg3)",
           "command (from /tmp, TMPDIR=/tmp):",
           "  rocprofv3 --kernel-trace --output-format csv -d <DIR> -o cfg3 -- python3 <repo>/bench.py --cfg3",
           "  python3 <repo>/bench.py --summarize-trace-cfg3 <DIR>",
           f"solves found: {len(starts)} (expected 16: four cases of one untimed and three timed solves)",
           "per case: the mean of its second and third solves"]
    bounds = starts + [len(trace)]
    for c, label in enumerate(cases):
        solves = [4 * c + 1, 4 * c + 2]
        if solves[-1] + 1 >= len(bounds):
            break
        tot, calls = {}, {}
        span = 0.0
        for k in solves:
            rows = trace[bounds[k]:bounds[k + 1]]
            span += (int(rows[-1]["End_Timestamp"]) - int(rows[0]["Start_Timestamp"])) / 1e3
            for r in rows:
                name = r["Kernel_Name"].split("(")[0].replace("void ", "")
                dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
                tot[name] = tot.get(name, 0.0) + dur
                calls[name] = calls.get(name, 0) + 1
        ns = len(solves)
        busy = sum(tot.values()) / ns
        out += ["", f"{label}: {span / ns / 1e3:.2f} ms per solve from its first kernel to its last "
                f"(kernels busy {busy / 1e3:.2f} ms)",
                f"  {'us/solve':>9} {'calls':>6} {'avg_us':>8}  name"]
        for name, t in sorted(tot.items(), key=lambda kv: -kv[1])[:top]:
            out.append(f"  {t / ns:>9.1f} {calls[name] / ns:>6.1f} {t / calls[name]:>8.1f}  {name}")
    print("\n".join(out))


TWO_D_KERNEL = "rkl::k_tau_strip<double, 4, 4, 1, true, false, false, true, "


def summarize_trace_2d(d):
    """rocprofv3 --kernel-trace --stats of the 2-D workload: the top kernels,
    and the 4096^2 pair pass's mean duration over the timed sweep."""
    stats = _rows(_find(d, "kernel_stats.csv"))
    trace = _rows(_find(d, "kernel_trace.csv"))
    out = ["Kernel trace of the two-dimensional workload (periodic 4096^2, float64 and mixed solves, pair-pass sweep)",
           "command (from /tmp, TMPDIR=/tmp):",
           "  rocprofv3 --kernel-trace --stats --output-format csv -d <DIR> -o two_d -- "
           "python3 <repo>/bench.py --only-two-d",
           "  python3 <repo>/bench.py --summarize-trace-2d <DIR>",
           "", "top kernels (rocprofv3 kernel_stats):",
           f"  {'calls':>6} {'total_ms':>9} {'avg_us':>8} {'pct':>6}  name"]
    for r in stats[:14]:
        name = r["Name"].split("(")[0].replace("void ", "")
        out.append(f"  {int(r['Calls']):>6} {float(r['TotalDurationNs']) / 1e6:>9.3f} "
                   f"{float(r['AverageNs']) / 1e3:>8.2f} {float(r['Percentage']):>6.2f}  {name}")
    order = sorted(trace, key=lambda r: int(r["Start_Timestamp"]))
    gsize = lambda r: int(r.get("Grid_Size_X", r.get("Grid_Size", "0")) or 0)  # noqa: E731
    top = max(gsize(r) for r in order if TWO_D_KERNEL in r["Kernel_Name"])  # the 4096^2 launches
    best, cur = [], []
    for r in order:
        if TWO_D_KERNEL in r["Kernel_Name"] and gsize(r) == top:
            cur.append(r)
            if len(cur) > len(best):
                best = list(cur)
        else:
            cur = []
    sw = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in best[-(SWEEP_STEPS // 2):]]
    n = 4096
    out += ["", f"2-D pair pass (two s = 2 tau-steps in one 4-stage pass): {TWO_D_KERNEL}",
            f"  timed sweep at 4096^2: {len(sw)} launches, mean duration {sum(sw) / len(sw):.2f} us "
            f"(min {min(sw):.2f}, max {max(sw):.2f})",
            f"  algorithmic bytes per launch: {3 * 8 * n * n} -> {3 * 8 * n * n / (sum(sw) / len(sw)) / 1e3:.1f} GB/s"]
    print("\n".join(out))


# ---------------------------------------------------------------- probes
def pmc_probe():
    """A plain copy of COPY_BYTES (three times) and ten finest-level tau-steps."""
    import torch

    import paper_2306_05332_amd as R
    import workloads as W
    dev = torch.device("cuda:0")
    R.load_library()
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    _, rho, f = sweep_inputs(torch, W, dev)
    u = torch.zeros_like(rho)
    R.smooth(f, u, (1.0 / N,) * 3, "periodic", s=2, tau_frac=0.9, n_steps=10)
    torch.cuda.synchronize()
    print("pmc probe done", flush=True)


BC_COUNTERS = ["SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_VMEM_RD SQ_INSTS_LDS SQ_WAVE_CYCLES SQ_WAIT_INST_ANY "
               "SQ_BUSY_CYCLES SQ_WAVES",
               "SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 SQ_ACTIVE_INST_VALU "
               "SQ_INST_CYCLES_VMEM SQ_WAIT_ANY SQ_INSTS_VMEM_WR SQ_ACTIVE_INST_ANY"]


def bc_probe():
    """Six float64 tau-steps (s = 2) of the stacked two-row strips (8
    wavefronts, 480 workgroups) at 256^3 on a periodic box, then six on a
    Dirichlet box, from the same random right-hand side."""
    import numpy as np
    import torch

    import paper_2306_05332_amd as R
    R.load_library()
    rng = np.random.default_rng(1)
    f = torch.from_numpy(rng.standard_normal((N, N, N))).cuda()
    for bc in ("periodic", "dirichlet"):
        R.tune_clear()
        R.tune_set([{"nx": N, "ny": N, "nz": N, "bc": bc, "prec": "fp64", "s": 2, "variant": "stripyx2x8",
                     "target": 480}])
        phi = torch.zeros_like(f)
        R.smooth(f, phi, (1.0 / N,) * 3, bc, s=2, n_steps=6)
        torch.cuda.synchronize()
    R.tune_clear()
    print("bc probe done", flush=True)


def summarize_bc_pmc(dirs):
    """Per-launch means of the counters that --bc-probe runs collected, for
    the periodic and the Dirichlet instantiation of the strip kernel."""
    sums = {}
    for d in dirs:
        for path in glob.glob(os.path.join(d, "*counter_collection.csv")):
            for r in csv.DictReader(open(path)):
                name = r["Kernel_Name"].split("(")[0].replace("void ", "")
                if "k_tau_strip_yx" not in name:
                    continue
                key = (name, r["Counter_Name"])
                sums.setdefault(key, {})
                sums[key][r["Dispatch_Id"]] = sums[key].get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    out = ["Instruction counters of the 256^3 float64 stacked two-row strip tau-step, periodic vs Dirichlet box",
           "commands (from /tmp, TMPDIR=/tmp), one counter set per run:"]
    for c in BC_COUNTERS:
        out.append(f"  rocprofv3 --pmc {c} --output-format csv -d <DIR> -o bc -- python3 <repo>/bench.py --bc-probe")
    out.append("  python3 <repo>/bench.py --summarize-bc-pmc <DIR> [<DIR> ...]")
    out.append("sources_sha256_16: " + sources_digest())
    # durations, from a kernel trace of the same program among the directories
    durs = {}
    for d in dirs:
        for path in glob.glob(os.path.join(d, "*kernel_trace.csv")):
            for r in csv.DictReader(open(path)):
                name = r["Kernel_Name"].split("(")[0].replace("void ", "")
                if "k_tau_strip_yx" in name:
                    durs.setdefault(name, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0)
    if durs:
        out.append("  rocprofv3 --kernel-trace --stats --output-format csv -d <DIR> -o bc -- python3 <repo>/bench.py "
                   "--bc-probe   (durations)")
    kernels = sorted({k[0] for k in sums} | set(durs))
    counters = sorted({k[1] for k in sums})
    for kern in kernels:
        out.append(f"{kern}  ({'periodic' if ', true, false, false, ' in kern else 'Dirichlet'})")
        if kern in durs:
            v = durs[kern]
            out.append(f"  {'duration_us':24s} {sum(v) / len(v):14.4g}  (mean of {len(v)} launches, "
                       f"min {min(v):.1f}, max {max(v):.1f})")
        for c in counters:
            per = sums.get((kern, c))
            if per:
                out.append(f"  {c:24s} {sum(per.values()) / len(per):14.4g}  (mean of {len(per)} launches)")
    print("\n".join(out))


def main():
    args = parse()
    if args.summarize_bc_pmc:
        return summarize_bc_pmc(args.summarize_bc_pmc)
    if args.bc_probe:
        return bc_probe()
    if args.summarize_pmc:
        return summarize_pmc(*args.summarize_pmc)
    if args.summarize_trace:
        return summarize_trace(args.summarize_trace)
    if args.summarize_trace_2d:
        return summarize_trace_2d(args.summarize_trace_2d)
    if args.summarize_trace_cfg3:
        return summarize_trace_cfg3(args.summarize_trace_cfg3)
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (this solver's path is single-GPU); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if args.pmc_probe:
        return pmc_probe()
    if args.cfg3:
        import torch

        import paper_2306_05332_amd as R
        import workloads as W
        if not torch.cuda.is_available():
            print("bench.py needs a GPU", file=sys.stderr)
            sys.exit(2)
        R.load_library()
        print(json.dumps(run_cfg3(R, W, torch)), flush=True)
        return
    if args.only_two_d:
        import torch

        import paper_2306_05332_amd as R
        import workloads as W
        if not torch.cuda.is_available():
            print("bench.py needs a GPU", file=sys.stderr)
            sys.exit(2)
        R.load_library()
        print(json.dumps(run_two_d(R, W, torch)), flush=True)
        return
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

    prob, rho, f = sweep_inputs(torch, W, dev)
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

    # ---------------- dominant kernel: finest-level tau-step, HIP events on the solver's stream
    u = torch.zeros_like(rho)
    R.smooth(f, u, h, "periodic", s=opts.s, tau_frac=opts.tau_frac, n_steps=2)  # warm
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    R.smooth(f, u, h, "periodic", s=opts.s, tau_frac=opts.tau_frac, n_steps=SWEEP_STEPS)
    ev1.record(stream)
    torch.cuda.synchronize()
    sweep_ms = ev0.elapsed_time(ev1)
    info = R.kernel_info(tuple(rho.shape), opts.s, "periodic", "fp64")
    launches = SWEEP_STEPS * info["launches_per_tau"]
    t_launch_s = sweep_ms * 1e-3 / launches
    achieved = info["bytes_per_launch"] / t_launch_s / 1e9
    traffic, traffic_note = read_traffic()
    print(f"# sweep: {t_launch_s * 1e6:.2f} us per launch, {achieved:.0f} GB/s", flush=True)

    # achievable ceiling of this HBM: a plain device-to-device copy (read + write)
    ca = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
    cb = torch.empty_like(ca)
    for _ in range(3):
        cb.copy_(ca)
    ev0.record(stream)
    for _ in range(20):
        cb.copy_(ca)
    ev1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * COPY_BYTES * 20 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del ca, cb
    print(f"# device copy: {copy_gbs:.0f} GB/s", flush=True)

    # ---------------- accuracy vs the exact discrete solution (CPU FFT)
    from oracle import exact
    us = exact.exact_solution(4.0 * math.pi * prob.rho, h, "periodic")
    den = np.abs(us).max()
    err64 = float(np.abs(phi.cpu().numpy() - us).max() / den)
    errm = float(np.abs(phim.cpu().numpy() - us).max() / den)

    stages0 = st.cycles * (opts.n_pre + opts.n_post) * opts.s
    value = n3 * stages0 / t_fp64

    extras = {}
    if not args.no_extras:
        extras = run_extras(R, W, torch, args)

    # ---------------- CPU oracle baseline (bounded sample)
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import multigrid as omg
        from oracle import operators as oop
        g = oop.Grid(N, N, N, *h, "periodic")
        fo = omg.prepare_source(prob.rho, g, omg.Options())
        lv = oop.build_hierarchy(g)
        uo = np.zeros(g.shape)
        ncyc = args.cpu_cycles
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
        "sweep_cell_updates_per_s": n3 * opts.s / t_launch_s,
        "achievable_ceiling": {"kernel": "device-to-device copy of 256 MiB (read + write)", "GB/s": copy_gbs,
                               "sweep_frac_of_ceiling": achieved / copy_gbs},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_note": traffic_note,
                     "kernel": kernel_symbol(R, (N, N, N), opts.s), "bytes_per_launch": info["bytes_per_launch"],
                     "mean_launch_us": t_launch_s * 1e6, "launches_timed": launches},
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


def run_extras(R, W, torch, args):
    """The batched workload (96 periodic grids of 32^3..128^3, mixed, tol 1e-8),
    the adjoint workload (8 x 128^3, forward + backward, float64) and the
    two-dimensional workload (periodic 4096^2)."""
    out = {}
    probs = W.batch_blob_problems(seed=4)
    rhos = [torch.from_numpy(p.rho).cuda() for p in probs]
    hs = [p.h for p in probs]
    cells = sum(p.rho.size for p in probs)
    ob = R.Options(tol=1e-8, prec="mixed")
    for _ in range(2):  # plans, graph capture and the first launches of its branches
        R.solve_batched(rhos, hs, "periodic", opts=ob)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        _, sts = R.solve_batched(rhos, hs, "periodic", opts=ob)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for r, hh in zip(rhos, hs):
        R.solve(r, hh, "periodic", opts=ob)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    cyc = [s.cycles for s in sts]
    out["batched"] = {"grids": len(probs), "cells": cells, "prec": "mixed", "tol": 1e-8, "ms": tb * 1e3,
                      "sequential_ms": ts * 1e3, "speedup_vs_sequential": ts / tb,
                      "cycles_min_max": [min(cyc), max(cyc)],
                      "vcycle_cell_updates_per_s": sum(p.rho.size * s.cycles for p, s in zip(probs, sts)) / tb}
    print(f"# batched: {tb * 1e3:.2f} ms ({ts * 1e3:.1f} ms one by one)", flush=True)
    del rhos

    rhos, w, _ = W.adjoint_inputs(128, nbatch=8, ndirs=1, seed=5)
    rho = torch.from_numpy(rhos).cuda().requires_grad_(True)
    wt = torch.from_numpy(w).cuda()
    h = (1.0 / 128,) * 3
    oa = R.Options(tol=1e-10)
    fw, bw = [], []
    for rep in range(4):  # the first pass (plans, capture) is not counted
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi = R.poisson_solve(rho, h, "periodic", opts=oa)
        loss = (wt * phi).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        rho.grad = None
        if rep > 0:
            fw.append((t1 - t0) * 1e3)
            bw.append((t2 - t1) * 1e3)
    fms, bms = sum(fw) / len(fw), sum(bw) / len(bw)
    out["adjoint"] = {"grids": 8, "n": 128, "prec": "fp64", "tol": 1e-10, "forward_ms": fms, "backward_ms": bms,
                      "reps": len(fw)}
    print(f"# adjoint 8x128^3: forward {fms:.2f} ms, backward {bms:.2f} ms", flush=True)
    del rho, wt, phi

    out["two_d"] = run_two_d(R, W, torch)
    out["sphere32"] = run_sphere32(R, W, torch)
    out["sphere256"] = run_sphere256(R, W, torch)
    out["cfg3"] = run_cfg3(R, W, torch, with_blobs=False)
    return out


def run_sphere32(R, W, torch):
    """The 32^3 uniform sphere (Dirichlet faces from -M/r), float64 to 1e-10:
    a latency-bound solve, reported as wall time; its L2 error against the
    continuous potential (the density is point-sampled at cell centres)."""
    import numpy as np
    p = W.uniform_sphere(32)
    rho = torch.from_numpy(p.rho).cuda()
    faces = R.pack_faces(p.faces)
    o = R.Options(tol=TOL)
    R.solve(rho, p.h, "dirichlet", faces=faces, opts=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 20
    for _ in range(reps):
        phi, st = R.solve(rho, p.h, "dirichlet", faces=faces, opts=o)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    e = phi.cpu().numpy() - p.phi_exact
    l2 = float(np.sqrt(np.mean(e * e)) / np.sqrt(np.mean(p.phi_exact ** 2)))
    print(f"# sphere 32^3: {t * 1e3:.3f} ms, cycles={st.cycles}, L2 error vs analytic {l2:.3e}", flush=True)
    return {"n": 32, "bc": "dirichlet", "tol": TOL, "ms": t * 1e3, "cycles": st.cycles,
            "rel_l2_error_vs_analytic": l2}


def run_sphere256(R, W, torch):
    """The same uniform sphere at 256^3 (Dirichlet faces from -M/r, the
    boundary data folded into the right-hand side), float64 and mixed to
    1e-10: Dirichlet at scale, wall time per solve."""
    import numpy as np
    p = W.uniform_sphere(256)
    rho = torch.from_numpy(p.rho).cuda()
    faces = R.pack_faces(p.faces)
    res = {"n": 256, "bc": "dirichlet", "tol": TOL}
    for prec in ("fp64", "mixed"):
        o = R.Options(tol=TOL, prec=prec)
        R.solve(rho, p.h, "dirichlet", faces=faces, opts=o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            phi, st = R.solve(rho, p.h, "dirichlet", faces=faces, opts=o)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        e = phi.cpu().numpy() - p.phi_exact
        l2 = float(np.sqrt(np.mean(e * e)) / np.sqrt(np.mean(p.phi_exact ** 2)))
        res[prec] = {"ms": t * 1e3, "cycles": st.cycles, "rel_l2_error_vs_analytic": l2}
        print(f"# sphere 256^3 {prec}: {t * 1e3:.3f} ms, cycles={st.cycles}, L2 error vs analytic {l2:.3e}",
              flush=True)
    del rho, faces, phi
    return res


def run_cfg3(R, W, torch, n=512, with_blobs=True):
    """512^3 periodic k^-3 random field (seed 3): mixed precision against
    float64, time to 1e-10 and max error against the FFT solution; and (with
    with_blobs) the 256^3 blob field (seed 2) for the same pair."""
    import numpy as np
    from oracle import exact
    out = {}
    cases = [("grf512", lambda: W.gaussian_random_field(n, seed=3))]
    if with_blobs:
        cases.append(("blobs256", lambda: W.gaussian_blobs(N, 16, seed=2)))
    for label, make in cases:
        prob = make()
        rho = torch.from_numpy(prob.rho).cuda()
        us = exact.exact_solution(4.0 * math.pi * prob.rho, prob.h, "periodic")
        res = {"n": prob.rho.shape[0]}
        for prec in ("fp64", "mixed"):
            o = R.Options(tol=TOL, prec=prec)
            R.solve(rho, prob.h, "periodic", opts=o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 3
            for _ in range(reps):
                phi, st = R.solve(rho, prob.h, "periodic", opts=o)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / reps
            err = float(np.abs(phi.cpu().numpy() - us).max() / np.abs(us).max())
            res[prec] = {"ms": t * 1e3, "cycles": st.cycles, "rel_res": st.rel_res, "max_rel_err_vs_fft": err}
            print(f"# {label} {prec}: {t * 1e3:.2f} ms, cycles={st.cycles}, err {err:.2e}", flush=True)
        res["mixed_speedup"] = res["fp64"]["ms"] / res["mixed"]["ms"]
        out[label] = res
        del rho
    return out


# 4096^2 in two dimensions: the exact discrete solution rounded to float64
# already has ||M u* - f|| / ||f|| = 1.55e-10 (eps Lambda ||u|| / ||f||, growing
# as n^2), so the 2-D solves stop at 1e-9, above that floor
TOL_2D = 1e-9


def run_two_d(R, W, torch, n=4096):
    """Two-dimensional workload: periodic 4096^2 (the cell count of 256^3),
    32 seeded Gaussian blobs, float64 and mixed solves to 1e-9, and the
    finest-level 2-D strip pass timed with HIP events on the solver's stream.
    On 2-D levels two s = 2 tau-steps run as one 4-stage pass (u and b read
    once, the result written once: 3 words of algorithmic traffic per cell
    per pass, for two tau-steps)."""
    import numpy as np
    from oracle import exact
    p = W.gaussian_blobs_2d(n, n, nblobs=32, seed=6)
    rho = torch.from_numpy(p.rho).cuda()
    res = {"n": n, "bc": "periodic", "tol": TOL_2D}
    us = exact.exact_solution(4.0 * math.pi * p.rho, p.h, "periodic")
    for prec in ("fp64", "mixed"):
        o = R.Options(tol=TOL_2D, prec=prec)
        R.solve(rho, p.h, "periodic", opts=o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            phi, st = R.solve(rho, p.h, "periodic", opts=o)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        err = float(np.abs(phi.cpu().numpy() - us).max() / np.abs(us).max())
        res[prec] = {"ms": t * 1e3, "cycles": st.cycles, "rel_res": st.rel_res, "max_rel_err_vs_exact": err}
        print(f"# 2-D {n}^2 {prec}: {t * 1e3:.3f} ms, cycles={st.cycles}", flush=True)
    f = rho * (4.0 * math.pi)
    u = torch.zeros_like(rho)
    stream = torch.cuda.current_stream()
    R.smooth(f, u, p.h, "periodic", s=2, n_steps=2)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    R.smooth(f, u, p.h, "periodic", s=2, n_steps=SWEEP_STEPS)
    ev1.record(stream)
    torch.cuda.synchronize()
    assert SWEEP_STEPS % 2 == 0 and R.tau_step_launches((n, n), 4) == 1
    launches = SWEEP_STEPS // 2  # pairs of tau-steps, one 4-stage pass each
    t_launch = ev0.elapsed_time(ev1) * 1e-3 / launches
    nbytes = 3 * 8 * n * n
    ach = nbytes / t_launch / 1e9
    res["tau_pair_pass"] = {"kernel": TWO_D_KERNEL,
                            "tau_steps_per_launch": 2, "mean_launch_us": t_launch * 1e6,
                            "us_per_tau_step": t_launch * 1e6 / 2, "bytes_per_launch": nbytes,
                            "achieved_GBs": ach, "frac_of_hbm_peak": ach / HBM_PEAK_GBS}
    print(f"# 2-D tau-step pair pass: {t_launch * 1e6:.2f} us, {ach:.0f} GB/s", flush=True)
    return res


if __name__ == "__main__":
    main()
