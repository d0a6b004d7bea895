"""Build the gfx950 shared library ``librklpoisson.so`` in the package directory.

Every HIP source under ``csrc/`` is compiled with hipcc for gfx950 and linked
into one shared library exporting the C ABI of ``include/rkl_poisson.h``.
Packed-FP32 instructions are disabled on purpose (``-packed-fp32-ops``).
Run ``python -m paper_2306_05332_amd.build`` or call ``build()``.
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "librklpoisson.so")
ARCH = os.environ.get("RKL_OFFLOAD_ARCH", "gfx950")

SOURCES = ["strip.hip", "strip_forms64.hip", "strip_forms32.hip", "strip_rs.hip", "kernels.hip", "transfer.hip",
           "coarse.hip", "tail.hip", "fused.hip", "plan.hip", "solve.hip", "batch.hip", "tune.hip", "levels.hip",
           "noalloc.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", CSRC, "-I", INCLUDE,
]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; the HIP toolchain is required to build librklpoisson.so")
    return exe


# LDS-poison debug build: the same sources with -DRKL_LDS_POISON (every
# kernel fills its floating-point LDS arrays with NaN on entry), for the GPU
# test that reruns the parity cases of the LDS-using kernels against it
# (tests/test_gpu_lds_poison.py).  A digest of the sources it was built from
# sits beside it, so a stale build is recognised.
POISON_LIB = os.path.join(PKG, "librklpoisson_ldspoison.so")
POISON_DIGEST = POISON_LIB + ".sources"


def sources_digest() -> str:
    """sha256 over the library's source and header texts (sorted by name)."""
    h = hashlib.sha256()
    for d in (CSRC, INCLUDE):
        for name in sorted(os.listdir(d)):
            if name.endswith((".hip", ".h")):
                h.update(name.encode())
                with open(os.path.join(d, name), "rb") as f:
                    h.update(f.read())
    return h.hexdigest()[:16]


def _compile(src, obj, verbose, extra=()):
    cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{res.stdout}\n{res.stderr}")
    return res.stderr


def _link(objs, out, verbose):
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = False, jobs: int = 8, lds_poison: bool = True) -> str:
    """Compile all sources and link the library (and, with lds_poison, the
    LDS-poison debug library); returns the library's path."""
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    variants = [("_build", (), LIB)]
    if lds_poison:
        variants.append((os.path.join("_build", "ldspoison"), ("-DRKL_LDS_POISON",), POISON_LIB))
    digest = sources_digest()
    tasks, objsets = [], []
    for sub, extra, _ in variants:
        objdir = os.path.join(PKG, sub)
        os.makedirs(objdir, exist_ok=True)
        objs = [os.path.join(objdir, s.replace(".hip", ".o")) for s in srcs]
        objsets.append(objs)
        tasks += [(s, o, extra) for s, o in zip(srcs, objs)]
    # longest compiles first
    tasks.sort(key=lambda a: 0 if a[0].startswith("strip") else 1)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda a: _compile(a[0], a[1], verbose, a[2]), tasks))
    for (_, _, out), objs in zip(variants, objsets):
        _link(objs, out, verbose)
    if lds_poison:
        with open(POISON_DIGEST, "w") as f:
            f.write(digest + "\n")
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
