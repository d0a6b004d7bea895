"""Host-side sanitizer build of ``librklpoisson.so``.

The library's host code (argument checks, plan and hierarchy set-up, the
App. A.3 rule, tuning tables, error paths) compiled with AddressSanitizer
and UndefinedBehaviorSanitizer, without sanitizing the device code (the
device objects are built at -O1), for the ABI tests that call no kernel.
The result is loaded with the clang ASan runtime preloaded; see
tests/test_abi_sanitized.py.  Run ``python -m paper_2306_05332_amd.build_sanitized``.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

from .build import ARCH, CSRC, INCLUDE, PKG, SOURCES, hipcc

HOST_SAN_LIB = os.path.join(PKG, "_build", "librklpoisson_hostsan.so")
HOST_SAN_FLAGS = [
    "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined",
    "-Wno-unused-command-line-argument", "-I", CSRC, "-I", INCLUDE,
]


def asan_runtime() -> str:
    """Path of the clang AddressSanitizer runtime that hipcc links against."""
    res = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = res.stdout.strip()
    if res.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("clang ASan runtime not found")
    return path


def build_host_sanitized(jobs: int = 4) -> str:
    """Compile the host code of every source with ASan + UBSan and link
    HOST_SAN_LIB; returns its path."""
    objdir = os.path.join(PKG, "_build", "hostsan")
    os.makedirs(objdir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objs = [os.path.join(objdir, s.replace(".hip", ".o")) for s in srcs]

    def one(a):
        src, obj = a
        res = subprocess.run([hipcc(), *HOST_SAN_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj],
                             capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc (host sanitizer build) failed on {src}:\n{res.stderr}")

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(one, zip(srcs, objs)))
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", "-o", HOST_SAN_LIB, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link (host sanitizer build) failed:\n{res.stderr}")
    return HOST_SAN_LIB


if __name__ == "__main__":
    print(build_host_sanitized())
