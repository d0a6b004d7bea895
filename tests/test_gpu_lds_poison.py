"""LDS-poison debug build: the parity cases of every kernel that uses LDS
(LDS-ring and z-queue tau-steps, the stacked-strip halo exchange, the
residual / restriction and prolongation tiles, the folded mixed update,
the GS-RB passes, the coarsest-level solvers, the one-workgroup coarse tail,
the 2-D transfers) rerun against
``librklpoisson_ldspoison.so``, whose kernels fill their floating-point LDS
arrays with NaN on entry.  A read of an LDS element that no thread of the
launch wrote then turns results into NaN and the oracle comparison fails.

The cases run in one child process (the library is chosen by RKL_LIB when
the package loads it).  The debug library is built next to the ordinary one
by ``build()``; a digest of the sources it was built from must match the
current sources."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CASES = [
    "tests/test_gpu_parity.py",
    "tests/test_gpu_tuning.py::test_forced_variant_matches_oracle",
    "tests/test_gpu_fusion.py",
    "tests/test_gpu_2d.py",
    "tests/test_gpu_f32.py",
    "tests/test_gpu_gsrb.py",
    "tests/test_gpu_mixed_fold.py",
]


@pytest.mark.timeout(900)
def test_lds_kernels_read_only_what_they_wrote():
    sys.path.insert(0, ROOT)
    from paper_2306_05332_amd import build as B
    if not os.path.exists(B.POISON_LIB) or not os.path.exists(B.POISON_DIGEST):
        pytest.skip("LDS-poison library not built (build() makes it)")
    with open(B.POISON_DIGEST) as f:
        built = f.read().strip()
    assert built == B.sources_digest(), "LDS-poison library is older than the sources: rebuild"
    env = dict(os.environ, RKL_LIB=B.POISON_LIB)
    print("LDS-poison run:", " ".join(CASES), flush=True)
    r = subprocess.run([sys.executable, "-u", "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "gpu",
                        "--timeout", "120", "--timeout-method", "thread", *CASES],
                       env=env, capture_output=True, text=True, cwd=ROOT, timeout=900)
    out = r.stdout + r.stderr
    print(out[-2000:], flush=True)
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
