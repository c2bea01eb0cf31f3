"""Host-side bounds check of the batch program (no GPU): every work item and
copy descriptor that setup and the tuner build stays inside the workspace
region it belongs to, for the full 64-problem workload and a mixed small
batch, under every launch-shape candidate of the tuner.  The check is built
from tests/batch_worklist_check.hip with hipcc (about a minute)."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from paper_2203_13382_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2203_13382_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    lib = os.path.join(PKG, "libslmgrit.so")
    if not os.path.exists(lib):
        pytest.skip("libslmgrit.so is not built")
    if not shutil.which(HIPCC):
        pytest.skip("hipcc not found")
    out = str(tmp_path_factory.mktemp("bwc") / "libbwc.so")
    # device code is compiled too (kernel registration needs it), unoptimised
    # since nothing here launches it
    cmd = [HIPCC, "--offload-arch=gfx950", "-O0", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           os.path.join(ROOT, "tests", "batch_worklist_check.hip"), "-o", out,
           "-L", PKG, "-lslmgrit", "-Wl,-rpath," + PKG]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    h = C.CDLL(out)
    h.check_batch.argtypes = [C.c_void_p, C.c_int, C.c_longlong]
    h.check_batch.restype = C.c_int
    return h


def _mixed():
    probs = []
    for i, (nx, nt, p, m) in enumerate([(64, 256, 1, 4), (200, 96, 5, 4), (1500, 64, 3, 2), (4096, 48, 3, 4),
                                        (8192, 32, 1, 4), (96, 17, 3, 4)]):
        pr = W.Problem(1, nx, nt, (0.85 + 0.3 * i) * 2 / nx, p, p, W.alpha_cfg12(0.3))
        probs.append((pr, W.Solver(m=[m], coarsest_max_points=2, gmres_rtol=1e-2)))
    return probs


@pytest.mark.slow
@pytest.mark.parametrize("which", ["full", "mixed_fp64"])
def test_batch_program_in_bounds(checker, which):
    from paper_2203_13382_amd import Batch
    if which == "full":
        probs, prec = W.batch_config()
    else:
        probs, prec = _mixed(), "fp64"
    b = Batch(probs, prec, device="cpu")
    assert checker.check_batch(b.h, 0, 0) == 0
    # a region 8 bytes short of what the first problem's items touch is caught
    assert checker.check_batch(b.h, 0, 8) > 0
