"""The library's walk and neighbour-index arithmetic, checked on the host.

tests/native/index_check.cpp includes the kernels' own device header and
runs its index functions (walk order, checkerboard coordinates, both
neighbour-addressing policies, the XCD block renumbering) on the CPU against
plain coordinate arithmetic, for every walk mode and a range of shapes up to
the largest the API accepts (V just below 2^32).  An index error in the
kernels would be an out-of-bounds access on the GPU; this catches it
without one.  tests/native/barrier_check.cpp does the same for the
persistent sweep's grid-barrier counter arithmetic.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_index_arithmetic_on_host(tmp_path):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "index_check")
    subprocess.run([HIPCC, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17",
                    "-I" + os.path.join(ROOT, "include"),
                    "-I" + os.path.join(ROOT, "paper_1104_5432_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "index_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "PASSED" in r.stdout, r.stdout[-2000:]


def test_staged_index_arithmetic_on_host(tmp_path):
    # the LDS-staged overrelaxation: every staple link a slab reads from LDS
    # is the link its loads put there, for every plan the chooser can pick
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "staged_check")
    subprocess.run([HIPCC, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17",
                    "-I" + os.path.join(ROOT, "include"),
                    "-I" + os.path.join(ROOT, "paper_1104_5432_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "staged_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "PASSED" in r.stdout, r.stdout[-2000:]


def test_grid_barrier_arithmetic_on_host(tmp_path):
    # the persistent batched sweep's barrier counter: no block passes early,
    # every block passes after the last arrival, the word needs no reset
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "barrier_check")
    subprocess.run([HIPCC, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17",
                    "-I" + os.path.join(ROOT, "include"),
                    "-I" + os.path.join(ROOT, "paper_1104_5432_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "barrier_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "PASSED" in r.stdout, r.stdout[-2000:]
