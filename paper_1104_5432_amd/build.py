"""Build libsu2.so (the HIP library behind include/su2.h) for gfx950, in-tree.

hipcc compiles every source as HIP for gfx950 only.  Packed-FP32 instruction
selection is switched off (-packed-fp32-ops): the kernels are written with
scalar float arithmetic and must not be lowered to v_pk_*_f32.  Floating-point
contraction is limited to single expressions (-ffp-contract=on).
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsu2.so")
SOURCES = ["su2_kernels.hip", "su2_staged.hip", "su2_observables.hip", "su2_learned.hip", "su2_api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-x", "hip", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # multiply-adds are fused only within one source expression, so every
    # kernel that forms a quantity with the same expressions rounds it the
    # same way (the staged and global-memory update kernels agree bitwise)
    "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-I" + INCLUDE, "-I" + CSRC,
]


# Per-source additions.  The staged kernels loop over the slices of a slab,
# and machine-level loop-invariant code motion hoists the sampler's and the
# index arithmetic's constants out of that loop into registers: FP64 staged
# kernels spill (28-288 bytes per lane) and the staged overrelaxation class
# at 64^4 FP64 takes 764 us instead of 525 us without the hoisting (FP32
# unchanged, 224 against 223 us).  The other kernels keep it: without it the
# global-memory FP64 heat bath, whose retry loop it serves, slows from 476
# to 546 us.
EXTRA = {"su2_staged.hip": ["-mllvm", "-disable-machine-licm"]}


def _deps():
    files = [os.path.join(CSRC, f) for f in os.listdir(CSRC)]
    files.append(os.path.join(INCLUDE, "su2.h"))
    return files


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compile and link libsu2.so; return its path."""
    os.makedirs(BUILD, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        cmd = [HIPCC] + FLAGS + EXTRA.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    bad = [p.wait() for p in procs]
    if any(bad):
        raise RuntimeError("hipcc failed building libsu2.so")
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in _deps())


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
