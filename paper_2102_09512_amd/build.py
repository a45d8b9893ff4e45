"""Builds liblbm.so (the HIP library behind include/lbm.h) for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
# the same library with the step kernel's LDS filled with NaN before use (debug)
POISON_LIB = os.path.join(HERE, "liblbm_poison.so")
SOURCES = ["lbm_api.hip", "lbm_kernels.hip", "lbm_nn.hip"]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are not generated (they are not trusted on this hardware)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = False) -> str:
    """Builds liblbm.so and its debug twin liblbm_poison.so (the step kernel
    with LBM_POISON_LDS); returns the path of liblbm.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = {}
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        _run([hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs[src] = obj
    poison_obj = os.path.join(CSRC, "lbm_kernels_poison.o")
    _run([hipcc, *HIPCC_FLAGS, "-DLBM_POISON_LDS=1", "-c", os.path.join(CSRC, "lbm_kernels.hip"), "-o", poison_obj],
         verbose)
    for lib, kernels in ((LIB, objs["lbm_kernels.hip"]), (POISON_LIB, poison_obj)):
        tmp = lib + ".tmp"
        _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, objs["lbm_api.hip"], kernels,
              objs["lbm_nn.hip"]], verbose)
        os.replace(tmp, lib)
    for o in [*objs.values(), poison_obj]:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
