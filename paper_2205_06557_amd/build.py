"""Builds libodust.so (HIP kernels for gfx950 behind the C-ABI of include/odust.h).

Run as ``python -m paper_2205_06557_amd.build`` or through
``__graft_entry__.build()``.  The library is built in-tree next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "odust.hip")
LIB = os.path.join(HERE, "libodust.so")
DEPS = [os.path.join(HERE, "csrc", f) for f in ("odust.hip", "kernels.hpp", "device_common.hpp", "batch.hpp", "batch_api.inc", "mlp.hpp", "mlp_api.inc", "cutoff.hpp", "pairsym.hpp", "worksplit.hpp", "symitems.hpp")] + [
    os.path.join(ROOT, "include", "odust.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 (v_pk_*_f32) is kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def needs_build() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    build_c_example(verbose)
    return LIB


C_EXAMPLE_SRC = os.path.join(ROOT, "tests", "c_abi_example.c")
C_EXAMPLE = os.path.join(ROOT, "tests", "c_abi_example")


def c_example_command(out: str = C_EXAMPLE) -> list:
    """gcc line of the C program that uses the library through odust.h only."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return ["gcc", "-std=c11", "-O2", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), C_EXAMPLE_SRC,
            "-o", out, "-L", HERE, "-lodust", "-Wl,-rpath,$ORIGIN/../paper_2205_06557_amd", "-L", os.path.join(rocm, "lib"),
            "-Wl,-rpath-link," + os.path.join(rocm, "lib"), "-lm"]


def build_c_example(verbose: bool = False) -> str:
    if not os.path.exists(C_EXAMPLE_SRC):
        return ""
    cmd = c_example_command()
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return C_EXAMPLE


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
