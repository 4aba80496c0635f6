"""Compile the HIP library ``libsph.so`` for gfx950 in-tree with hipcc."""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsph.so")
SOURCES = ["api.hip", "encode.hip", "build_cells.hip", "interact.hip", "step.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CC = os.environ.get("CC", "gcc")
ROCM_INC, ROCM_LIB = "/opt/rocm/include", "/opt/rocm/lib"
RUNNER = os.path.join(HERE, "sph_run")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-fvisibility=hidden",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, "csrc", s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I" + os.path.join(ROOT, "include"), "-o", tmp, *srcs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    build_runner()
    return LIB


def build_runner() -> str:
    """Compile ``sph_run``, a plain C program that drives the library through
    its C ABI only (host code: the C compiler, the HIP runtime and libsph.so)."""
    tmp = RUNNER + ".tmp"
    cmd = [CC, "-O2", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC,
           "-I" + os.path.join(ROOT, "include"), os.path.join(HERE, "csrc", "sph_run.c"),
           "-o", tmp, "-L" + HERE, "-lsph", "-L" + ROCM_LIB, "-lamdhip64",
           "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + ROCM_LIB]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("building sph_run failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, RUNNER)
    return RUNNER


if __name__ == "__main__":
    print(build(verbose=True))
