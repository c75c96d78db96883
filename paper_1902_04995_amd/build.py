"""Builds the HIP library librgb.so in-tree for gfx950 with hipcc.

Flags: -ffp-contract=off keeps the solver's FMAs exactly where the source
writes them (the exact-sign determinants depend on it); packed FP32 ops are
disabled because some of their forms have given wrong results on this
hardware class.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librgb.so")
BUILD_DIR = os.path.join(os.path.dirname(HERE), "_build")
SOURCES = ["rgb_kernels.hip", "rgb_api.hip", "rgb_server.hip", "rgb_host.hip", "rgb_crowd.hip", "rgb_reduce.hip",
           "rgb_seidel3.hip", "rgb_seidelN.hip", "rgb_table.cpp"]
ARCH = os.environ.get("RGB_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = ["-std=c++20", "-O3", f"--offload-arch={ARCH}", "-fPIC", "-ffp-contract=off",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(os.path.dirname(HERE), "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, src + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source and link librgb.so (always rebuilds)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
