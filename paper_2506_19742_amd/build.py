"""Builds libnic.so (HIP for gfx950) in-tree with hipcc, and the memory-ceiling microbenchmark.

Every HIP source is compiled for gfx950 only, with packed-FP32 instructions disabled and hardware
FP32 atomics; the objects are linked into paper_2506_19742_amd/libnic.so next to this file.  The
microbenchmark (csrc/ubench.hip, a program of its own) becomes paper_2506_19742_amd/nic_ubench.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libnic.so")
UBENCH = os.path.join(HERE, "nic_ubench")
BUILD_DIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["nic_kernels.hip", "nic_capi.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-fno-gpu-rdc",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    "-I", INCLUDE, "-I", CSRC,
]


def _compile(src: str, extra) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
    if msg.strip():
        print(msg, file=sys.stderr)
    return obj


def _build_ubench() -> str:
    tmp = UBENCH + ".tmp"
    cmd = [HIPCC, *FLAGS, os.path.join(CSRC, "ubench.hip"), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
        raise RuntimeError(f"hipcc failed for ubench.hip:\n{msg}")
    os.replace(tmp, UBENCH)
    return UBENCH


def build(verbose: bool = False, extra=()) -> str:
    """Compiles every source for gfx950, links libnic.so and builds nic_ubench; returns the
    library's path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES) + 1)) as ex:
        ub = ex.submit(_build_ubench)
        objs = list(ex.map(lambda s: _compile(s, list(extra)), SOURCES))
        ub.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, "and", UBENCH)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
