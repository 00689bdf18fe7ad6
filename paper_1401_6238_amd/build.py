"""Builds libhankel.so (HIP kernels for gfx950 + the C ABI) in-tree.

    python -m paper_1401_6238_amd.build [-j JOBS]
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhankel.so")
ARCH = "gfx950"

HIP_SOURCES = ["hk_f32.hip", "hk_f64.hip", "hk_f32_odd.hip", "hk_f64_odd.hip", "hk_levels.hip", "hk_noalloc.hip", "hk_adjoint.hip"]
HOST_SOURCES = ["hk_plan.cpp", "hk_batch.cpp", "hk_api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DEVICE_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", f"--offload-arch={ARCH}"]


def _compile(src: str) -> str:
    obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    flags = DEVICE_FLAGS if src.endswith(".hip") else HOST_FLAGS
    cmd = [HIPCC] + flags + ["-I", CSRC, "-c", path, "-o", obj]
    subprocess.run(cmd, check=True)
    return obj


def build(jobs: int = 0, verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    srcs = HIP_SOURCES + HOST_SOURCES
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=0)
    args = ap.parse_args(argv)
    build(args.j, verbose=True)


if __name__ == "__main__":
    sys.exit(main())
