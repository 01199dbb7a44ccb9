"""Builds libnmf.so (all HIP sources under csrc/) for gfx950 with hipcc.

Each translation unit is compiled to an object in _build/ (in parallel), then
linked into paper_1509_09313_amd/libnmf.so next to this file.  Always
recompiles: this is the "does it build" step.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build", "libnmf")
LIB_PATH = os.path.join(HERE, "libnmf.so")

ARCH = os.environ.get("NMF_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-I", INCLUDE, "-I", CSRC,
    # packed FP32 VALU ops stay off: the compiler forms them from plain float code and some of their
    # forms have given wrong results without an error on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


# additions for single sources
FILE_FLAGS = {
    # the network inference applies its ReLU to every MFMA result: accumulators held in VGPRs
    # spare one copy out of the accumulation registers per value
    "mlp.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def flags_for(src: str) -> list[str]:
    return HIP_FLAGS + FILE_FLAGS.get(os.path.basename(src), [])


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = ["hipcc", *flags_for(src), "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr}")
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = jobs or min(8, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB_PATH + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("linking libnmf.so failed:\n" + res.stderr)
    os.replace(tmp, LIB_PATH)
    if verbose:
        print("built", LIB_PATH, "from", len(srcs), "sources")
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
