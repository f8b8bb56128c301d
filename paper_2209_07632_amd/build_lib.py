"""Compile librad.so (HIP for gfx950 + host C++) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "librad.so")

SOURCES = ["api.cpp", "build.cpp", "build_kernels.hip", "matvec_kernels.hip", "matmat_kernels.hip", "raycast.hip",
           "lowp_kernels.hip", "warmstart.hip", "timestep.hip",
           "group.cpp", "autotune.cpp", "serialize.cpp", "krylov.hip", "schedule.cpp"]

# geometry, entries and ray tests are evaluated without contraction so that
# their zero/non-zero and hit/miss decisions equal plain FP64 arithmetic
NO_CONTRACT = {"build.cpp", "build_kernels.hip", "raycast.hip"}

# packed FP32 instructions are disabled for every HIP translation unit
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-I" + INCLUDE, "-I" + CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [hipcc(), *COMMON, "-fopenmp", "-c", os.path.join(CSRC, src), "-o", obj]
    if src in NO_CONTRACT:
        cmd.insert(1, "-ffp-contract=off")
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    subprocess.run(cmd, check=True)
    return obj


def build(jobs: int = 4) -> str:
    """Compile every source for gfx950 and link ``librad.so`` next to this file."""
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-fopenmp", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
