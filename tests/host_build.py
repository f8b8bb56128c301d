"""Compiles a host-only program from tests/host/*.cpp that includes one of
librad's translation units (no device code runs), for CPU tests of host logic."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2209_07632_amd")


def compile_harness(name: str, outdir) -> str:
    hipcc = next((c for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")) if c and os.path.exists(c)), None)
    if hipcc is None:
        pytest.skip("hipcc not available")
    if not os.path.exists(os.path.join(PKG, "librad.so")):
        pytest.fail("librad.so is missing: build it first")
    exe = os.path.join(str(outdir), name)
    cmd = [hipcc, "-O1", "-std=c++17", "-x", "hip", "--offload-host-only", "-fopenmp",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(PKG, "csrc"),
           "-Wno-unused-command-line-argument", os.path.join(ROOT, "tests", "host", name + ".cpp"),
           "-o", exe, "-L" + PKG, "-lrad", "-Wl,-rpath," + PKG]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe
