"""Stochastic rounding of stored populations, checked on the host.

The rounding helpers of the HIP library (paper_2112_13930_amd/csrc/lks_sr.hpp)
are host-compilable; tests/native/sr_check.cpp sweeps the random word over a
stratified grid for values across many binades (binary16 subnormals, binade
edges, exact values, both signs) and requires neighbours only, exact values
unchanged, and the exact rounding-up probability to within the sweep's
resolution (2^-13 for binary16, which takes 13 random bits; in binary16's
subnormal range the count of round-ups over all 2^13 words is checked
exactly).  The device form of the binary16 rounding (the hardware's
stochastic conversion) is checked against the same definition on the GPU
(tests/test_gpu_rounding.py).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = os.environ.get("LKS_HOST_CLANG", "/opt/rocm/llvm/bin/clang++")


@pytest.mark.skipif(not (os.path.exists(CLANG) or shutil.which(CLANG)), reason="no clang++ for _Float16")
def test_stochastic_rounding_is_exact(tmp_path):
    exe = str(tmp_path / "sr_check")
    subprocess.run([CLANG, "-std=c++17", "-O2", "-I", os.path.join(ROOT, "paper_2112_13930_amd", "csrc"),
                    "-o", exe, os.path.join(ROOT, "tests", "native", "sr_check.cpp")], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("OK")
