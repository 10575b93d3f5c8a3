"""The GPU kernels' threshold-index arithmetic (a 96-bit product split into
32-bit pieces, a clamp and one 64-bit shift), compiled for the host and checked
against the 128-bit definition; and the split kernel's equivalent decision (a
threshold on the product from the inverse of the table), checked against the
table lookup for every shift the instance compiler can choose."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_theta_index_matches_128bit_definition():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = os.path.join(HERE, "_build", "index_check")
    os.makedirs(os.path.dirname(exe), exist_ok=True)
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17",
                    os.path.join(HERE, "index_check.cpp"), "-o", exe], check=True, capture_output=True)
    res = subprocess.run([exe], capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    assert " 0 mismatches" in res.stdout
