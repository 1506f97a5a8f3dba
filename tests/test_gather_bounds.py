"""The D2Q5 gather offsets of the forward ADR step and its adjoint, compiled
for the host from the header the kernels include, stay inside each species'
block of five planes for every node and bounce-back mask (32- and 64-bit
offsets, FP32 and FP64 populations): a gather never reads past the lattice,
which on the 64-bit path (raw pointers, no buffer bounds) would read past
the workspace."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2109_04455_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_gather_offsets_stay_in_block(tmp_path):
    exe = str(tmp_path / "gather_bounds")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC,
                           os.path.join(HERE, "gather_bounds.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0 and out.stdout.startswith("ok")
