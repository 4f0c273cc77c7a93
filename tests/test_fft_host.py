"""The transform kernels' radix butterflies (csrc/fft.hpp), compiled for the host against a
small stand-in for the HIP header, checked on the CPU against the DFT in double precision:
radix 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, forward and inverse, with and without zero-pruned inputs."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2604_02624_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_radix_butterflies_match_the_dft(tmp_path):
    exe = tmp_path / "butterflies"
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I", os.path.join(HERE, "host_fft"),
           "-I", CSRC, os.path.join(HERE, "host_fft", "butterflies.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    worst = float(out.strip())
    # single precision butterflies of at most 20 points: a few ulp of the largest output
    assert worst < 5e-7, worst
