"""The transform kernels' radix butterflies (csrc/fft.hpp), compiled for the host against a
small stand-in for the HIP header, checked on the CPU against the DFT in double precision:
radix 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, forward and inverse, with and without zero-pruned inputs;
and the LDS layouts of the transform plans."""
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


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_lds_layouts_fit_their_regions(tmp_path):
    """Every exchange of every plan stores a transform's entries at distinct slots inside the
    region its row or column kernel reserves, the column tile's staged rows fit, and two
    1024-point column or row blocks fit one CU's 160 KB of LDS (host build of fft.hpp)."""
    exe = tmp_path / "lds_layout"
    cmd = ["g++", "-O2", "-std=c++17", "-I", os.path.join(HERE, "host_fft"),
           "-I", CSRC, os.path.join(HERE, "host_fft", "lds_layout.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    run = subprocess.run([str(exe)], capture_output=True, text=True)
    assert run.returncode == 0 and run.stdout.strip() == "ok", run.stdout
