"""Build the dpx HIP library for gfx950 in-tree: paper_2604_02624_amd/libdpx.so.

    python -m paper_2604_02624_amd.build      (or __graft_entry__.build())
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libdpx.so")
BUILD = os.path.join(PKG, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          # no packed-FP32 instructions (v_pk_*_f32) anywhere in the device code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          # no implicit contraction: fused multiply-adds only where written (fmaf), so results
          # do not depend on how a kernel inlines the shared code
          "-ffp-contract=off",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# transform lengths with their own translation unit of pass kernels (dpx_pass.hip)
LENGTHS = [64, 96, 128, 192, 256, 384, 512, 1024, 1600]
# (source, object name, extra flags); the long-running pass units first
UNITS = ([("dpx_pass.hip", f"dpx_pass_{m}.o", [f"-DDPX_M={m}"]) for m in sorted(LENGTHS, reverse=True)]
         + [("dpx_kernels.hip", "dpx_kernels.o", []), ("dpx_api.cpp", "dpx_api.o", [])])


def _compile(unit):
    src, obj, extra = unit
    out = os.path.join(BUILD, obj)
    cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} {' '.join(extra)} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    workers = max(1, min(len(UNITS), int(os.environ.get("MAX_JOBS", "0")) or (os.cpu_count() or 4)))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, UNITS))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
