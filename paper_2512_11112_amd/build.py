"""Build libspdz.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2512_11112_amd.build

Every .hip file under csrc/ is compiled to an object in _build/ (in
parallel), then linked into paper_2512_11112_amd/libspdz.so.  The calibration
program calib/mfma_rate.hip (the int8 MFMA rate this GPU sustains, reported
beside the GEMM's measurements) is a measurement probe, not part of the
library: the matrix-triple benchmark compiles it on first use (build_calib()),
and build() leaves it alone.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libspdz.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall",
    "-Wno-unused-function", "-Wno-unused-variable",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)), 16)
    with cf.ThreadPoolExecutor(max_workers=max(jobs, 1)) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} from {len(srcs)} sources", file=sys.stderr)
    return OUT


CALIB = os.path.join(PKG, "calib", "mfma_rate")


def build_calib():
    """Compile the MFMA-rate probe; its path, or None if hipcc failed."""
    r = subprocess.run([HIPCC, *CFLAGS, os.path.join(PKG, "calib", "mfma_rate.hip"), "-o", CALIB],
                       capture_output=True, text=True)
    return CALIB if r.returncode == 0 else None


if __name__ == "__main__":
    build()
