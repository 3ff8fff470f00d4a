"""Build libdrr.so (the HIP/gfx950 C-ABI library) in-tree with hipcc, and the
gather-rate calibration library calib/libgathercal.so used by the benchmark.

Usage: python -m paper_2208_12737_amd.build [-v]
"""

from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdrr.so")
CALIB_LIB = os.path.join(HERE, "calib", "libgathercal.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _hipcc(out: str, srcs, verbose: bool) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{err}")
    if verbose and err.strip():
        print(err)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    _hipcc(CALIB_LIB, [os.path.join(HERE, "calib", "gather_lines.hip")], verbose)
    return _hipcc(LIB, sources(), verbose)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
