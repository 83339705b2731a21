"""Build libkfvol.so (the HIP kernels and the C ABI of include/kf.h) for gfx950."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB_PATH = os.path.join(HERE, "libkfvol.so")
SOURCES = ["kf_integrate.hip", "kf_backward.hip", "kf_raycast.hip", "kf_texture.hip",
           "kf_mesh.hip", "kf_capi.hip", "kf_decimate.cpp"]

# IEEE single precision everywhere: no contraction into fma beyond the explicit fmaf
# calls, correctly rounded division and square root, no packed-FP32 instructions.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-ffp-contract=off", "-fno-fast-math", "-fhip-fp32-correctly-rounded-divide-sqrt",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # wave-wide atomics (queue tickets, list appends) are combined with a DPP prefix
         # sum rather than a loop over the active lanes
         "-mllvm", "-amdgpu-atomic-optimizer-strategy=DPP",
         "-Wall", "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libkfvol.so (always recompiles)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc, *FLAGS, "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
