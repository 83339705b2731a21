"""Build the GPU test helpers of tests/gpu_check (compiled like the library, for gfx950)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "librecipcheck.so")


def build() -> str:
    from paper_1602_06645_amd import build as kbuild
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *kbuild.FLAGS, "-I" + kbuild.CSRC, "-o", LIB + ".tmp",
           os.path.join(HERE, "recip_check.hip")]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB
