"""Build the CPU emulation of libkfvol: the library's HIP sources compiled for the host
with clang against emu_shim.h, with AddressSanitizer and UBSan (a checking tool; the
product is only ever built for gfx950)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "..", "paper_1602_06645_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"


def asan_runtime() -> str:
    return subprocess.check_output([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                                   text=True).strip()


def build(out_dir: str) -> str:
    out = os.path.join(out_dir, "libkfvol_emu.so")
    cmd = [CLANG, "-std=c++20", "-O1", "-g", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           # fibers switch stacks: ASan's fake stacks for use-after-return make every
           # switch very slow, and heap and global buffers are what this build checks
           "-fsanitize-address-use-after-return=never",
           "-fno-omit-frame-pointer", "-I" + os.path.join(HERE, "include"), "-I" + CSRC,
           "-x", "c++", os.path.join(HERE, "emu.cpp"), "-o", out, "-lpthread"]
    subprocess.check_call(cmd)
    return out
