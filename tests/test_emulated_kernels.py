"""The HIP kernels and host code of libkfvol compiled for the CPU (tests/emu: a HIP-subset
shim with one fiber per GPU thread, wave collectives and barriers switching between
them, bounds-checked buffer loads) and run under AddressSanitizer and UBSan.  Checks
without a GPU that the kernels' logic equals the oracle (bit for bit in the forward, to
the adjoint tolerance in the backward) and touches no memory outside its buffers: two
scans and an odd-sized volume (partial bricks and culling chunks) in one batch (RGB8 and
float images, 6 and 32 frames, 8 frames per pass), passes of more than 32 frames (40
frames at 36 per pass), every compiled brick shape on the odd-sized volume, the
allocation-free entry point on two batches in a row, the per-voxel outcome codes of every
frame of a scan, the ray cast of an integrated volume, the quadric-error decimation of its
marching-cubes mesh, and the adjoint over 6 and 32 frames (a live frame in bit 31 of a
brick's frame mask), with its image gradient added per HD tile from records, scattered
with atomics, and both (a record buffer that runs out)."""
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "emu")


@pytest.fixture(scope="module")
def emu_build():
    if not os.path.exists(os.path.join(EMU, "build.py")):
        pytest.skip("tests/emu is not present")
    sys.path.insert(0, EMU)
    import build
    if not os.path.exists(build.CLANG):
        pytest.skip("host clang of the ROCm toolchain not found")
    return build


@pytest.fixture(scope="module")
def emulated(emu_build, tmp_path_factory):
    return emu_build.build(str(tmp_path_factory.mktemp("emu")))


def test_emulated_kernels_match_oracle(emu_build, emulated):
    env = dict(os.environ, LD_PRELOAD=emu_build.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:detect_stack_use_after_return=0:"
                            "max_malloc_fill_size=1000000000:malloc_fill_byte=190",
               UBSAN_OPTIONS="halt_on_error=1", EMU_THREADS="4")
    r = subprocess.run([sys.executable, os.path.join(EMU, "run_emulated.py"), emulated],
                       env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-4000:]
    res = json.loads(r.stdout.split("JSON:", 1)[1])
    assert res["forward_mismatches"] == 0
    assert res["wide_pass_mismatches"] == 0
    assert res["noalloc_mismatches"] == 0
    assert res["shape_mismatches"] == 0
    assert res["status_mismatches"] == 0
    assert res["raycast_mismatches"] == 0
    assert res["texture_mismatches"] == 0
    assert res["nearest_mismatches"] == 0 and res["nearest_status_mismatches"] == 0
    assert res["mesh_mismatches"] == 0
    assert res["decimate_mismatches"] == 0
    for case in ("backward_6", "backward_32", "backward_odd", "backward_direct", "backward_overflow",
                 "backward_chunked", "backward_chunked_6"):
        assert res[case]["rgb"] <= 1.0 and res[case]["xi"] <= 1.0, res
    for case in ("backward_6", "backward_odd", "backward_direct", "backward_overflow",
                 "backward_chunked", "backward_chunked_6"):
        # with the depth-pose adjoint
        assert res[case]["pose"] <= 1.0, res
