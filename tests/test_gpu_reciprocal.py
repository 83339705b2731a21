"""The library's reciprocal (hardware reciprocal plus one Newton step, the IEEE division
outside the normal range up to 2^125) equals 1.0f / z bit for bit for every one of the
2^32 single-precision inputs (needs gfx950).  The projections of the integration, the
colour update and the adjoint rely on it for bit-exactness with the oracle."""
import ctypes as C
import os

import pytest

pytestmark = pytest.mark.gpu
LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gpu_check", "librecipcheck.so")


def test_reciprocal_matches_ieee_division_everywhere():
    import torch
    assert torch.cuda.is_available()
    if not os.path.exists(LIB):
        pytest.fail("tests/gpu_check/librecipcheck.so is not built (run __graft_entry__.build())")
    lib = C.CDLL(LIB)
    lib.kf_test_recip_mismatches.restype = C.c_longlong
    assert lib.kf_test_recip_mismatches() == 0
