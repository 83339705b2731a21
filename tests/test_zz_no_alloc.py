"""The allocation-free entry point kf_integrate_batch_noalloc (workspace in the library's
fixed device array) against kf_integrate_batch, bit for bit, on two calls in a row: a
Kinect-sized volume (256^3 / 512^3, 24 frames of 640x480 depth + 1920x1080 RGB8) beside
the tiny scan in one batch, then the tiny scan alone (a smaller input that finds the
array holding the first call's tables, lists and maps)."""
import pytest
import torch

import paper_1602_06645_amd as kf
from gpu_helpers import STATE_NAMES, say
from kf_synth import configs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _equal(a: kf.Volume, b: kf.Volume, where: str) -> None:
    torch.cuda.synchronize()
    for name, x, y in zip(STATE_NAMES, a.arrays(), b.arrays()):
        assert torch.equal(x.view(torch.int32), y.view(torch.int32)), f"{where}: {name} differs"


def test_noalloc_equals_batch_twice():
    say("no-alloc: generating the kinect volume's first 24 frames and the tiny scan")
    kspec, kfr = configs.kinect(device=DEV, n_frames=24)
    tspec, tfr = configs.tiny(device=DEV)
    kscan, tscan = kf.Scan.from_frames(kfr), kf.Scan.from_frames(tfr)

    say("no-alloc: call 1, kinect volume + tiny scan, 8 frames per pass")
    got = [kf.Volume(kspec), kf.Volume(tspec)]
    want = [kf.Volume(kspec), kf.Volume(tspec)]
    kf.integrate_batch_noalloc([(got[0], kscan), (got[1], tscan)], frames_per_pass=8)
    kf.integrate_batch([(want[0], kscan), (want[1], tscan)], frames_per_pass=8)
    _equal(got[0], want[0], "call 1 kinect volume")
    _equal(got[1], want[1], "call 1 tiny volume")
    assert float(want[0].w_col.count_nonzero()) > 1e6

    say("no-alloc: call 2, the tiny scan alone, 4 frames per pass")
    got2, want2 = kf.Volume(tspec), kf.Volume(tspec)
    kf.integrate_batch_noalloc([(got2, tscan)], frames_per_pass=4)
    kf.integrate_batch([(want2, tscan)], frames_per_pass=4)
    _equal(got2, want2, "call 2 tiny volume")
    assert float(want2.w_col.count_nonzero()) > 1e4
