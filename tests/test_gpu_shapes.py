"""Brick shapes of the forward integration on the GPU (needs gfx950): every compiled shape
gives the oracle's volume bit for bit (the tiny scan, and an odd-sized volume with partial
bricks on every axis), the same accounting counters (the per-voxel ones do not depend on
the shape), and, on the Kinect-sized volume, the same volume as the default shapes, with
and without a recorded graph."""
import numpy as np
import pytest
import torch

import paper_1602_06645_amd as kf
from gpu_helpers import STATE_NAMES, assert_bitwise, say, to_host
from kf_synth import configs
from kf_synth.scenes import VolumeSpec

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _pairs():
    sh = kf.brick_shapes()
    n = max(len(sh["geometry"]), len(sh["colour"]))
    return [{"geometry": sh["geometry"][min(q, len(sh["geometry"]) - 1)],
             "colour": sh["colour"][min(q, len(sh["colour"]) - 1)]} for q in range(n)]


@pytest.fixture(scope="module")
def oracle_tiny(oracle):
    spec, fr = configs.tiny(n_frames=10)
    odd = VolumeSpec((45, 37, 29), (135, 111, 87), (-0.41, -0.37, -0.46), (0.9, 0.74, 0.58))
    out = []
    for sp in (spec, odd):
        st = oracle.State(sp, np.float32)
        oracle.integrate(sp, fr.numpy(), st)
        out.append((sp, st.arrays()))
    return fr, out


@pytest.mark.parametrize("q", range(5))
def test_every_shape_matches_oracle(oracle_tiny, q):
    pairs = _pairs()
    if q >= len(pairs):
        pytest.skip("fewer compiled shapes")
    bricks = pairs[q]
    fr, cases = oracle_tiny
    scan = kf.Scan.from_frames(fr.to(DEV))
    for sp, want in cases:
        say(f"shapes: {bricks} on {sp.gdim}")
        vol = kf.Volume(sp)
        cnt = kf.integrate_batch_counted([(vol, scan)], frames_per_pass=4, bricks=bricks)
        assert_bitwise(to_host(vol), want, f"bricks {bricks} {sp.gdim}: ")
        ref = kf.Volume(sp)
        ref_cnt = kf.integrate_batch_counted([(ref, scan)], frames_per_pass=4)
        assert list(cnt[:6]) == list(ref_cnt[:6])
        assert 0 < cnt[7] <= int(np.prod(sp.cdim)) * fr.n


def test_shapes_equal_on_kinect_volume():
    say("shapes: kinect volume, 24 frames, each shape pair against the defaults")
    spec, fr = configs.kinect(device=DEV, n_frames=24)
    scan = kf.Scan.from_frames(fr)
    ref = kf.Volume(spec)
    kf.integrate_batch([(ref, scan)], frames_per_pass=12)
    torch.cuda.synchronize()
    for bricks in _pairs()[1:]:
        for graph in (False, True):
            vol = kf.Volume(spec)
            kf.integrate_batch([(vol, scan)], frames_per_pass=12, use_graph=graph, bricks=bricks)
            torch.cuda.synchronize()
            for name, x, y in zip(STATE_NAMES, vol.arrays(), ref.arrays()):
                assert torch.equal(x.view(torch.int32), y.view(torch.int32)), \
                    f"bricks {bricks} graph={graph}: {name} differs"
            del vol
    assert float(ref.w_col.count_nonzero()) > 1e6
