"""GPU parity of the ray caster (needs gfx950): kf_raycast against the oracle's FP32 ray
cast, bit for bit, on volumes the oracle integrated (uploaded to the GPU) and on analytic
volumes; whole images at small sizes (including ragged 16 x 16 tiles), sampled pixels of
640 x 480 images of the full-size kinect volume."""
import numpy as np
import pytest
import torch

import paper_1602_06645_amd as kf
from gpu_helpers import say
from kf_synth import configs
from kf_synth.scenes import VolumeSpec

pytestmark = pytest.mark.gpu
DEV = "cuda"
OUTS = (("depth", "depth"), ("vertex", "vertex"), ("normal", "normal"), ("rgb", "colour"))


def upload(spec, st):
    vol = kf.Volume(spec)
    for name, a in zip(("tsdf", "w_geom", "r", "g", "b", "w_col"), st.arrays()):
        getattr(vol, name).copy_(torch.as_tensor(np.ascontiguousarray(a, np.float32)))
    return vol


def assert_same(got, want, pixels=None):
    for gname, oname in OUTS:
        g = got[gname].cpu().numpy()
        if pixels is not None:
            g = g.reshape((-1,) + g.shape[2:])[pixels]
        w = want[oname]
        bad = g.view(np.uint32) != w.astype(np.float32).view(np.uint32)
        assert not bad.any(), f"{gname}: {bad.sum()} values differ (first at {np.argwhere(bad)[0]})"


def K_for(width):
    f = 525.0 * width / 640
    return np.array([[f, 0, (width - 1) / 2], [0, f, (width * 3 / 4 - 1) / 2], [0, 0, 1.0]])


@pytest.fixture(scope="module")
def tiny(oracle):
    spec, fr = configs.tiny(n_frames=6)
    fr = fr.numpy()
    st = oracle.State(spec, np.float32)
    oracle.integrate(spec, fr, st)
    return spec, fr, st


@pytest.mark.parametrize("width,height", [(160, 120), (157, 113)])
def test_raycast_tiny_whole_image(oracle, tiny, width, height):
    spec, fr, st = tiny
    say(f"raycast: tiny volume, {width}x{height}")
    vol = upload(spec, st)
    K = K_for(width)
    novel = fr.T_world_from_cam[1].copy()
    novel[:3, 3] += np.array([0.05, -0.04, 0.03])
    for T in (fr.T_world_from_cam[3], novel):
        got = vol.raycast(K, T, width, height, 0.011)
        torch.cuda.synchronize()
        want = oracle.raycast(spec, st, K, T, width, height, 0.011)
        assert np.count_nonzero(want["depth"]) > 0.05 * width * height
        assert_same(got, want)


def test_raycast_outputs_optional_and_misses(oracle, tiny):
    spec, fr, st = tiny
    say("raycast: optional outputs, misses")
    vol = upload(spec, st)
    K = K_for(160)
    T = fr.T_world_from_cam[0]
    full = vol.raycast(K, T, 160, 120, 0.011)
    only = vol.raycast(K, T, 160, 120, 0.011, vertex=False, normal=False, rgb=False)
    assert set(only) == {"depth"}
    torch.cuda.synchronize()
    assert torch.equal(full["depth"], only["depth"])
    away = T @ np.diag([-1.0, 1.0, -1.0, 1.0])            # turned around
    got = vol.raycast(K, away, 160, 120, 0.011)
    torch.cuda.synchronize()
    assert_same(got, oracle.raycast(spec, st, K, away, 160, 120, 0.011))
    assert float(got["depth"].abs().sum()) == 0.0
    empty = kf.Volume(spec)
    got = empty.raycast(K, T, 160, 120, 0.011)
    torch.cuda.synchronize()
    assert float(got["depth"].abs().sum()) == 0.0


def test_raycast_analytic_sphere(oracle):
    say("raycast: analytic sphere, anisotropic volume")
    from test_raycast_pins import analytic_state, affine_colour
    spec = VolumeSpec((72, 64, 80), (144, 128, 160), (-0.5, -0.45, -0.55), (1.0, 0.9, 1.1))
    c, R, trunc = np.array([0.02, -0.01, 0.08]), 0.27, 0.05
    st = analytic_state(oracle, spec, lambda p: (np.linalg.norm(p - c, axis=1) - R) / trunc,
                        affine_colour)
    vol = upload(spec, st)
    K = np.array([[140.0, 0, 82.5], [0, 121.0, 57.25], [0, 0, 1.0]])
    T = np.eye(4)
    T[:3, 3] = (0.0, 0.0, -0.85)
    got = vol.raycast(K, T, 168, 124, 0.015)
    torch.cuda.synchronize()
    want = oracle.raycast(spec, st, K, T, 168, 124, 0.015)
    assert np.count_nonzero(want["depth"]) > 3000
    assert_same(got, want)


def test_raycast_full_size_sampled(oracle):
    """kinect volume (256^3 / 512^3) integrated by the oracle from 12 frames; 640 x 480
    images from a scan pose and a novel pose; 3000 sampled pixels compared bit for bit."""
    say("raycast: full-size volume, 640x480, sampled pixels")
    spec, fr = configs.kinect(device=DEV, n_frames=12)
    fr = fr.numpy()
    st = oracle.State(spec, np.float32)
    oracle.integrate(spec, fr, st)
    vol = upload(spec, st)
    K = fr.K_d
    rng = np.random.default_rng(12)
    novel = fr.T_world_from_cam[5].copy()
    novel[:3, 3] += np.array([0.03, 0.02, -0.04])
    for T in (fr.T_world_from_cam[7], novel):
        got = vol.raycast(K, T, 640, 480, 0.0094)
        torch.cuda.synchronize()
        pix = rng.choice(640 * 480, 4000, replace=False)
        want = oracle.raycast(spec, st, K, T, 640, 480, 0.0094, pixels=pix)
        assert np.count_nonzero(want["depth"]) > 800
        assert_same(got, want, pixels=pix)
