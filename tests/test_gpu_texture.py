"""GPU parity of the per-polygon texture maps (needs gfx950): kf_texture_generate against the
oracle's FP32 texels, bit for bit (float and 8-bit atlases), on colour volumes the oracle
integrated (uploaded to the GPU) and on analytic ones; small maps of ragged sizes (not
multiples of the 8 x 8 texel blocks), degenerate and out-of-volume triangles, and the full
kinect volume with its 8192-triangle mesh (about 20 M texels, every texel compared)."""
import numpy as np
import pytest
import torch

import paper_1602_06645_amd as kf
from gpu_helpers import say
from kf_synth import configs
from kf_synth.scenes import VolumeSpec

pytestmark = pytest.mark.gpu
DEV = "cuda"


def upload(spec, st):
    vol = kf.Volume(spec)
    for name, a in zip(("tsdf", "w_geom", "r", "g", "b", "w_col"), st.arrays()):
        getattr(vol, name).copy_(torch.as_tensor(np.ascontiguousarray(a, np.float32)))
    return vol


def run_both(oracle, spec, st, vol, tri, size_pixel, H, fill=(0.0, 0)):
    rects, W = kf.texture_layout(tri, size_pixel, H)
    orects, oW = oracle.texture_layout(tri, size_pixel, H)
    assert W == oW and np.array_equal(rects, orects)
    out = {"rgb": torch.full((H, W, 3), fill[0], dtype=torch.float32, device=DEV),
           "rgb8": torch.full((H, W, 3), fill[1], dtype=torch.uint8, device=DEV)}
    got = vol.texture(torch.as_tensor(tri, device=DEV), torch.as_tensor(rects, device=DEV),
                      W, H, out=out)
    torch.cuda.synchronize()
    want = np.full((H, W, 3), fill[0], np.float32)
    want8 = np.full((H, W, 3), fill[1], np.uint8)
    oracle.texture(spec, st, tri, rects, W, H, atlas=want, atlas8=want8)
    g, g8 = got["rgb"].cpu().numpy(), got["rgb8"].cpu().numpy()
    bad = g.view(np.uint32) != want.view(np.uint32)
    assert not bad.any(), f"{bad.sum()} float texels differ (first at {np.argwhere(bad)[0]})"
    bad8 = g8 != want8
    assert not bad8.any(), f"{bad8.sum()} byte texels differ (first at {np.argwhere(bad8)[0]})"
    return rects, W, want


@pytest.fixture(scope="module")
def tiny(oracle):
    spec, fr = configs.tiny(n_frames=6)
    fr = fr.numpy()
    st = oracle.State(spec, np.float32)
    oracle.integrate(spec, fr, st)
    return spec, st


def test_texture_tiny_scan(oracle, tiny):
    spec, st = tiny
    say("texture: tiny volume, surface + degenerate + outside triangles")
    vol = upload(spec, st)
    tri, size_pixel = configs.tiny_triangles()
    rng = np.random.default_rng(31)
    extra = (rng.uniform(-0.6, 0.6, (16, 1, 3)) + rng.uniform(-0.1, 0.1, (16, 3, 3)))
    extra[0, 1] = extra[0, 0]
    extra[1, 1:] = extra[1, 0]
    tri = np.ascontiguousarray(np.concatenate([tri, extra.astype(np.float32)]))
    _, _, want = run_both(oracle, spec, st, vol, tri, size_pixel, 128, fill=(-3.0, 9))
    assert np.count_nonzero(want[want != -3.0]) > 20000


@pytest.mark.parametrize("size_pixel", [0.0031, 0.0117])
def test_texture_analytic_ragged(oracle, size_pixel):
    """An anisotropic colour volume with a smooth colour field and random weights (some
    zero), random triangles of every size class: maps from 2 x 2 to well over 8 x 8 blocks,
    ragged on both axes."""
    say(f"texture: analytic anisotropic volume, size_pixel {size_pixel}")
    spec = VolumeSpec((40, 36, 44), (120, 108, 132), (-0.5, -0.45, -0.55), (1.0, 0.9, 1.1))
    rng = np.random.default_rng(32)
    st = oracle.State(spec, np.float32)
    s = np.asarray(spec.extent) / np.asarray(spec.cdim)
    ax = [spec.origin[k] + (np.arange(spec.cdim[k]) + 0.5) * s[k] for k in range(3)]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    for a, (f, ph) in zip((st.r, st.g, st.b), ((7.0, 0.1), (11.0, 0.7), (5.0, 1.9))):
        a[:] = (0.5 + 0.45 * np.sin(f * x + ph) * np.cos(f * y - ph * z)).ravel()
    st.wc[:] = np.where(rng.uniform(size=st.wc.size) < 0.02, 0.0,
                        rng.uniform(0.1, 5.0, st.wc.size)).astype(np.float32)
    vol = upload(spec, st)
    V1 = rng.uniform(-0.55, 0.55, (300, 1, 3))
    span = rng.choice([0.004, 0.03, 0.15], (300, 1, 1))
    tri = (V1 + rng.uniform(-1, 1, (300, 3, 3)) * span).astype(np.float32)
    tri[:, 0] = V1[:, 0]
    run_both(oracle, spec, st, vol, tri, size_pixel, 256, fill=(0.25, 3))


def test_texture_outputs_and_empty(oracle, tiny):
    spec, st = tiny
    say("texture: one output at a time, no triangles")
    vol = upload(spec, st)
    tri, size_pixel = configs.tiny_triangles(n_tri=40)
    rects, W = kf.texture_layout(tri, size_pixel, 128)
    t, r = torch.as_tensor(tri, device=DEV), torch.as_tensor(rects, device=DEV)
    both = vol.texture(t, r, W, 128)
    only_f = vol.texture(t, r, W, 128, rgb8=False)
    only_8 = vol.texture(t, r, W, 128, rgb=False)
    torch.cuda.synchronize()
    assert set(only_f) == {"rgb"} and set(only_8) == {"rgb8"}
    assert torch.equal(both["rgb"], only_f["rgb"]) and torch.equal(both["rgb8"], only_8["rgb8"])
    with pytest.raises(RuntimeError):
        vol.texture(t, r, W, 128, rgb=False, rgb8=False)
    empty = vol.texture(t[:0], r[:0], 4, 4)
    torch.cuda.synchronize()
    assert float(empty["rgb"].abs().sum()) == 0.0


def test_texture_full_size(oracle):
    """The kinect volume (256^3 / 512^3) integrated by the oracle from 12 frames and the
    8192-triangle kinect mesh in a 4096-row atlas: every texel compared."""
    say("texture: full-size volume, 8192 triangles, 4096-row atlas")
    spec, fr = configs.kinect(device=DEV, n_frames=12)
    fr = fr.numpy()
    st = oracle.State(spec, np.float32)
    oracle.integrate(spec, fr, st)
    vol = upload(spec, st)
    tri, size_pixel = configs.kinect_triangles(n_frames=12)
    rects, W, want = run_both(oracle, spec, st, vol, tri, size_pixel, 4096)
    assert (rects[:, 2].astype(np.int64) * rects[:, 3]).sum() > 15_000_000
    assert np.count_nonzero(want.any(-1)) > 15_000_000
