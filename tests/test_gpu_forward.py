"""GPU parity of the forward integration against the FP32 oracle (needs gfx950).

Bar: geometry and colour weights and per-voxel status codes bit-exact; TSDF and colour
within 1e-5 absolute (the same single-precision operation sequence is implemented on
both sides, so they are expected to agree exactly).
"""
import numpy as np
import pytest
import torch

import paper_1602_06645_amd as kf
from gpu_helpers import (assert_bitwise, assert_matches_oracle, integrate_plain, say, to_host)
from helpers import camera_volume, frames, intrinsics, plane_depth, posed, ramp_image
from kf_synth import configs
from kf_synth.scenes import VolumeSpec, default_rgb_extrinsic

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def tiny():
    spec, fr = configs.tiny()
    return spec, fr


def _oracle_state(oracle, spec, fr, K=1):
    st = oracle.State(spec, np.float32)
    cnt = oracle.integrate(spec, fr.numpy(), st, frames_per_pass=K)
    return st.arrays(), cnt


def test_tiny_plain_matches_oracle(oracle, tiny):
    spec, fr = tiny
    say("tiny: 64^3/128^3, 10 frames, kf_integrate per frame")
    vol = kf.Volume(spec)
    integrate_plain(vol, fr.to(DEV))
    want, cnt = _oracle_state(oracle, spec, fr)
    got = to_host(vol)
    assert cnt[4] > 10000
    assert_matches_oracle(got, want)
    assert_bitwise(got, want, "tiny plain vs oracle: ")


def test_tiny_status_codes_bit_exact(oracle, tiny):
    spec, fr = tiny
    say("tiny: per-frame status codes")
    vol = kf.Volume(spec)
    frd = fr.to(DEV)
    st = oracle.State(spec, np.float32)
    frn = fr.numpy()
    seen = set()
    for f in range(fr.n):
        gs, cs = vol.status(frd.depth[f], frd.rgb[f], fr.K_d, fr.K_rgb, fr.T_rgb_from_d,
                            fr.T_world_from_cam[f], fr.trunc, fr.w_max)
        ogs, ocs = oracle.status(spec, frn, st, f)
        gs, cs = gs.cpu().numpy(), cs.cpu().numpy()
        assert np.array_equal(gs, ogs), f"frame {f}: geometry status differs at {np.flatnonzero(gs != ogs)[:5]}"
        assert np.array_equal(cs, ocs), f"frame {f}: colour status differs at {np.flatnonzero(cs != ocs)[:5]}"
        seen |= set(np.unique(cs).tolist())
        vol.integrate(frd.depth[f], frd.rgb[f], fr.K_d, fr.K_rgb, fr.T_rgb_from_d,
                      fr.T_world_from_cam[f], fr.trunc, fr.w_max)
        oracle.integrate(spec, frn.select(f), st)
    assert {0, 1, 2, 4, 6} <= seen


@pytest.mark.parametrize("K", [1, 2, 3, 10])
def test_tiny_batch_fused_equals_plain_and_oracle(oracle, tiny, K):
    spec, fr = tiny
    say(f"tiny: kf_integrate_batch K={K}")
    vol = kf.Volume(spec)
    kf.integrate_batch([(vol, kf.Scan.from_frames(fr.to(DEV)))], frames_per_pass=K)
    want, _ = _oracle_state(oracle, spec, fr)
    assert_bitwise(to_host(vol), want, f"batch K={K}: ")


@pytest.mark.parametrize("K", [1, 4, 10])
def test_counters_match_oracle(oracle, tiny, K):
    spec, fr = tiny
    say(f"tiny: counted batch K={K}")
    vol = kf.Volume(spec)
    cnt = kf.integrate_batch_counted([(vol, kf.Scan.from_frames(fr.to(DEV)))], frames_per_pass=K)
    want_state, want = _oracle_state(oracle, spec, fr, K)
    assert list(cnt[:6]) == list(want)
    assert 0 < cnt[7] and cnt[6] <= 64 ** 3 * fr.n and cnt[7] <= 128 ** 3 * fr.n
    assert_bitwise(to_host(vol), want_state, "counted: ")


@pytest.mark.parametrize("K", [40, 64, 1000])
def test_passes_wider_than_32_frames(oracle, K):
    """70 frames in passes of 40 (40 + 30) or 64 (64 + 6) frames, and K = 1000, which acts
    as 64: 64-bit frame masks with live frames above bit 31; state and counters (whose
    per-pass figures depend on the pass length) equal the oracle's."""
    spec, fr = configs.tiny(n_frames=70)
    say(f"tiny: 70 frames, counted batch K={K}")
    vol = kf.Volume(spec)
    cnt = kf.integrate_batch_counted([(vol, kf.Scan.from_frames(fr.to(DEV)))], frames_per_pass=K)
    want_state, want = _oracle_state(oracle, spec, fr, min(K, 64))
    assert list(cnt[:6]) == list(want)
    assert_bitwise(to_host(vol), want_state, f"K={K}: ")
    vol2 = kf.Volume(spec)
    kf.integrate_batch([(vol2, kf.Scan.from_frames(fr.to(DEV)))], frames_per_pass=K, use_graph=True)
    assert_bitwise(to_host(vol2), want_state, f"K={K} graph: ")


def test_camera_inside_the_volume(oracle):
    """The camera sits inside the volume, so voxel columns cross its plane (Z <= 0 at one end,
    > 0 at the other): those columns take the per-voxel reciprocal with its range test, the
    others the column-checked Newton reciprocal; both bit-exact with the oracle, plain and
    fused."""
    Kd = intrinsics(131.25, 79.5, 59.5)
    spec = camera_volume(g=32, ratio=2, z0=-0.25, size=1.0)
    poses = np.stack([posed((4.0 * f, -3.0 * f), (0.01 * f, -0.005 * f, 0.02 * f)) for f in range(5)])
    fr = frames(np.full((5, 120, 160), 0.6), ramp_image(320, 240), Kd,
                intrinsics(262.5, 159.5, 119.5), default_rgb_extrinsic(), poses, 0.03)
    say("camera inside the volume: columns crossing the camera plane")
    want, cnt = _oracle_state(oracle, spec, fr)
    assert cnt[0] > 1000 and cnt[4] > 1000
    vol = kf.Volume(spec)
    integrate_plain(vol, fr.to(DEV))
    assert_bitwise(to_host(vol), want, "plain: ")
    vol2 = kf.Volume(spec)
    kf.integrate_batch([(vol2, kf.Scan.from_frames(fr.to(DEV)))], frames_per_pass=5)
    assert_bitwise(to_host(vol2), want, "fused: ")


def test_ragged_volume_and_anisotropic_cameras(oracle):
    """Volume dimensions that are not multiples of the 64 x 4 x 8 brick in any axis,
    unequal focal lengths, float images."""
    spec, fr = configs.tiny(n_frames=4)
    spec = VolumeSpec((37, 29, 21), (70, 61, 45), (-0.5, -0.45, -0.5), (1.0, 0.9, 1.0))
    fr.K_d = np.array([[140.0, 0.0, 83.25], [0.0, 124.0, 57.75], [0.0, 0.0, 1.0]])
    fr.K_rgb = np.array([[281.0, 0.0, 150.5], [0.0, 246.5, 124.0], [0.0, 0.0, 1.0]])
    fr = fr.as_float_rgb()
    say("ragged 37x29x21 / 70x61x45, float RGB")
    vol = kf.Volume(spec)
    integrate_plain(vol, fr.to(DEV))
    want, cnt = _oracle_state(oracle, spec, fr)
    assert cnt[4] > 1000
    assert_bitwise(to_host(vol), want, "ragged: ")
    vol2 = kf.Volume(spec)
    kf.integrate_batch([(vol2, kf.Scan.from_frames(fr.to(DEV)))], frames_per_pass=3)
    assert_bitwise(to_host(vol2), want, "ragged batch: ")


def test_rgb8_and_float_agree_bitwise(tiny):
    spec, fr = tiny
    say("tiny: RGB8 vs float32 images")
    a, b = kf.Volume(spec), kf.Volume(spec)
    integrate_plain(a, fr.to(DEV))
    integrate_plain(b, fr.as_float_rgb().to(DEV))
    assert_bitwise(to_host(a), to_host(b), "rgb8 vs f32: ")


def test_degenerate_inputs(oracle):
    """All-hole depth, NaN/inf/negative depth, a 1x1 depth map, a 2x2 HD image, a single
    voxel volume and a camera looking away: nothing faults, results match the oracle."""
    K = intrinsics(131.25, 79.5, 59.5)
    K2 = intrinsics(1.0, 0.5, 0.5)
    spec = camera_volume(g=9, ratio=3)
    D = np.full((120, 160), 0.8, np.float32)
    D[:, :50] = 0.0
    D[:, 50:60] = np.nan
    D[:, 60:70] = -1.0
    D[:, 70:80] = np.inf
    away = np.diag([1.0, -1.0, -1.0, 1.0])
    cases = {
        "holes": frames(D, np.full((240, 320, 3), 9, np.uint8), K, intrinsics(262.5, 159.5, 119.5), np.eye(4), np.eye(4), 0.03),
        "zero-depth": frames(np.zeros((120, 160)), np.full((240, 320, 3), 9, np.uint8), K, intrinsics(262.5, 159.5, 119.5), np.eye(4), np.eye(4), 0.03),
        "tiny-images": frames(np.full((1, 1), 0.8), np.full((2, 2, 3), 200, np.uint8), intrinsics(1.0, 0.0, 0.0), K2, np.eye(4), np.eye(4), 0.03),
        "looking-away": frames(np.full((120, 160), 0.8), np.full((240, 320, 3), 9, np.uint8), K, intrinsics(262.5, 159.5, 119.5), np.eye(4), away, 0.03),
    }
    for name, fr in cases.items():
        for sp in (spec, VolumeSpec((1, 1, 1), (1, 1, 1), (-0.01, -0.01, 0.79), (0.02, 0.02, 0.02))):
            say(f"degenerate: {name} {sp.gdim}")
            vol = kf.Volume(sp)
            integrate_plain(vol, fr.to(DEV))
            st = oracle.State(sp, np.float32)
            oracle.integrate(sp, fr, st)
            assert_bitwise(to_host(vol), st.arrays(), f"{name}: ")


def test_empty_batch_and_zero_frames(tiny):
    spec, fr = tiny
    say("empty batch / zero-frame scan")
    kf.integrate_batch([])
    vol = kf.Volume(spec)
    scan = kf.Scan.from_frames(fr.select(slice(0, 0)).to(DEV))
    kf.integrate_batch([(vol, scan)], frames_per_pass=4)
    torch.cuda.synchronize()
    assert all(float(t.abs().sum()) == 0.0 for t in vol.arrays())


def test_reset_zeroes_volume(tiny):
    spec, fr = tiny
    say("reset")
    vol = kf.Volume(spec)
    integrate_plain(vol, fr.select(slice(0, 2)).to(DEV))
    vol.reset()
    torch.cuda.synchronize()
    assert all(float(t.abs().sum()) == 0.0 for t in vol.arrays())


def test_resume_mid_sequence_is_bit_identical(tiny):
    """The volume is the whole state: copying it out and back in between two halves of
    the scan gives the same result as one uninterrupted run."""
    spec, fr = tiny
    frd = fr.to(DEV)
    say("resume mid-sequence")
    a = kf.Volume(spec)
    integrate_plain(a, frd)
    b = kf.Volume(spec)
    integrate_plain(b, frd.select(slice(0, 5)))
    saved = [t.cpu().clone() for t in b.arrays()]
    c = kf.Volume(spec)
    for t, s in zip(c.arrays(), saved):
        t.copy_(s.to(DEV))
    integrate_plain(c, frd.select(slice(5, 10)))
    assert_bitwise(to_host(a), to_host(c), "resume: ")


def test_plane_closed_form_on_gpu():
    """Fronto-parallel plane: F = min(1, (d0 - Z)/trunc) within 1e-5, weights = frame count."""
    K = intrinsics(131.25, 79.5, 59.5)
    spec = camera_volume(g=32, ratio=2)
    d0, trunc, n = np.float32(0.8), 0.0375, 5
    fr = frames(np.full((n, 120, 160), d0), np.full((240, 320, 3), 60, np.uint8), K,
                intrinsics(262.5, 159.5, 119.5), np.eye(4), np.eye(4), trunc)
    say("plane closed form")
    vol = kf.Volume(spec)
    kf.integrate_batch([(vol, kf.Scan.from_frames(fr.to(DEV)))], frames_per_pass=n)
    tsdf, wg, r, g, b, wc = to_host(vol)
    import brute
    pc = brute.voxel_centres(spec.gdim, spec.origin, spec.extent)
    sdf = float(d0) - pc[:, 2]
    band = (sdf >= -trunc) & (np.abs(sdf + trunc) > 1e-5)
    x = 131.25 * pc[:, 0] / pc[:, 2] + 79.5
    y = 131.25 * pc[:, 1] / pc[:, 2] + 59.5
    inside = (np.rint(x) >= 0) & (np.rint(x) <= 159) & (np.rint(y) >= 0) & (np.rint(y) <= 119)
    sel = band & inside
    np.testing.assert_array_equal(wg[sel], n)
    np.testing.assert_allclose(tsdf[sel], np.minimum(1.0, sdf / trunc)[sel], atol=1e-5)
    seen = wc > 0
    assert seen.sum() > 1000
    np.testing.assert_array_equal(r[seen], np.float32(60) * np.float32(1 / 255.0))
