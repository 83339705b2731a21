"""GPU parity of the nearest-pixel HD sampling variant (needs gfx950): the forward
integration with hd_sampling = nearest against the oracle's FP32 nearest variant, bit for
bit (state and per-voxel status codes), on the tiny scan (plain and fused passes, 8-bit and
float images) and on seeded slabs of the full kinect volume in the benchmark's launch
configuration; the adjoint refuses the variant."""
import dataclasses

import numpy as np
import pytest
import torch

import paper_1602_06645_amd as kf
from gpu_helpers import assert_bitwise, integrate_plain, say, to_host
from kf_synth import configs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def nearest(spec):
    return dataclasses.replace(spec, hd_sampling="nearest")


def oracle_state(oracle, spec, fr, gz=None, cz=None):
    st = oracle.State(spec, np.float32, gz=gz, cz=cz)
    oracle.integrate(spec, fr.numpy(), st)
    return st


@pytest.mark.parametrize("float_rgb", [False, True])
def test_nearest_tiny_plain_and_fused(oracle, float_rgb):
    spec, fr = configs.tiny()
    spec = nearest(spec)
    if float_rgb:
        fr = fr.as_float_rgb()
    say(f"nearest: tiny scan, float RGB {float_rgb}")
    want = oracle_state(oracle, spec, fr)
    bil = oracle_state(oracle, configs.tiny()[0], fr)
    assert not np.array_equal(want.r, bil.r)          # the variant changes the colours
    vol = kf.Volume(spec)
    integrate_plain(vol, fr.to(DEV))
    assert_bitwise(to_host(vol), want.arrays(), "nearest plain: ")
    vol2 = kf.Volume(spec)
    kf.integrate_batch([(vol2, kf.Scan.from_frames(fr.to(DEV)))], frames_per_pass=4)
    assert_bitwise(to_host(vol2), want.arrays(), "nearest fused: ")


def test_nearest_status_codes(oracle):
    spec, fr = configs.tiny(n_frames=4)
    spec = nearest(spec)
    say("nearest: per-frame status codes")
    vol = kf.Volume(spec)
    frd, frn = fr.to(DEV), fr.numpy()
    st = oracle.State(spec, np.float32)
    for f in range(fr.n):
        gs, cs = vol.status(frd.depth[f], frd.rgb[f], fr.K_d, fr.K_rgb, fr.T_rgb_from_d,
                            fr.T_world_from_cam[f], fr.trunc, fr.w_max)
        ogs, ocs = oracle.status(spec, frn, st, f)
        assert np.array_equal(gs.cpu().numpy(), ogs) and np.array_equal(cs.cpu().numpy(), ocs)
        vol.integrate(frd.depth[f], frd.rgb[f], fr.K_d, fr.K_rgb, fr.T_rgb_from_d,
                      fr.T_world_from_cam[f], fr.trunc, fr.w_max)
        oracle.integrate(spec, frn.select(f), st)


def test_nearest_kinect_slabs(oracle):
    spec, fr = configs.kinect(device=DEV, n_frames=8)
    spec = nearest(spec)
    say("nearest: kinect full size, K=8, graph replay")
    vol = kf.Volume(spec)
    kf.integrate_batch([(vol, kf.Scan.from_frames(fr))], frames_per_pass=8, use_graph=True)
    got = to_host(vol)
    rng = np.random.default_rng(78)
    updated = 0
    for _ in range(2):
        c0 = int(rng.integers(24, 150))          # the ground and the objects
        cz = (c0, c0 + 6)
        g0 = c0 // 2
        gz = (g0, g0 + 3)
        say(f"  oracle slabs geometry z{gz} colour z{cz}")
        st = oracle_state(oracle, spec, fr, gz, cz)
        n_g, n_c = spec.gdim[0] * spec.gdim[1], spec.cdim[0] * spec.cdim[1]
        for g, w, n, z in zip(got, st.arrays(), [n_g] * 2 + [n_c] * 4, [gz] * 2 + [cz] * 4):
            assert np.array_equal(g[z[0] * n:z[1] * n].view(np.uint32), w.view(np.uint32))
        updated += int((st.wc > 0).sum())
    assert updated > 1000


def test_nearest_adjoint_refused():
    spec, fr = configs.tiny(n_frames=2)
    fr = fr.as_float_rgb().to(DEV)
    scan = kf.Scan.from_frames(fr)
    g = torch.zeros((3, spec.n_colour), dtype=torch.float32, device=DEV)
    with pytest.raises(kf.api.L.KfError) as e:
        kf.integrate_backward(nearest(spec), scan, g)
    assert e.value.status == kf.api.L.KF_E_UNSUPPORTED
