"""Pins of the oracle's nearest-pixel HD sampling variant (CPU only).

With nearest-pixel sampling the colour update takes the HD pixel whose centre is nearest
the projection of the voxel centre (Eq. 2-4 then rounding, ties to even) instead of the
bilinear sample.  Checked against an independent FP64 projection:
* an image whose pixels hold their own coordinates gives every observed voxel exactly the
  coordinates of the rounded projection (not the floor, not the bilinear value);
* the image border: a projection within half a pixel outside the last pixel centres is
  sampled (it rounds onto the border pixel), further out it is not; bilinear sampling
  needs both neighbours, so those bands are the only voxels where the two variants'
  masks differ, and the colour weights agree wherever both update;
* a constant image gives the constant exactly.
"""
import dataclasses

import numpy as np

import brute
from helpers import camera_volume, frames, intrinsics
from kf_synth.scenes import default_rgb_extrinsic

K160 = intrinsics(131.25, 79.5, 59.5)
K320 = intrinsics(262.5, 159.5, 119.5)


def nearest(vol):
    return dataclasses.replace(vol, hd_sampling="nearest")


def hd_projection(vol, T_rd, f=262.5):
    pw = brute.voxel_centres(vol.cdim, vol.origin, vol.extent)      # camera = world
    q = pw @ T_rd[:3, :3].T + T_rd[:3, 3]
    return f * q[:, 0] / q[:, 2] + 159.5, f * q[:, 1] / q[:, 2] + 119.5


def coordinate_image(W=320, H=240):
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float32), np.arange(W, dtype=np.float32),
                         indexing="ij")
    return np.stack([xx, yy, np.full_like(xx, 0.5)], -1)


def run(oracle, vol, fr):
    st = oracle.State(vol, np.float32)
    oracle.integrate(vol, fr, st)
    return st


def test_nearest_pixel_of_the_voxel_centre(oracle):
    T_rd = default_rgb_extrinsic()
    vol = camera_volume(g=16, ratio=3, z0=0.7, size=0.25)
    fr = frames(np.full((3, 120, 160), 0.8), coordinate_image(), K160, K320, T_rd, np.eye(4), 0.05)
    st = run(oracle, nearest(vol), fr)
    xh, yh = hd_projection(vol, T_rd)
    seen = st.wc > 0
    clear = (np.abs(xh - np.floor(xh) - 0.5) > 1e-3) & (np.abs(yh - np.floor(yh) - 0.5) > 1e-3)
    ok = seen & clear
    assert ok.sum() > 500
    np.testing.assert_array_equal(st.r[ok], np.rint(xh[ok]).astype(np.float32))
    np.testing.assert_array_equal(st.g[ok], np.rint(yh[ok]).astype(np.float32))
    np.testing.assert_array_equal(st.b[seen], np.float32(0.5))
    # the rounding is to nearest: many voxels lie in the upper half of their pixel
    assert (ok & (xh - np.floor(xh) > 0.5)).sum() > 100
    # bilinear sampling of the same image gives the projection itself
    stb = run(oracle, vol, fr)
    np.testing.assert_allclose(stb.r[ok], xh[ok], atol=2e-4)


def test_image_border_bands(oracle):
    # an HD camera with a narrower field of view than the depth camera: all four image
    # borders cross the observed surface
    T_rd = default_rgb_extrinsic()
    f_hd = 300.0
    vol = camera_volume(g=32, ratio=4, z0=0.3, size=1.2)
    fr = frames(np.full((2, 120, 160), 0.8), coordinate_image(), K160,
                intrinsics(f_hd, 159.5, 119.5), T_rd, np.eye(4), 0.05)
    stn = run(oracle, nearest(vol), fr)
    stb = run(oracle, vol, fr)
    xh, yh = hd_projection(vol, T_rd, f_hd)
    W, H = 320, 240
    ties = ((np.abs(xh - np.floor(xh) - 0.5) < 1e-3) | (np.abs(yh - np.floor(yh) - 0.5) < 1e-3) |
            (np.abs(xh - np.rint(xh)) < 1e-3) | (np.abs(yh - np.rint(yh)) < 1e-3))
    in_n = (xh > -0.5) & (xh < W - 0.5) & (yh > -0.5) & (yh < H - 0.5)
    in_b = (xh >= 0) & (xh < W - 1) & (yh >= 0) & (yh < H - 1)
    un, ub = stn.wc > 0, stb.wc > 0
    # every voxel updated by either variant passed the depth tests; among those, the HD
    # test alone separates them
    depth_ok = un | ub
    band = depth_ok & in_n & ~in_b & ~ties
    assert band.sum() > 20
    assert un[band].all() and not ub[band].any()
    outside = depth_ok & ~in_n & ~ties
    assert not un[outside].any()
    both = un & ub
    assert both.sum() > 1000
    np.testing.assert_array_equal(stn.wc[both], stb.wc[both])
    # the border pixel is what the band samples
    np.testing.assert_array_equal(stn.r[band], np.rint(xh[band]).astype(np.float32))
    np.testing.assert_array_equal(stn.g[band], np.rint(yh[band]).astype(np.float32))
    edge = (stn.r[band] == 0) | (stn.r[band] == W - 1) | (stn.g[band] == 0) | (stn.g[band] == H - 1)
    assert edge.all()
    x0, x1 = (stn.r[band] == 0).any(), (stn.r[band] == W - 1).any()
    y0, y1 = (stn.g[band] == 0).any(), (stn.g[band] == H - 1).any()
    assert (x0 or x1) and (y0 or y1) and (x1 or y1)     # both axes, and a far border


def test_constant_image_exact(oracle):
    vol = camera_volume(g=16, ratio=2, z0=0.7, size=0.25)
    img = np.empty((240, 320, 3), np.uint8)
    img[...] = np.array([200, 17, 99], np.uint8)
    fr = frames(np.full((2, 120, 160), 0.8), img, K160, K320, default_rgb_extrinsic(),
                np.eye(4), 0.05)
    st = run(oracle, nearest(vol), fr)
    seen = st.wc > 0
    assert seen.sum() > 500
    for arr, c in zip((st.r, st.g, st.b), (200, 17, 99)):
        np.testing.assert_array_equal(arr[seen], np.float32(c) * np.float32(1.0 / 255.0))
