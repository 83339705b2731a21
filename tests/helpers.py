"""Small analytic scans used by the closed-form pins and the parity tests."""
from __future__ import annotations

import numpy as np

from kf_synth.scenes import Frames, VolumeSpec, intrinsics, rigid, rot_x, rot_y


def frames(depth, rgb, K_d, K_rgb, T_rd, poses, trunc, w_max=64.0) -> Frames:
    depth = np.asarray(depth, np.float32)
    if depth.ndim == 2:
        depth = depth[None]
    n = depth.shape[0]
    poses = np.asarray(poses, float)
    if poses.ndim == 2:
        poses = np.repeat(poses[None], n, axis=0)
    rgb = np.asarray(rgb)
    if rgb.ndim == 3:
        rgb = np.repeat(rgb[None], n, axis=0)
    return Frames(depth, rgb, np.asarray(K_d, float), np.asarray(K_rgb, float),
                  np.asarray(T_rd, float), poses, float(trunc), float(w_max))


def plane_depth(K, W, H, normal, offset):
    """Depth (z) of the plane n . X = offset seen by a camera at the origin."""
    u = np.arange(W, dtype=float)
    v = np.arange(H, dtype=float)
    vv, uu = np.meshgrid(v, u, indexing="ij")
    r = np.stack([(uu - K[0, 2]) / K[0, 0], (vv - K[1, 2]) / K[1, 1], np.ones_like(uu)], -1)
    return offset / (r @ np.asarray(normal, float))


def camera_volume(g=32, ratio=2, z0=0.6, size=0.4):
    """A cube in front of a camera at the world origin looking along +z."""
    return VolumeSpec((g, g, g), (g * ratio,) * 3, (-size / 2, -size / 2, z0), (size,) * 3)


def ramp_image(W, H, a=0.2, b=0.001, c=0.0015):
    x = np.arange(W, dtype=float)
    y = np.arange(H, dtype=float)
    yy, xx = np.meshgrid(y, x, indexing="ij")
    img = a + b * xx + c * yy
    return np.repeat(img[..., None], 3, axis=-1).astype(np.float32)


def posed(R_deg=(10.0, -7.0), t=(0.03, -0.02, 0.05)):
    return rigid(rot_x(R_deg[0]) @ rot_y(R_deg[1]), t)


__all__ = ["frames", "plane_depth", "camera_volume", "ramp_image", "posed", "intrinsics"]
