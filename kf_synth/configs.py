"""The seeded workloads (volume shape + scan) used by the tests and the benchmark.

Each stands in for the hand-held scans of Sec. V (small textured objects in a cube of
variable size, 384^3 geometry / 768^3 colour in the paper) with synthetic data of the
same structure; the recipes are stated in each function.
"""
from __future__ import annotations

import numpy as np

from .scenes import (DEPTH_INTRINSICS, RGB_INTRINSICS, Frames, Scene, VolumeSpec, intrinsics,
                     orbit_poses, random_scene, render_scan, surface_triangles)


def tiny(device="cpu", n_frames: int = 10) -> tuple[VolumeSpec, Frames]:
    """64^3 geometry / 128^3 colour over a 1 m cube; 10 frames of 160x120 depth
    (noise sd 0.002 z^2, no holes) and 320x240 RGB; a 0.2 m sphere on the ground plane;
    10 poses evenly spaced on a 0.8 m orbit; trunc = 3 geometry voxels; w_max = 64."""
    rng = np.random.default_rng(1001)
    vol = VolumeSpec.cube(64, 2, 1.0)
    poses = orbit_poses(n_frames)
    fr = render_scan(_tiny_scene(), poses, (160, 120), (320, 240), 0.002, 0.0, rng,
                     trunc=3 * vol.geom_voxel, w_max=64, device=device)
    return vol, fr


def _tiny_scene() -> Scene:
    sc = Scene(-0.45, np.array([[0.85, 0.8, 0.2], [0.2, 0.3, 0.75]]), noise_seed=11)
    sc.spheres.append((np.array([0.0, 0.0, -0.25]), 0.2, np.array([[0.9, 0.25, 0.2],
                                                                   [0.25, 0.8, 0.35]])))
    return sc


def tiny_triangles(n_tri: int = 160, edge_px: int = 6, n_frames: int = 10, seed: int = 2001):
    """Triangles on the surfaces of the tiny() scene (three depth pixels e = 6 apart in its
    160x120 views, about 3.7 cm at the 0.8 m orbit) and a texel size of 5 mm.  Returns
    (float32 [n_tri, 3, 3], size_pixel)."""
    K = intrinsics(*DEPTH_INTRINSICS[(160, 120)])
    tri = surface_triangles(_tiny_scene(), K, 160, 120, orbit_poses(n_frames), n_tri, edge_px,
                            np.random.default_rng(seed), box=(-0.5, 0.5))
    return tri, 0.005


def kinect(device="cpu", n_frames: int = 300, gdim: int = 256, ratio: int = 2,
           size: float = 0.75, seed: int = 1002, n_spheres: int = 3, n_boxes: int = 2,
           depth_size=(640, 480), rgb_size=(1920, 1080)) -> tuple[VolumeSpec, Frames]:
    """Kinect-like plain fusion: 256^3 geometry / 512^3 colour over 0.75 m; 300 frames of
    640x480 depth (noise sd 0.0012 z^2, 1 % holes) and 1920x1080 RGB; 3 spheres and
    2 boxes on a plane; 360 deg orbit (r 0.8 m, h 0.3 m) with +-5 cm jitter per axis;
    trunc = 4 geometry voxels; w_max = 128.  The orbit is drawn for 300 frames and
    the first n_frames of it are rendered."""
    rng = np.random.default_rng(seed)
    vol = VolumeSpec.cube(gdim, ratio, size)
    sc = random_scene(rng, size, n_spheres, n_boxes)
    poses = orbit_poses(300 if n_frames <= 300 else n_frames, jitter=0.05, rng=rng)[:n_frames]
    fr = render_scan(sc, poses, depth_size, rgb_size, 0.0012, 0.01, rng,
                     trunc=4 * vol.geom_voxel, w_max=128, device=device)
    return vol, fr


def kinect_triangles(n_tri: int = 8192, edge_px: int = 16, n_frames: int = 300,
                     seed: int = 2002, size: float = 0.75, scene_seed: int = 1002,
                     device="cpu"):
    """A mesh-like triangle set on the surfaces of the kinect() scene, for texture maps:
    n_tri triangles whose vertices are the surface points of three depth pixels e = 16
    pixels apart (2.4 cm across at the 0.8 m orbit, longer where the view grazes the
    ground), seen from the first n_frames scan poses, inside the volume's box: a
    simplified model of a few thousand polygons.  At the default sizes the maps hold
    about 20 M texels (a 4096-row atlas about 7400 texels wide).  The texel size is the footprint of one HD pixel at the scan distance
    (0.8 m / f_hd, Sec. IV.D: set by the HD camera's resolution and the scanning distance).
    Returns (float32 [n_tri, 3, 3] triangles, size_pixel in metres)."""
    rng = np.random.default_rng(scene_seed)      # the scene and poses of kinect(seed=1002)
    sc = random_scene(rng, size, 3, 2)
    poses = orbit_poses(300 if n_frames <= 300 else n_frames, jitter=0.05, rng=rng)[:n_frames]
    K = intrinsics(*DEPTH_INTRINSICS[(640, 480)])
    tri = surface_triangles(sc, K, 640, 480, poses, n_tri, edge_px,
                            np.random.default_rng(seed), box=(-size / 2, size / 2), device=device)
    return tri, 0.8 / RGB_INTRINSICS[(1920, 1080)][0]


def fused(device="cpu", n_frames: int = 256) -> tuple[VolumeSpec, Frames]:
    """Fused multi-frame workload: 512^3 geometry / 1024^3 colour over 1.0 m; 256 frames
    of 640x480 + 1920x1080 from the Kinect-like generator with 4 spheres + 4 boxes."""
    rng = np.random.default_rng(1003)
    vol = VolumeSpec.cube(512, 2, 1.0)
    sc = random_scene(rng, 1.0, 4, 4)
    poses = orbit_poses(n_frames, jitter=0.05, rng=rng)
    fr = render_scan(sc, poses, (640, 480), (1920, 1080), 0.0012, 0.01, rng,
                     trunc=4 * vol.geom_voxel, w_max=128, device=device)
    return vol, fr


GEOM_CHOICES = (96, 128, 192, 256, 384)
DEPTH_CHOICES = ((320, 240), (480, 360), (640, 480))
RGB_CHOICES = ((960, 540), (1280, 720), (1920, 1080))


def multi_scene_draw(j: int, budget_bytes: float = 160e9):
    """Shape draw for scene j of the many-uneven-scenes workload.  Returns
    (seed, gdim, ratio, depth_size, rgb_size).  The whole batch is redrawn with
    seed + 100 until its state fits the budget (see multi_scene_shapes)."""
    rng = np.random.default_rng(4000 + j)
    g = int(rng.choice(GEOM_CHOICES))
    ratio = int(rng.choice((2, 3)))
    ds = DEPTH_CHOICES[int(rng.integers(3))]
    cs = RGB_CHOICES[int(rng.integers(3))]
    return 4000 + j, g, ratio, ds, cs


def state_bytes(g: int, ratio: int) -> int:
    return 8 * g ** 3 + 16 * (g * ratio) ** 3


def multi_scene_shapes(n_scenes: int = 16, budget_bytes: float = 160e9):
    offset = 0
    while True:
        shapes = []
        for j in range(n_scenes):
            rng = np.random.default_rng(4000 + j + offset)
            g = int(rng.choice(GEOM_CHOICES))
            ratio = int(rng.choice((2, 3)))
            ds = DEPTH_CHOICES[int(rng.integers(3))]
            cs = RGB_CHOICES[int(rng.integers(3))]
            shapes.append((4000 + j + offset, g, ratio, ds, cs))
        if sum(state_bytes(s[1], s[2]) for s in shapes) <= budget_bytes:
            return shapes
        offset += 100


def multi_scene(device="cpu", n_scenes: int = 16, n_frames: int = 32, scale: float = 1.0,
                budget_bytes: float = 160e9):
    """Many uneven scenes: 16 independent seeded scans, geometry drawn from
    {96,128,192,256,384}^3 with colour ratio 2 or 3 over 0.75 m, 32 frames each with
    depth from {320x240, 480x360, 640x480} and RGB from {960x540, 1280x720, 1920x1080}.
    `scale` < 1 shrinks every volume dimension (rounded, at least 8) for tests."""
    out = []
    for seed, g, ratio, ds, cs in multi_scene_shapes(n_scenes, budget_bytes):
        rng = np.random.default_rng(seed)
        gs = max(8, int(round(g * scale)))
        vol = VolumeSpec.cube(gs, ratio, 0.75)
        sc = random_scene(rng, 0.75, 3, 2)
        poses = orbit_poses(n_frames, jitter=0.05, rng=rng)
        fr = render_scan(sc, poses, ds, cs, 0.0012, 0.01, rng, trunc=4 * vol.geom_voxel,
                         w_max=128, device=device)
        out.append((vol, fr))
    return out


def gradient_weights(n_colour: int, seed: int = 5005, device="cpu"):
    """The seeded random linear functional g (3 x n_colour, N(0,1)) of the backward."""
    import torch
    rng = np.random.default_rng(seed)
    return torch.as_tensor(rng.standard_normal((3, n_colour), dtype=np.float32), device=device)
