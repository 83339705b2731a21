"""MI355X-native per-frame volumetric integration (TSDF geometry volume + asymmetric
colour volume through a depth-to-HD calibration) from "Creating Simplified 3D Models
with High Quality Textures" (arXiv 1602.06645), with batched/fused and differentiable
forms, ray casting of the volumes, marching cubes and quadric-error decimation of the mesh
(Sec. IV.C) and per-polygon texture maps (Sec. IV.D).  The work runs in libkfvol.so (HIP
for gfx950 and host C++, C ABI in include/kf.h)."""
from .api import (Scan, Volume, brick_shapes, decimate, integrate_backward,  # noqa: F401
                  integrate_batch, integrate_batch_counted, integrate_batch_noalloc,
                  integrate_batch_timed, release_graphs, texture_layout, volume_desc)
from .autograd import KFColourFn, se3_exp, se3_left_jacobian  # noqa: F401
