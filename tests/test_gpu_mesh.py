"""GPU parity of marching cubes (needs gfx950): kf_mesh_extract against the oracle's FP32
mesh, bit for bit (vertex positions, triangle indices and their order), on the oracle's
integration of the tiny scan, on random sign fields with zeros and unobserved voxels over
an odd-sized volume (every cube configuration), on an analytic sphere in a volume of
about 22 M voxels (many scan blocks, a ragged last block) and on the full kinect volume."""
import numpy as np
import pytest
import torch

import paper_1602_06645_amd as kf
from gpu_helpers import say
from kf_synth import configs
from kf_synth.scenes import VolumeSpec

pytestmark = pytest.mark.gpu
DEV = "cuda"


def upload_geometry(spec, tsdf, wg):
    vol = kf.Volume(spec)
    vol.tsdf.copy_(torch.as_tensor(np.ascontiguousarray(tsdf, np.float32)))
    vol.w_geom.copy_(torch.as_tensor(np.ascontiguousarray(wg, np.float32)))
    return vol


def assert_same_mesh(oracle, spec, tsdf, wg, min_tris=1000):
    vol = upload_geometry(spec, tsdf, wg)
    verts, tris = vol.mesh()
    torch.cuda.synchronize()
    ov, ot = oracle.marching_cubes(spec, tsdf, wg, "f32")
    assert len(ot) >= min_tris
    assert verts.shape == ov.shape and tris.shape == ot.shape
    v = verts.cpu().numpy()
    bad = v.view(np.uint32) != ov.view(np.uint32)
    assert not bad.any(), f"{bad.sum()} vertex coordinates differ (first at {np.argwhere(bad)[0]})"
    t = tris.cpu().numpy()
    bad = t != ot
    assert not bad.any(), f"{bad.sum()} triangle indices differ (first at {np.argwhere(bad)[0]})"
    return vol, ov, ot


def test_mesh_tiny_scan(oracle):
    say("mesh: tiny scan")
    spec, fr = configs.tiny(n_frames=6)
    st = oracle.State(spec, np.float32)
    oracle.integrate(spec, fr.numpy(), st)
    assert_same_mesh(oracle, spec, st.tsdf, st.wg)


def test_mesh_random_fields_odd_volume(oracle):
    say("mesh: random sign fields, odd volume")
    spec = VolumeSpec((45, 37, 29), (90, 74, 58), (-0.41, -0.37, -0.46), (0.9, 0.74, 0.58))
    rng = np.random.default_rng(61)
    n = int(np.prod(spec.gdim))
    F = rng.uniform(-1, 1, n).astype(np.float32)
    F[rng.uniform(size=n) < 0.01] = 0.0
    F[rng.uniform(size=n) < 0.01] = -0.0
    W = np.where(rng.uniform(size=n) < 0.03, 0.0, rng.uniform(0.5, 3, n)).astype(np.float32)
    assert_same_mesh(oracle, spec, F, W, min_tris=50000)


def test_mesh_sphere_many_blocks(oracle):
    say("mesh: analytic sphere, 300x260x280 voxels")
    spec = VolumeSpec((300, 260, 280), (600, 520, 560), (-0.6, -0.52, -0.56), (1.2, 1.04, 1.12))
    s = np.asarray(spec.extent) / np.asarray(spec.gdim)
    ax = [spec.origin[k] + (np.arange(spec.gdim[k]) + 0.5) * s[k] for k in range(3)]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    d = np.sqrt((x - 0.03) ** 2 + (y + 0.02) ** 2 + (z - 0.01) ** 2) - 0.45
    F = np.clip(d / 0.02, -1, 1).astype(np.float32).ravel()
    W = (np.abs(d) < 0.05).astype(np.float32).ravel()
    vol, ov, ot = assert_same_mesh(oracle, spec, F, W, min_tris=400000)
    # the capacity contract: too small is refused, the exact size works
    with pytest.raises(kf.api.L.KfError):
        vol.mesh(capacity=(len(ov), len(ot) - 1))
    v2, t2 = vol.mesh(capacity=(len(ov), len(ot)))
    torch.cuda.synchronize()
    assert torch.equal(t2.cpu(), torch.as_tensor(ot))


def test_mesh_empty_and_flat(oracle):
    say("mesh: unobserved volume, volume without a surface")
    spec = VolumeSpec((17, 9, 12), (34, 18, 24), (-0.5, -0.4, -0.55), (1.0, 0.8, 1.1))
    n = int(np.prod(spec.gdim))
    vol = upload_geometry(spec, np.full(n, -0.5, np.float32), np.zeros(n, np.float32))
    v, t = vol.mesh()
    torch.cuda.synchronize()
    assert v.shape == (0, 3) and t.shape == (0, 3)
    vol = upload_geometry(spec, np.full(n, 0.5, np.float32), np.ones(n, np.float32))
    v, t = vol.mesh()
    torch.cuda.synchronize()
    assert v.shape == (0, 3) and t.shape == (0, 3)


def test_mesh_full_size(oracle):
    """The kinect volume (256^3) integrated by the oracle from 12 frames: every vertex and
    triangle compared."""
    say("mesh: full-size kinect volume")
    spec, fr = configs.kinect(device=DEV, n_frames=12)
    st = oracle.State(spec, np.float32)
    oracle.integrate(spec, fr.numpy(), st)
    assert_same_mesh(oracle, spec, st.tsdf, st.wg, min_tris=80000)
