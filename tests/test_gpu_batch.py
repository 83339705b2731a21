"""GPU parity of the batched forms: fused K-frame passes, many uneven scans in one
persistent launch, graph replay, and the Kinect-like workload at full size on sampled
z-slabs (needs gfx950)."""
import numpy as np
import pytest
import torch

import paper_1602_06645_amd as kf
from gpu_helpers import assert_bitwise, integrate_plain, say, to_host
from kf_synth import configs
from kf_synth.scenes import VolumeSpec

pytestmark = pytest.mark.gpu
DEV = "cuda"


def test_multi_scene_uneven_equals_per_scene_plain(oracle):
    """Six scans of different volume sizes, colour ratios, image sizes and frame counts in
    one batch; each must equal its own frame-by-frame integration and the oracle."""
    scans = configs.multi_scene(n_scenes=6, n_frames=5, scale=0.125)
    scans[2] = (scans[2][0], scans[2][1].select(slice(0, 2)))      # uneven frame counts
    scans[4] = (scans[4][0], scans[4][1].select(slice(0, 0)))
    scans[5] = (scans[5][0], scans[5][1].as_float_rgb())
    say("multi-scene: " + ", ".join(f"{s.gdim[0]}^3 x{s.cdim[0] // s.gdim[0]} n={f.n}" for s, f in scans))
    vols = [kf.Volume(s) for s, _ in scans]
    pairs = [(v, kf.Scan.from_frames(f.to(DEV))) for v, (s, f) in zip(vols, scans)]
    kf.integrate_batch(pairs, frames_per_pass=3)
    for q, (spec, fr) in enumerate(scans):
        plain = kf.Volume(spec)
        integrate_plain(plain, fr.to(DEV))
        assert_bitwise(to_host(vols[q]), to_host(plain), f"scene {q} batch vs plain: ")
        st = oracle.State(spec, np.float32)
        oracle.integrate(spec, fr.numpy(), st)
        assert_bitwise(to_host(vols[q]), st.arrays(), f"scene {q} vs oracle: ")


def test_mixed_scans_in_wide_passes(oracle):
    """A 70-frame scan and a 12-frame scan (float images) on different volumes in one batch
    of 64-frame passes: the first pass holds 64 + 12 frames, the second 6 + 0; each scan
    equals the oracle."""
    spec_a, fr_a = configs.tiny(n_frames=70)
    spec_b = VolumeSpec((45, 37, 29), (90, 74, 58), (-0.41, -0.37, -0.46), (0.9, 0.74, 0.58))
    fr_b = fr_a.select(slice(20, 32)).as_float_rgb()
    say("mixed batch: 70 frames on 64^3/128^3 + 12 float frames on 45x37x29, K=64")
    va, vb = kf.Volume(spec_a), kf.Volume(spec_b)
    kf.integrate_batch([(va, kf.Scan.from_frames(fr_a.to(DEV))),
                        (vb, kf.Scan.from_frames(fr_b.to(DEV)))], frames_per_pass=64)
    for vol, spec, fr, name in ((va, spec_a, fr_a, "70-frame"), (vb, spec_b, fr_b, "12-frame")):
        st = oracle.State(spec, np.float32)
        oracle.integrate(spec, fr.numpy(), st)
        assert int((st.wc > 0).sum()) > 1000
        assert_bitwise(to_host(vol), st.arrays(), f"{name} scan vs oracle: ")


def test_graph_replays_match_eager():
    """The graph is recorded on first use and replayed afterwards; every replay (with
    eager work and synchronisation in between) equals the eager batch."""
    spec, fr = configs.tiny(n_frames=6)
    frd = fr.to(DEV)
    say("graph capture and replays")
    ref = kf.Volume(spec)
    kf.integrate_batch([(ref, kf.Scan.from_frames(frd))], frames_per_pass=2)
    want = to_host(ref)
    vol = kf.Volume(spec)
    scan = kf.Scan.from_frames(frd)
    for rep in range(4):
        vol.reset()
        junk = torch.randn(1 << 20, device=DEV).sum()      # unrelated eager work
        kf.integrate_batch([(vol, scan)], frames_per_pass=2, use_graph=True)
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert_bitwise(to_host(vol), want, f"replay {rep}: ")


def test_release_graphs_and_record_again():
    """kf_release_graphs empties the graph cache (at least the graph just recorded, with its
    workspace); the next call records the batch again and gives the same volume."""
    spec, fr = configs.tiny(n_frames=5)
    scan = kf.Scan.from_frames(fr.to(DEV))
    say("graph cache release")
    vol = kf.Volume(spec)
    kf.integrate_batch([(vol, scan)], frames_per_pass=3, use_graph=True)
    want = to_host(vol)
    n, nbytes = kf.release_graphs()
    assert n >= 1 and nbytes > 0
    assert kf.release_graphs() == (0, 0)
    vol.reset()
    kf.integrate_batch([(vol, scan)], frames_per_pass=3, use_graph=True)
    assert_bitwise(to_host(vol), want, "recorded again: ")


@pytest.fixture(scope="module")
def kinect8():
    """The Kinect-like workload at full size (256^3 / 512^3, 640x480 depth, 1920x1080
    RGB8), first 8 frames, generated on the GPU."""
    say("generating Kinect-like scan (8 frames) on the GPU")
    spec, fr = configs.kinect(device=DEV, n_frames=8)
    return spec, fr


def _oracle_slabs(oracle, spec, fr, gz, cz):
    st = oracle.State(spec, np.float32, gz=gz, cz=cz)
    oracle.integrate(spec, fr.numpy(), st)
    return st


def _slab(arr, dims, z):
    n = dims[0] * dims[1]
    return arr[z[0] * n:z[1] * n]


@pytest.mark.parametrize("K,use_graph", [(8, True), (1, False)])
def test_kinect_full_size_sampled_slabs(oracle, kinect8, K, use_graph):
    """Full-size volume in the benchmark's launch configuration (persistent fused passes,
    graph replay); compared with the oracle on seeded z-slab samples, which the oracle
    computes exactly because voxels are independent."""
    spec, fr = kinect8
    say(f"kinect full size: batch K={K} graph={use_graph}")
    vol = kf.Volume(spec)
    kf.integrate_batch([(vol, kf.Scan.from_frames(fr))], frames_per_pass=K, use_graph=use_graph)
    got = to_host(vol)
    rng = np.random.default_rng(77)
    total_upd = 0
    for _ in range(2):
        g0 = int(rng.integers(0, spec.gdim[2] - 6))
        c0 = int(rng.integers(0, spec.cdim[2] - 6))
        gz, cz = (g0, g0 + 6), (c0, c0 + 6)
        say(f"  oracle slabs geometry z{gz} colour z{cz}")
        st = _oracle_slabs(oracle, spec, fr, gz, cz)
        for name, g, w, dims, z in zip(["tsdf", "w_geom", "r", "g", "b", "w_col"], got,
                                       st.arrays(), [spec.gdim] * 2 + [spec.cdim] * 4,
                                       [gz] * 2 + [cz] * 4):
            gs = _slab(g, dims, z)
            assert np.array_equal(gs.view(np.uint32), w.view(np.uint32)), f"{name} slab {z} differs"
        total_upd += int((st.wc > 0).sum()) + int((st.wg > 0).sum())
    assert total_upd > 1000


def test_kinect_properties_at_any_size(kinect8):
    """Whole-volume properties: weights are integers bounded by the frame count and
    w_max, TSDF in [-1, 1], colour in [0, 1], colour weights in [0, 1]."""
    spec, fr = kinect8
    say("kinect full size: whole-volume invariants")
    vol = kf.Volume(spec)
    kf.integrate_batch([(vol, kf.Scan.from_frames(fr))], frames_per_pass=4)
    tsdf, wg, r, g, b, wc = vol.arrays()
    torch.cuda.synchronize()
    assert bool((wg == torch.round(wg)).all()) and float(wg.max()) <= min(fr.n, fr.w_max)
    seen = wg > 0
    assert bool((tsdf[seen] <= 1).all()) and bool((tsdf[seen] >= -1 - 1e-6).all())
    assert float(wc.min()) >= 0 and float(wc.max()) <= 1
    for c in (r, g, b):
        assert float(c.min()) >= 0 and float(c.max()) <= 1 + 1e-6
    assert int((wc > 0).sum()) > 10 ** 5


def test_culling_changes_nothing(kinect8, monkeypatch):
    """Skipping bricks that cannot pass the depth tests leaves every bit of the volume
    unchanged (the library reads KF_DISABLE_CULL on every call)."""
    spec, fr = kinect8
    say("kinect full size: culling on vs off")
    a, b = kf.Volume(spec), kf.Volume(spec)
    scan = kf.Scan.from_frames(fr)
    kf.integrate_batch([(a, scan)], frames_per_pass=8)
    monkeypatch.setenv("KF_DISABLE_CULL", "1")
    kf.integrate_batch([(b, scan)], frames_per_pass=8)
    monkeypatch.delenv("KF_DISABLE_CULL")
    assert_bitwise(to_host(a), to_host(b), "cull vs no cull: ")


def test_kinect_full_size_wide_passes(oracle, monkeypatch):
    """The full-size workload, 70 frames in passes of 64 frames (64 + 6) replayed from a
    graph: seeded z-slabs equal the oracle's, and culling changes nothing."""
    say("generating Kinect-like scan (70 frames) on the GPU")
    spec, fr = configs.kinect(device=DEV, n_frames=70)
    scan = kf.Scan.from_frames(fr)
    vol = kf.Volume(spec)
    kf.integrate_batch([(vol, scan)], frames_per_pass=64, use_graph=True)
    got = to_host(vol)
    rng = np.random.default_rng(78)
    g0 = int(rng.integers(24, 150))
    c0 = int(rng.integers(24, 150))
    gz, cz = (g0, g0 + 4), (c0, c0 + 4)
    say(f"  oracle slabs geometry z{gz} colour z{cz}")
    st = _oracle_slabs(oracle, spec, fr, gz, cz)
    for name, g, w, dims, z in zip(["tsdf", "w_geom", "r", "g", "b", "w_col"], got, st.arrays(),
                                   [spec.gdim] * 2 + [spec.cdim] * 4, [gz] * 2 + [cz] * 4):
        assert np.array_equal(_slab(g, dims, z).view(np.uint32), w.view(np.uint32)), \
            f"{name} slab {z} differs"
    assert int((st.wc > 0).sum()) > 1000 and int((st.wg > 0).sum()) > 1000
    say("  culling off")
    monkeypatch.setenv("KF_DISABLE_CULL", "1")
    b = kf.Volume(spec)
    kf.integrate_batch([(b, scan)], frames_per_pass=64)
    monkeypatch.delenv("KF_DISABLE_CULL")
    assert_bitwise(got, to_host(b), "cull vs no cull, 64 frames per pass: ")
