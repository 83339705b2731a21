"""GPU parity at the full sizes of the two batched workloads (needs gfx950 and about
130 GB of device memory):

* the fused multi-frame scan: geometry 512^3 / colour 1024^3 over 1 m, 256 frames of
  640x480 depth + 1920x1080 RGB8, integrated in passes of K = 8 frames replayed from a
  HIP graph and at the tuned K; seeded z-slabs equal the oracle's bit for bit, and the
  whole volume equals the frame-by-frame result and the other K;
* the many-uneven-scenes batch: 16 seeded scans of volumes from 96^3 to 384^3 with
  colour ratios 2 and 3 (86 GB of state), 32 frames each of mixed image sizes, in one
  batch call (one pass: one cull and one persistent launch per brick kind); every scene
  equals its own frame-by-frame integration and, on seeded z-slabs, the oracle.

Voxels are independent, so the oracle computes any set of z-slabs exactly.
"""
import numpy as np
import pytest
import torch

import paper_1602_06645_amd as kf
from gpu_helpers import STATE_NAMES, integrate_plain, say
from kf_synth import configs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _slab(t: torch.Tensor, dims, z) -> np.ndarray:
    n = dims[0] * dims[1]
    return t[z[0] * n:z[1] * n].cpu().numpy()


def _check_slabs(oracle, spec, fr_host, vol, gz, cz, where):
    """The volume's geometry slab gz and colour slab cz against the oracle's; returns the
    numbers of observed geometry and colour voxels in them."""
    say(f"  {where}: oracle slabs geometry z{gz} colour z{cz}")
    st = oracle.State(spec, np.float32, gz=gz, cz=cz)
    oracle.integrate(spec, fr_host, st)
    torch.cuda.synchronize()
    for name, got, want, dims, z in zip(STATE_NAMES, vol.arrays(), st.arrays(),
                                        [spec.gdim] * 2 + [spec.cdim] * 4, [gz] * 2 + [cz] * 4):
        g = _slab(got, dims, z)
        bad = np.flatnonzero(g.view(np.uint32) != want.view(np.uint32))
        assert bad.size == 0, (f"{where}: {name} slab {z}: {bad.size} voxels differ, first at "
                               f"{bad[:4]}: gpu {g[bad[:4]]} oracle {want[bad[:4]]}")
    return int((st.wg > 0).sum()), int((st.wc > 0).sum())


def _equal_on_device(a: kf.Volume, b: kf.Volume, where: str) -> None:
    for name, x, y in zip(STATE_NAMES, a.arrays(), b.arrays()):
        assert torch.equal(x.view(torch.int32), y.view(torch.int32)), f"{where}: {name} differs"


# ------------------------------------------------------------------ fused scan, 512^3 / 1024^3


@pytest.fixture(scope="module")
def fused_scan():
    say("fused workload: generating 256 frames of 640x480 + 1920x1080 on the GPU")
    spec, fr = configs.fused(device=DEV)
    return spec, fr


@pytest.fixture(scope="module")
def fused_k8(fused_scan):
    spec, fr = fused_scan
    say("fused workload: K = 8 passes, graph capture and replay")
    vol = kf.Volume(spec)
    scan = kf.Scan.from_frames(fr)
    kf.integrate_batch([(vol, scan)], frames_per_pass=8, use_graph=True)
    torch.cuda.synchronize()
    # replay the recorded graph on a reset volume: the replay must give the same volume
    ref = [t.clone() for t in vol.arrays()]
    vol.reset()
    kf.integrate_batch([(vol, scan)], frames_per_pass=8, use_graph=True)
    torch.cuda.synchronize()
    for name, x, y in zip(STATE_NAMES, vol.arrays(), ref):
        assert torch.equal(x.view(torch.int32), y.view(torch.int32)), f"graph replay: {name} differs"
    del ref
    yield vol
    del vol
    torch.cuda.empty_cache()


def test_fused_scan_k8_graph_slabs_match_oracle(oracle, fused_scan, fused_k8):
    spec, fr = fused_scan
    fr_host = fr.numpy()
    rng = np.random.default_rng(1303)
    seen_g = seen_c = 0
    for _ in range(2):
        g0 = int(rng.integers(40, spec.gdim[2] - 44))
        c0 = int(rng.integers(80, spec.cdim[2] - 84))
        sg, sc = _check_slabs(oracle, spec, fr_host, fused_k8, (g0, g0 + 4), (c0, c0 + 4),
                              "fused K=8")
        seen_g += sg
        seen_c += sc
    assert seen_g > 1000 and seen_c > 10000


def test_fused_scan_tuned_k_equals_k8(fused_scan, fused_k8):
    from paper_1602_06645_amd import autotune
    spec, fr = fused_scan
    K = autotune.frames_per_pass("fused", default=64)
    say(f"fused workload: tuned K = {K} against K = 8, whole volume")
    vol = kf.Volume(spec)
    kf.integrate_batch([(vol, kf.Scan.from_frames(fr))], frames_per_pass=K, use_graph=True)
    torch.cuda.synchronize()
    _equal_on_device(vol, fused_k8, f"K={K} vs K=8")
    del vol
    torch.cuda.empty_cache()


def test_fused_scan_plain_equals_fused(fused_scan, fused_k8):
    spec, fr = fused_scan
    say("fused workload: 256 kf_integrate calls, whole volume against the fused K = 8 scan")
    vol = kf.Volume(spec)
    integrate_plain(vol, fr)
    torch.cuda.synchronize()
    _equal_on_device(vol, fused_k8, "plain vs fused K=8")
    del vol
    torch.cuda.empty_cache()


# ------------------------------------------------------------- 16 uneven scenes in one batch


@pytest.fixture(scope="module")
def many_scenes():
    say("many-scenes workload: generating 16 scans (32 frames each) on the GPU")
    scans = configs.multi_scene(device=DEV)
    say("many-scenes workload: " + ", ".join(
        f"{s.gdim[0]}^3 x{s.cdim[0] // s.gdim[0]} d{f.depth.shape[2]} c{f.rgb.shape[2]}"
        for s, f in scans))
    return scans


def test_many_scenes_full_size_one_batch(oracle, many_scenes):
    scans = many_scenes
    total = sum(configs.state_bytes(s.gdim[0], s.cdim[0] // s.gdim[0]) for s, _ in scans)
    assert total <= 160e9 and len(scans) == 16
    say(f"many-scenes workload: one batch call over {total / 1e9:.1f} GB of state, K = 32, graph")
    vols = [kf.Volume(s) for s, _ in scans]
    pairs = [(v, kf.Scan.from_frames(f)) for v, (_, f) in zip(vols, scans)]
    kf.integrate_batch(pairs, frames_per_pass=32, use_graph=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1404)
    seen = 0
    for q, (spec, fr) in enumerate(scans):
        say(f"  scene {q}: {spec.gdim[0]}^3 / {spec.cdim[0]}^3, frame-by-frame reference")
        plain = kf.Volume(spec)
        integrate_plain(plain, fr)
        torch.cuda.synchronize()
        _equal_on_device(vols[q], plain, f"scene {q} batch vs plain")
        del plain
        torch.cuda.empty_cache()
        g0 = int(rng.integers(spec.gdim[2] // 4, spec.gdim[2] // 2))
        c0 = g0 * (spec.cdim[2] // spec.gdim[2]) + int(rng.integers(0, 8))
        _, sc = _check_slabs(oracle, spec, fr.numpy(), vols[q], (g0, g0 + 3), (c0, c0 + 3),
                             f"scene {q}")
        seen += sc
    assert seen > 10000
    del vols, pairs
    torch.cuda.empty_cache()
