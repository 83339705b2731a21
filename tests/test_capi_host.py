"""Host-only checks of the C ABI (no GPU needed): the library loads, exports every
function declared in include/kf.h, and rejects bad arguments before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1602_06645_amd import _lib as L
from paper_1602_06645_amd.api import volume_desc
from kf_synth.scenes import VolumeSpec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "kf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kf_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = declared_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/kf.h but not exported"
    assert set(names) == set(L.SIGNATURES), "binding and header disagree"


def _desc(**kw):
    spec = VolumeSpec.cube(16, 2, 1.0)
    d = volume_desc(spec)
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def test_status_strings():
    lib = L.load()
    assert lib.kf_status_str(0) == b"ok"
    assert lib.kf_status_str(4) == b"device error"
    assert lib.kf_status_str(99) == b"unknown status"


def test_buffer_bytes_and_desc_validation():
    lib = L.load()
    out = (C.c_size_t * 6)()
    assert lib.kf_volume_buffer_bytes(C.byref(_desc()), out) == L.KF_OK
    assert list(out) == [16 ** 3 * 4] * 2 + [32 ** 3 * 4] * 4
    bad = _desc()
    bad.geom_dim[1] = 0
    assert lib.kf_volume_buffer_bytes(C.byref(bad), out) == L.KF_E_SHAPE
    assert b"dimension" in lib.kf_last_error()
    bad = _desc()
    bad.extent[2] = -1.0
    assert lib.kf_volume_buffer_bytes(C.byref(bad), out) == L.KF_E_ARG
    bad = _desc(colour_band=float("nan"))
    assert lib.kf_volume_buffer_bytes(C.byref(bad), out) == L.KF_E_ARG
    bad = _desc()
    bad.colour_dim[:] = [2048, 2048, 1024]
    assert lib.kf_volume_buffer_bytes(C.byref(bad), out) == L.KF_E_RANGE
    bad = _desc()
    bad.colour_dim[:] = [8192, 8192, 8]      # one z slice of 2^26 voxels
    assert lib.kf_volume_buffer_bytes(C.byref(bad), out) == L.KF_E_RANGE
    assert b"slice" in lib.kf_last_error()
    bad.colour_dim[:] = [8192, 8191, 8]
    assert lib.kf_volume_buffer_bytes(C.byref(bad), out) == L.KF_OK
    assert lib.kf_volume_buffer_bytes(None, out) == L.KF_E_ARG


def _volume():
    lib = L.load()
    bufs = L.VolumeBuffers(*([0x1000] * 6))   # never dereferenced by these host-only calls
    h = C.c_void_p()
    assert lib.kf_volume_create(C.byref(_desc()), C.byref(bufs), C.byref(h)) == L.KF_OK
    return h


def test_create_rejects_null_buffers():
    lib = L.load()
    bufs = L.VolumeBuffers(0x1000, 0x1000, 0, 0x1000, 0x1000, 0x1000)
    h = C.c_void_p()
    assert lib.kf_volume_create(C.byref(_desc()), C.byref(bufs), C.byref(h)) == L.KF_E_ARG


def _call_integrate(h, **over):
    lib = L.load()
    K = np.array([[525.0, 0, 319.5], [0, 525.0, 239.5], [0, 0, 1]])
    Kr = np.array([[1050.0, 0, 959.5], [0, 1050.0, 539.5], [0, 0, 1]])
    T = np.eye(4)
    args = dict(depth=0x2000, dw=640, dh=480, rgb=0x3000, fmt=0, cw=1920, ch=1080, K_d=K,
                K_rgb=Kr, T_rd=T, T_wc=T, trunc=0.01, w_max=128.0)
    args.update(over)
    keep = [np.ascontiguousarray(args[k], np.float64) for k in ("K_d", "K_rgb", "T_rd", "T_wc")]
    return lib.kf_integrate(h, C.c_void_p(args["depth"]), args["dw"], args["dh"],
                            C.c_void_p(args["rgb"]), args["fmt"], args["cw"], args["ch"],
                            *[C.c_void_p(a.ctypes.data) for a in keep], args["trunc"],
                            args["w_max"], None)


@pytest.mark.parametrize("over,code", [
    (dict(depth=0), L.KF_E_ARG),
    (dict(dw=0), L.KF_E_SHAPE),
    (dict(cw=1), L.KF_E_SHAPE),
    (dict(fmt=7), L.KF_E_ARG),
    (dict(trunc=0.0), L.KF_E_ARG),
    (dict(trunc=float("inf")), L.KF_E_ARG),
    (dict(w_max=0.5), L.KF_E_ARG),
    (dict(K_d=np.array([[525.0, 1.0, 319.5], [0, 525.0, 239.5], [0, 0, 1]])), L.KF_E_ARG),
    (dict(K_rgb=np.array([[-5.0, 0, 9.0], [0, 5.0, 5.0], [0, 0, 1]])), L.KF_E_ARG),
    (dict(K_d=np.array([[525.0, 0, 319.5], [0, 525.0, 239.5], [0, 0, 2.0]])), L.KF_E_ARG),
    (dict(T_wc=np.diag([1.0, 1.0, 1.1, 1.0])), L.KF_E_ARG),
    (dict(T_rd=np.array([[1.0, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0.1, 1]])), L.KF_E_ARG),
    (dict(T_wc=np.full((4, 4), np.nan)), L.KF_E_ARG),
    (dict(cw=50000, ch=50000), L.KF_E_RANGE),
    (dict(dw=65536, dh=2), L.KF_E_RANGE),
    (dict(dw=30000, dh=20000), L.KF_E_RANGE),
])
def test_integrate_rejects_bad_arguments(over, code):
    h = _volume()
    try:
        assert _call_integrate(h, **over) == code
        assert L.load().kf_last_error() != b""
    finally:
        L.load().kf_volume_destroy(h)


def test_null_handles():
    lib = L.load()
    assert lib.kf_volume_reset(None, None) == L.KF_E_ARG
    lib.kf_volume_destroy(None)
    assert _call_integrate(None) == L.KF_E_ARG


def test_batch_rejects_bad_arguments():
    lib = L.load()
    h = _volume()
    try:
        assert lib.kf_integrate_batch(None, 1, 1, 0, None) == L.KF_E_ARG
        sc = (L.Scene * 2)()
        for q in range(2):
            sc[q].vol = h.value
            sc[q].n_frames = 0
        assert lib.kf_integrate_batch(sc, 2, 1, 0, None) == L.KF_E_ARG   # same volume twice
        assert b"twice" in lib.kf_last_error()
        assert lib.kf_integrate_batch(sc, 1, 0, 0, None) == L.KF_E_ARG   # K < 1
        sc[0].n_frames = -1
        assert lib.kf_integrate_batch(sc, 1, 1, 0, None) == L.KF_E_ARG
        assert lib.kf_integrate_batch_counted(sc, 1, 1, None, None, None) == L.KF_E_ARG
    finally:
        lib.kf_volume_destroy(h)


def test_noalloc_batch_refuses_workspace_above_its_array():
    """kf_integrate_batch_noalloc checks its arguments like kf_integrate_batch and returns
    KF_E_RANGE, before any device work, when the batch's workspace exceeds the library's
    256 MiB array (a 512^3 / 1024^3 pair of volumes needs 75 MB of live lists, and 64
    frames of 640x480 take 5 MB each; the buffers here are fake addresses)."""
    lib = L.load()
    spec = VolumeSpec.cube(512, 2, 1.0)
    bufs = L.VolumeBuffers(*([0x1000] * 6))
    h = C.c_void_p()
    assert lib.kf_volume_create(C.byref(volume_desc(spec)), C.byref(bufs), C.byref(h)) == L.KF_OK
    K = np.ascontiguousarray([[525.0, 0, 319.5], [0, 525.0, 239.5], [0, 0, 1]])
    Kr = np.ascontiguousarray([[1050.0, 0, 959.5], [0, 1050.0, 539.5], [0, 0, 1]])
    T = np.ascontiguousarray(np.eye(4))
    Tw = np.ascontiguousarray(np.tile(np.eye(4), (64, 1, 1)))
    try:
        sc = (L.Scene * 1)()
        sc[0].vol, sc[0].n_frames, sc[0].depth, sc[0].rgb = h.value, 64, 0x2000, 0x3000
        sc[0].fmt, sc[0].dw, sc[0].dh, sc[0].cw, sc[0].ch = L.KF_RGB8, 640, 480, 1920, 1080
        sc[0].K_d, sc[0].K_rgb = K.ctypes.data, Kr.ctypes.data
        sc[0].T_rgb_from_d, sc[0].T_world_from_cam = T.ctypes.data, Tw.ctypes.data
        sc[0].trunc_m, sc[0].w_max = 0.008, 128.0
        assert lib.kf_integrate_batch_noalloc(sc, 1, 1, None) == L.KF_E_RANGE
        assert b"workspace" in lib.kf_last_error()
        assert lib.kf_integrate_batch_noalloc(sc, 1, 0, None) == L.KF_E_ARG      # K < 1
        assert lib.kf_integrate_batch_noalloc(None, 1, 1, None) == L.KF_E_ARG
        sc[0].trunc_m = -1.0
        assert lib.kf_integrate_batch_noalloc(sc, 1, 1, None) == L.KF_E_ARG
    finally:
        lib.kf_volume_destroy(h)


def test_brick_shapes_are_listed_and_checked():
    """kf_brick_shapes lists the compiled shapes (default first, 64 columns each); a shape
    outside the list is KF_E_UNSUPPORTED before any device work (fake buffers)."""
    lib = L.load()
    for kind in (0, 1):
        n = C.c_int32(0)
        assert lib.kf_brick_shapes(kind, None, 0, C.byref(n)) == L.KF_OK and n.value >= 2
        buf = np.zeros((n.value, 3), np.int32)
        assert lib.kf_brick_shapes(kind, buf.ctypes.data, n.value, C.byref(n)) == L.KF_OK
        assert all(x * y == 64 for x, y, _ in buf)
        assert len({tuple(r) for r in buf}) == n.value
    assert tuple(buf[0]) == (8, 8, 8)
    assert lib.kf_brick_shapes(2, None, 0, C.byref(n)) == L.KF_E_ARG
    h = _volume()
    try:
        sc = (L.Scene * 1)()
        sc[0].vol = h.value
        sc[0].n_frames = 0
        b = L.Bricks()
        b.geom[:] = (16, 4, 8)
        b.colour[:] = (4, 4, 4)
        assert lib.kf_integrate_batch_bricks(sc, 1, 1, 0, C.byref(b), None) == L.KF_E_UNSUPPORTED
        assert b"not one of the compiled shapes" in lib.kf_last_error()
        b.colour[:] = (8, 8, 8)
        b.geom[:] = (8, 8, 32)
        assert lib.kf_integrate_batch_bricks(sc, 1, 1, 0, C.byref(b), None) == L.KF_E_UNSUPPORTED
        assert lib.kf_integrate_batch_counted(sc, 1, 1, C.byref(b), None, None) == L.KF_E_UNSUPPORTED
    finally:
        lib.kf_volume_destroy(h)


def test_autotune_entries_are_keyed_by_architecture(tmp_path):
    import json
    from paper_1602_06645_amd import autotune
    path = tmp_path / "tuning.json"
    path.write_text(json.dumps({"gfx950": {"fused": {"frames_per_pass": 48, "bricks": {
        "geometry": [32, 2, 8], "colour": [8, 8, 4]}}}}))
    assert autotune.frames_per_pass("fused", arch="gfx950", path=str(path)) == 48
    assert autotune.bricks("fused", arch="gfx950", path=str(path)) == {"geometry": (32, 2, 8),
                                                                      "colour": (8, 8, 4)}
    assert autotune.frames_per_pass("fused", default=7, arch="gfx942", path=str(path)) == 7
    assert autotune.bricks("fused", arch="gfx942", path=str(path)) is None
    assert autotune.bricks("kinect", arch="gfx950", path=str(path)) is None


def test_timed_batch_rejects_bad_arguments():
    """Event arrays are checked, and too few events for the passes is an argument error
    returned before any device work (the volume buffers here are fake addresses)."""
    lib = L.load()
    h = _volume()
    try:
        K = np.array([[525.0, 0, 319.5], [0, 525.0, 239.5], [0, 0, 1]])
        Kr = np.array([[1050.0, 0, 959.5], [0, 1050.0, 539.5], [0, 0, 1]])
        T = np.eye(4)
        poses = np.stack([np.eye(4)] * 3)
        sc = (L.Scene * 1)()
        sc[0].vol = h.value
        sc[0].n_frames = 3
        sc[0].depth, sc[0].rgb, sc[0].fmt = 0x2000, 0x3000, L.KF_RGB8
        sc[0].dw, sc[0].dh, sc[0].cw, sc[0].ch = 640, 480, 1920, 1080
        sc[0].K_d, sc[0].K_rgb = K.ctypes.data, Kr.ctypes.data
        sc[0].T_rgb_from_d, sc[0].T_world_from_cam = T.ctypes.data, poses.ctypes.data
        sc[0].trunc_m, sc[0].w_max = 0.01, 128.0
        ev = (C.c_void_p * 3)(0x10, 0x20, 0x30)
        assert lib.kf_integrate_batch_timed(sc, 1, 1, None, None, None, ev, 3, None) == L.KF_E_ARG
        assert lib.kf_integrate_batch_timed(sc, 1, 1, None, ev, None, ev, 0, None) == L.KF_E_ARG
        holey = (C.c_void_p * 3)(0x10, None, 0x30)
        assert lib.kf_integrate_batch_timed(sc, 1, 1, None, ev, None, holey, 3, None) == L.KF_E_ARG
        assert lib.kf_integrate_batch_timed(sc, 1, 1, None, ev, holey, ev, 3, None) == L.KF_E_ARG
        # K = 1 makes three passes; two events are too few
        assert lib.kf_integrate_batch_timed(sc, 1, 1, None, ev, ev, ev, 2, None) == L.KF_E_ARG
        assert b"below the number of passes" in lib.kf_last_error()
    finally:
        lib.kf_volume_destroy(h)


def test_raycast_rejects_bad_arguments():
    lib = L.load()
    h = _volume()
    try:
        K = np.array([[131.25, 0, 79.5], [0, 131.25, 59.5], [0, 0, 1.0]])
        T = np.eye(4)
        out = C.c_void_p(0x4000)

        def call(K=K, T=T, w=160, hgt=120, step=0.01, depth=out):
            Kc, Tc = np.ascontiguousarray(K, np.float64), np.ascontiguousarray(T, np.float64)
            return lib.kf_raycast(h, w, hgt, C.c_void_p(Kc.ctypes.data), C.c_void_p(Tc.ctypes.data),
                                  step, depth, None, None, None, None)
        assert call(step=0.0) == L.KF_E_ARG
        assert call(step=float("nan")) == L.KF_E_ARG
        assert call(w=0) == L.KF_E_SHAPE
        assert call(depth=None) == L.KF_E_ARG
        assert call(K=np.array([[131.25, 0.5, 79.5], [0, 131.25, 59.5], [0, 0, 1.0]])) == L.KF_E_ARG
        assert call(T=np.diag([1.0, 1.0, 1.2, 1.0])) == L.KF_E_ARG
        assert call(w=50000, hgt=50000) == L.KF_E_RANGE
        assert lib.kf_raycast(None, 4, 4, None, None, 0.01, out, None, None, None, None) == L.KF_E_ARG
    finally:
        lib.kf_volume_destroy(h)
    # a volume with a single voxel along an axis cannot be ray cast
    d = _desc()
    d.geom_dim[2] = 1
    bufs = L.VolumeBuffers(*([0x1000] * 6))
    h1 = C.c_void_p()
    assert lib.kf_volume_create(C.byref(d), C.byref(bufs), C.byref(h1)) == L.KF_OK
    try:
        Kc = np.array([[131.25, 0, 79.5], [0, 131.25, 59.5], [0, 0, 1.0]])
        Tc = np.eye(4)
        assert lib.kf_raycast(h1, 8, 8, C.c_void_p(Kc.ctypes.data), C.c_void_p(Tc.ctypes.data),
                              0.01, C.c_void_p(0x4000), None, None, None, None) == L.KF_E_SHAPE
    finally:
        lib.kf_volume_destroy(h1)


def test_texture_layout_matches_oracle(oracle):
    """kf_texture_layout is host logic: its rects and atlas width equal the oracle's, bit
    for bit, for the kinect mesh in several atlas heights and for a ragged random set."""
    from kf_synth import configs
    from paper_1602_06645_amd import texture_layout
    tri, size_pixel = configs.kinect_triangles(n_tri=2048)
    rng = np.random.default_rng(41)
    rnd = (rng.uniform(-0.5, 0.5, (500, 1, 3)) + rng.uniform(-0.05, 0.05, (500, 3, 3)))
    for t, sp, H in ((tri, size_pixel, 4096), (tri, size_pixel, 700), (tri, 2 * size_pixel, 333),
                     (rnd.astype(np.float32), 0.0013, 200)):
        rects, W = texture_layout(t, sp, H)
        orects, oW = oracle.texture_layout(t, sp, H)
        assert W == oW and np.array_equal(rects, orects)
        assert len(np.unique(rects[:, 0])) > 1


def test_texture_rejects_bad_arguments():
    lib = L.load()
    tri = np.zeros((1, 3, 3), np.float32)
    tri[0, 1, 0] = 1.0
    rects = np.zeros((1, 4), np.int32)
    W = C.c_int32(0)

    def lay(n=1, sp=0.01, H=200, t=tri):
        return lib.kf_texture_layout(n, t.ctypes.data, sp, H, rects.ctypes.data, C.byref(W))
    assert lay() == L.KF_OK and W.value == 100 and list(rects[0]) == [0, 0, 100, 2]
    assert lay(n=-1) == L.KF_E_ARG
    assert lay(sp=0.0) == L.KF_E_ARG and lay(sp=float("inf")) == L.KF_E_ARG
    assert lay(H=1) == L.KF_E_SHAPE
    assert lay(H=100, t=tri[:, [0, 2, 1]].copy()) == L.KF_OK          # 100 rows fit exactly
    assert lay(H=99, t=tri[:, [0, 2, 1]].copy()) == L.KF_E_RANGE      # one row too many
    assert lay(sp=1e-5) == L.KF_E_RANGE                               # 100000 columns
    assert lib.kf_texture_layout(0, None, 0.01, 16, None, C.byref(W)) == L.KF_OK and W.value == 0
    assert lib.kf_texture_layout(1, None, 0.01, 16, None, C.byref(W)) == L.KF_E_ARG
    h = _volume()
    p = C.c_void_p(0x4000)
    try:
        gen = lib.kf_texture_generate
        assert gen(h, 1, p, p, 8, 8, None, None, None) == L.KF_E_ARG    # no output
        assert gen(h, -1, p, p, 8, 8, p, None, None) == L.KF_E_ARG
        assert gen(h, 1, None, p, 8, 8, p, None, None) == L.KF_E_ARG
        assert gen(h, 1, p, p, -8, 8, p, None, None) == L.KF_E_SHAPE
        assert gen(None, 1, p, p, 8, 8, p, None, None) == L.KF_E_ARG
    finally:
        lib.kf_volume_destroy(h)
    d = _desc()
    d.colour_dim[0] = 1
    bufs = L.VolumeBuffers(*([0x1000] * 6))
    h1 = C.c_void_p()
    assert lib.kf_volume_create(C.byref(d), C.byref(bufs), C.byref(h1)) == L.KF_OK
    try:
        assert lib.kf_texture_generate(h1, 1, p, p, 8, 8, p, None, None) == L.KF_E_SHAPE
    finally:
        lib.kf_volume_destroy(h1)


def test_hd_sampling_is_validated():
    lib = L.load()
    out = (C.c_size_t * 6)()
    for mode, code in ((L.KF_HD_BILINEAR, L.KF_OK), (L.KF_HD_NEAREST, L.KF_OK), (2, L.KF_E_ARG),
                       (-1, L.KF_E_ARG)):
        d = _desc()
        d.hd_sampling = mode
        assert lib.kf_volume_buffer_bytes(C.byref(d), out) == code
    # the adjoint is defined for bilinear sampling only
    d = _desc()
    d.hd_sampling = L.KF_HD_NEAREST
    args = [C.byref(d), None, 1, C.c_void_p(0x1), C.c_void_p(0x1), 640, 480, 1920, 1080,
            None, None, None, None, C.c_void_p(0x1), C.c_void_p(0x1), C.c_void_p(0x1), None, None]
    assert lib.kf_integrate_backward(*args) == L.KF_E_UNSUPPORTED


def test_mesh_rejects_bad_arguments():
    lib = L.load()
    counts = np.zeros(2, np.int64)
    cp = counts.ctypes.data_as(C.c_void_p)
    p = C.c_void_p(0x4000)
    assert lib.kf_mesh_extract(None, None, 0, None, 0, cp, None) == L.KF_E_ARG
    h = _volume()
    try:
        assert lib.kf_mesh_extract(h, None, 0, None, 0, None, None) == L.KF_E_ARG
        assert lib.kf_mesh_extract(h, p, -1, p, 4, cp, None) == L.KF_E_ARG
        assert lib.kf_mesh_extract(h, p, 4, None, 0, cp, None) == L.KF_E_ARG     # one output
    finally:
        lib.kf_volume_destroy(h)
    bufs = L.VolumeBuffers(*([0x1000] * 6))
    for dims, code in (((1, 16, 16), L.KF_OK), ((1024, 1024, 512), L.KF_E_RANGE)):
        d = _desc()
        d.geom_dim[0], d.geom_dim[1], d.geom_dim[2] = dims
        h1 = C.c_void_p()
        assert lib.kf_volume_create(C.byref(d), C.byref(bufs), C.byref(h1)) == L.KF_OK
        try:
            counts[:] = 7
            # a volume without cubes has an empty mesh (no device work); one of 2^29 voxels
            # would overflow the 32-bit counts
            assert lib.kf_mesh_extract(h1, None, 0, None, 0, cp, None) == code
            assert (counts == 0).all()
        finally:
            lib.kf_volume_destroy(h1)


def test_backward_rejects_bad_arguments():
    lib = L.load()
    d = _desc()
    args = [C.byref(d), None, 65, C.c_void_p(0x1), C.c_void_p(0x1), 640, 480, 1920, 1080,
            None, None, None, None, C.c_void_p(0x1), C.c_void_p(0x1), C.c_void_p(0x1), None, None]
    assert lib.kf_integrate_backward(*args) == L.KF_E_ARG     # K_d is NULL (65 frames: chunked)
    args[2] = 4
    assert lib.kf_integrate_backward(*args) == L.KF_E_ARG     # K_d is NULL
    args[2] = -1
    assert lib.kf_integrate_backward(*args) == L.KF_E_ARG


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        L.load()


@pytest.mark.parametrize("shape", [(2, 24, 32, 1), (2, 24, 32, 4), (2, 3, 24, 32), (2, 24, 32)])
def test_binding_rejects_rgb_without_three_interleaved_channels(shape):
    """The kernels read 3 interleaved channels per HD pixel: any other layout (1 or 4
    channels, channel-first, a missing channel axis) is refused by the binding before a
    pointer reaches the library."""
    import torch
    from paper_1602_06645_amd import api
    depth = torch.zeros((2, 12, 16), dtype=torch.float32)
    rgb = torch.zeros(shape, dtype=torch.uint8)
    eye = np.eye(3)
    with pytest.raises(ValueError, match="3 interleaved channels"):
        api.Scan(depth, rgb, eye, eye, np.eye(4), np.stack([np.eye(4)] * 2), 0.01, 64)
    with pytest.raises(ValueError, match="3 interleaved channels"):
        api._rgb(rgb[0], 3)
    # the right layout gets past the shape check (and then needs a device tensor)
    with pytest.raises(ValueError, match="CUDA/HIP tensor"):
        api.Scan(depth, torch.zeros((2, 24, 32, 3), dtype=torch.uint8), eye, eye, np.eye(4),
                 np.stack([np.eye(4)] * 2), 0.01, 64)


def test_se3_helpers_against_expm_and_differences():
    """kf_se3_compose equals scipy's matrix exponential of the twist times T; kf_se3_pullback
    maps the gradient for a left perturbation at exp(xi^) T to the gradient in xi, checked
    by central differences of a linear function of the composed transform."""
    from scipy.linalg import expm
    from paper_1602_06645_amd.autograd import se3_exp_times, se3_pullback

    def twist(x):
        M = np.zeros((4, 4))
        M[:3, :3] = [[0, -x[5], x[4]], [x[5], 0, -x[3]], [-x[4], x[3], 0]]
        M[:3, 3] = x[:3]
        return M
    rng = np.random.default_rng(7)
    T = expm(twist(rng.normal(size=6)))
    W = rng.normal(size=(4, 4))
    f = lambda M: float((W * M).sum())                      # noqa: E731
    for scale in (1e-3, 0.3, 2.0):
        xi = rng.normal(size=6) * scale
        np.testing.assert_allclose(se3_exp_times(xi, T), expm(twist(xi)) @ T, atol=1e-12)
        base = expm(twist(xi)) @ T
        h = 1e-6
        d_eps = np.array([(f(expm(twist(h * e)) @ base) - f(expm(twist(-h * e)) @ base)) / (2 * h)
                          for e in np.eye(6)])
        d_xi = np.array([(f(expm(twist(xi + h * e)) @ T) - f(expm(twist(xi - h * e)) @ T)) / (2 * h)
                         for e in np.eye(6)])
        np.testing.assert_allclose(se3_pullback(xi, d_eps), d_xi, rtol=1e-6, atol=1e-6)
    lib = L.load()
    bad = np.array([0, 0, 0, 20.0, 0, 0])
    out = np.zeros(16)
    assert lib.kf_se3_compose(bad.ctypes.data, np.eye(4).ctypes.data, out.ctypes.data) == L.KF_E_ARG
    assert lib.kf_se3_compose(np.zeros(6).ctypes.data, np.diag([1.0, 1, 2, 1]).ctypes.data,
                              out.ctypes.data) == L.KF_E_ARG
