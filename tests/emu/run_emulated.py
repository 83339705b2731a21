"""Driver run in a child process (with the sanitizer runtime preloaded): integrates and
differentiates seeded scans through the emulated C ABI with host buffers and prints one
JSON line comparing every output with the oracle."""
import ctypes as C
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.abspath(os.path.join(HERE, "..", ".."))
sys.path.insert(0, ROOT)
from paper_1602_06645_amd import _lib as L          # noqa: E402
from paper_1602_06645_amd.api import volume_desc    # noqa: E402
from kf_synth import configs                        # noqa: E402
from oracle import oracle as O                      # noqa: E402

lib = C.CDLL(sys.argv[1])
for name, (res, args) in L.SIGNATURES.items():
    fn = getattr(lib, name)
    fn.restype = res
    fn.argtypes = args


def check(st):
    if st != 0:
        raise RuntimeError(f"status {st}: {lib.kf_last_error().decode()}")


class Vol:
    def __init__(self, spec):
        ng, nc = int(np.prod(spec.gdim)), int(np.prod(spec.cdim))
        self.arrs = [np.zeros(ng, np.float32) for _ in range(2)] + \
                    [np.zeros(nc, np.float32) for _ in range(4)]
        bufs = L.VolumeBuffers(*[a.ctypes.data for a in self.arrs])
        self.desc = volume_desc(spec)
        self.h = C.c_void_p()
        check(lib.kf_volume_create(C.byref(self.desc), C.byref(bufs), C.byref(self.h)))


def scene(vol, fr, keep):
    s = L.Scene()
    d = np.ascontiguousarray(fr.depth, np.float32)
    rgb = np.ascontiguousarray(fr.rgb)
    mats = [np.ascontiguousarray(m, np.float64)
            for m in (fr.K_d, fr.K_rgb, fr.T_rgb_from_d, fr.T_world_from_cam)]
    keep += [d, rgb] + mats
    s.vol, s.n_frames = vol.h.value, d.shape[0]
    s.depth, s.rgb = d.ctypes.data, rgb.ctypes.data
    s.fmt = L.KF_RGB8 if rgb.dtype == np.uint8 else L.KF_RGBF32
    s.dh, s.dw, s.ch, s.cw = d.shape[1], d.shape[2], rgb.shape[1], rgb.shape[2]
    s.K_d, s.K_rgb, s.T_rgb_from_d, s.T_world_from_cam = [m.ctypes.data for m in mats]
    s.trunc_m, s.w_max = float(fr.trunc), float(fr.w_max)
    return s


def forward_case(pairs, K, specs=None, noalloc=False, bricks=None):
    keep = []
    arr = (L.Scene * len(pairs))(*[scene(v, f, keep) for v, f in pairs])
    if noalloc:
        check(lib.kf_integrate_batch_noalloc(arr, len(pairs), K, None))
    elif bricks is not None:
        b = L.Bricks()
        b.geom[:], b.colour[:] = bricks
        check(lib.kf_integrate_batch_bricks(arr, len(pairs), K, 0, C.byref(b), None))
    else:
        check(lib.kf_integrate_batch(arr, len(pairs), K, 0, None))
    worst = 0
    for (v, fr), spec in zip(pairs, specs or SPECS):
        st = O.State(spec, np.float32)
        O.integrate(spec, fr, st)
        for a, b in zip(v.arrs, st.arrays()):
            worst += int(np.count_nonzero(a.view(np.uint32) != b.astype(np.float32).view(np.uint32)))
    return worst


def backward_case(spec, fr, pose=False):
    fr = fr.as_float_rgb()
    d = np.ascontiguousarray(fr.depth, np.float32)
    rgb = np.ascontiguousarray(fr.rgb, np.float32)
    mats = [np.ascontiguousarray(m, np.float64)
            for m in (fr.K_d, fr.K_rgb, fr.T_rgb_from_d, fr.T_world_from_cam)]
    g = configs.gradient_weights(spec.n_colour).numpy()
    d_rgb = np.empty_like(rgb)
    d_xi = np.empty(6, np.float64)
    d_pose = np.full((d.shape[0], 6), np.nan)
    desc = volume_desc(spec)
    check(lib.kf_integrate_backward(
        C.byref(desc), None, d.shape[0], d.ctypes.data, rgb.ctypes.data, d.shape[2],
        d.shape[1], rgb.shape[2], rgb.shape[1], *[m.ctypes.data for m in mats], g.ctypes.data,
        d_rgb.ctypes.data, d_xi.ctypes.data, d_pose.ctypes.data if pose else None, None))
    want_rgb, want_xi, want_pose = O.backward(spec, fr, g.astype(np.float64), decide_f32=True,
                                              pose=True)
    def rel(got, want):
        floor = 1e-3 * np.abs(want).max()
        return float((np.abs(got - want) / (1e-3 * np.abs(want) + floor)).max())
    out = {"rgb": rel(d_rgb, want_rgb), "xi": rel(d_xi, want_xi)}
    if pose:
        out["pose"] = rel(d_pose, want_pose)
    return out


def status_case(spec, fr):
    """kf_debug_status of every frame, each against the state after the frames before it,
    equals the oracle's outcome codes."""
    v = Vol(spec)
    st = O.State(spec, np.float32)
    keep = []
    bad = 0
    for f in range(fr.n):
        one = fr.select(f)
        d = np.ascontiguousarray(one.depth[0], np.float32)
        rgb = np.ascontiguousarray(one.rgb[0])
        mats = [np.ascontiguousarray(m, np.float64)
                for m in (fr.K_d, fr.K_rgb, fr.T_rgb_from_d, one.T_world_from_cam[0])]
        gs = np.empty(v.arrs[0].size, np.uint8)
        cs = np.empty(v.arrs[2].size, np.uint8)
        check(lib.kf_debug_status(v.h, d.ctypes.data, d.shape[1], d.shape[0], rgb.ctypes.data,
                                  L.KF_RGB8 if rgb.dtype == np.uint8 else L.KF_RGBF32,
                                  rgb.shape[1], rgb.shape[0], *[m.ctypes.data for m in mats],
                                  float(fr.trunc), float(fr.w_max), gs.ctypes.data,
                                  cs.ctypes.data, None))
        ogs, ocs = O.status(spec, fr, st, f)
        bad += int(np.count_nonzero(gs != np.asarray(ogs).ravel()))
        bad += int(np.count_nonzero(cs != np.asarray(ocs).ravel()))
        arr = (L.Scene * 1)(scene(v, one, keep))
        check(lib.kf_integrate_batch(arr, 1, 1, 0, None))
        O.integrate(spec, one, st)
    return bad


def raycast_case(spec, fr):
    """kf_raycast on the oracle's own integration of the scan equals the oracle's ray cast
    bit for bit (every output), from an in-scan camera and an off-scan one."""
    st = O.State(spec, np.float32)
    O.integrate(spec, fr, st)
    v = Vol(spec)
    for a, b in zip(v.arrs, st.arrays()):
        a[:] = b
    K = np.array([[131.25, 0, 79.5], [0, 131.25, 59.5], [0, 0, 1.0]])
    bad = 0
    cams = (fr.T_world_from_cam[2], fr.T_world_from_cam[0] @ np.diag([1.0, -1.0, -1.0, 1.0]))
    for ci, T in enumerate(cams):
        T = np.ascontiguousarray(T, np.float64)
        W, H = 160, 120
        outs = {n: np.zeros((H, W, 3) if n != "depth" else (H, W), np.float32)
                for n in ("depth", "vertex", "normal", "colour")}
        check(lib.kf_raycast(v.h, W, H, K.ctypes.data, T.ctypes.data, 0.012,
                             outs["depth"].ctypes.data, outs["vertex"].ctypes.data,
                             outs["normal"].ctypes.data, outs["colour"].ctypes.data, None))
        want = O.raycast(spec, st, K, T, W, H, 0.012)
        for n in outs:
            bad += int(np.count_nonzero(outs[n].view(np.uint32) != want[n].view(np.uint32)))
        if ci == 0 and np.count_nonzero(want["depth"]) < 1000:
            bad += 1   # the in-scan camera must see the surface
    return bad


def texture_case(spec, fr):
    """kf_texture_layout equals the oracle's layout, and kf_texture_generate on the oracle's
    own integration of the scan equals the oracle's texels bit for bit (float and bytes),
    for surface triangles plus triangles leaving the volume and degenerate ones; texels
    outside the maps and the maps of rects outside the atlas stay untouched."""
    st = O.State(spec, np.float32)
    O.integrate(spec, fr, st)
    v = Vol(spec)
    for a, b in zip(v.arrs, st.arrays()):
        a[:] = b
    tri, size_pixel = configs.tiny_triangles()
    rng = np.random.default_rng(22)
    extra = rng.uniform(-0.6, 0.6, (12, 1, 3)) + rng.uniform(-0.1, 0.1, (12, 3, 3))
    extra = extra.astype(np.float32)                                   # partly outside
    extra[0, 1] = extra[0, 0]                                          # V1 = V2
    extra[1, 1:] = extra[1, 0]                                         # a point
    tri = np.ascontiguousarray(np.concatenate([tri, extra]), np.float32)
    H = 128
    bad = 0
    rects = np.zeros((len(tri), 4), np.int32)
    width = C.c_int32(0)
    check(lib.kf_texture_layout(len(tri), tri.ctypes.data, size_pixel, H, rects.ctypes.data,
                                C.byref(width)))
    orects, owidth = O.texture_layout(tri, size_pixel, H)
    bad += int(np.count_nonzero(rects != orects)) + int(width.value != owidth)
    W = width.value
    rects_bad = rects.copy()
    rects_bad[3, 0] = W - 1                       # leaves the atlas: skipped
    rects_bad[5, 2] = 1                           # narrower than 2: skipped
    atlas = np.full((H, W, 3), -7.0, np.float32)
    atlas8 = np.full((H, W, 3), 77, np.uint8)
    check(lib.kf_texture_generate(v.h, len(tri), tri.ctypes.data, rects_bad.ctypes.data, W, H,
                                  atlas.ctypes.data, atlas8.ctypes.data, None))
    keep = np.ones(len(tri), bool)
    keep[[3, 5]] = False
    want = np.full((H, W, 3), -7.0, np.float32)
    want8 = np.full((H, W, 3), 77, np.uint8)
    O.texture(spec, st, tri[keep], orects[keep], W, H, atlas=want, atlas8=want8)
    bad += int(np.count_nonzero(atlas.view(np.uint32) != want.view(np.uint32)))
    bad += int(np.count_nonzero(atlas8 != want8))
    if np.count_nonzero(want[want != -7.0]) < 20000:
        bad += 1                                  # most surface texels must be coloured
    return bad


def mesh_case(spec, fr, spec_rand):
    """kf_mesh_extract equals the oracle's marching cubes bit for bit (vertex positions,
    triangle indices, order) on the oracle's integration of the scan and on a random sign
    field with unobserved voxels over an odd-sized volume; capacity handling."""
    bad = 0
    st = O.State(spec, np.float32)
    O.integrate(spec, fr, st)
    rng = np.random.default_rng(23)
    n = int(np.prod(spec_rand.gdim))
    F = rng.uniform(-1, 1, n).astype(np.float32)
    F[rng.uniform(size=n) < 0.01] = 0.0
    W = np.where(rng.uniform(size=n) < 0.03, 0.0, 1.0).astype(np.float32)
    for sp, tsdf, wg in ((spec, st.tsdf, st.wg), (spec_rand, F, W)):
        v = Vol(sp)
        v.arrs[0][:] = tsdf
        v.arrs[1][:] = wg
        counts = np.zeros(2, np.int64)
        check(lib.kf_mesh_extract(v.h, None, 0, None, 0, counts.ctypes.data, None))
        nv, nt = int(counts[0]), int(counts[1])
        verts = np.full((nv + 1, 3), -9.0, np.float32)
        tris = np.full((nt + 1, 3), -9, np.int32)
        if nt > 0 and lib.kf_mesh_extract(v.h, verts.ctypes.data, nv, tris.ctypes.data, nt - 1,
                                          counts.ctypes.data, None) != L.KF_E_RANGE:
            bad += 1                                    # too small: refused
        check(lib.kf_mesh_extract(v.h, verts.ctypes.data, nv, tris.ctypes.data, nt,
                                  counts.ctypes.data, None))
        ov, ot = O.marching_cubes(sp, tsdf, wg, "f32")
        if (nv, nt) != (len(ov), len(ot)):
            bad += 1_000_000
            continue
        bad += int(np.count_nonzero(verts[:nv].view(np.uint32) != ov.view(np.uint32)))
        bad += int(np.count_nonzero(tris[:nt] != ot))
        bad += int((verts[nv] != -9.0).any()) + int((tris[nt] != -9).any())   # nothing beyond
        if nt < 1000:
            bad += 1                                    # the case must make a real mesh
    return bad


import time
T0 = time.time()
def tick(msg):
    print(f"{time.time() - T0:7.1f} s {msg}", file=sys.stderr, flush=True)
out = {}
spec6, fr6 = configs.tiny(n_frames=6)
fr6 = fr6.numpy()
spec32, fr32 = configs.tiny(n_frames=32)
fr32 = fr32.numpy()
# a third volume with partial bricks and culling chunks on every axis (geometry bricks
# 16x4x8, colour 8x8x8, chunks of 4^3 bricks), over a box that cuts the scene off-centre
from kf_synth.scenes import VolumeSpec  # noqa: E402
spec_odd = VolumeSpec((45, 37, 29), (135, 111, 87), (-0.41, -0.37, -0.46), (0.9, 0.74, 0.58))
SPECS = [spec6, spec32, spec_odd]
tick("inputs")
out["forward_mismatches"] = forward_case([(Vol(spec6), fr6), (Vol(spec32), fr32.as_float_rgb()),
                                          (Vol(spec_odd), fr32)], 8)
tick("forward")
# passes of more than 32 frames (64-bit frame masks, one wave per brick in the culling):
# 40 frames at 36 per pass (a wide pass, then a narrow one) beside the 6-frame scan
spec40, fr40 = configs.tiny(n_frames=40)
fr40 = fr40.numpy()
out["wide_pass_mismatches"] = forward_case([(Vol(spec6), fr6), (Vol(spec40), fr40)], 36,
                                           [spec6, spec40])
tick("wide passes")
# the allocation-free entry point (workspace in the library's fixed array): the three-scan
# batch, then a smaller one reusing the array
out["noalloc_mismatches"] = (
    forward_case([(Vol(spec6), fr6), (Vol(spec32), fr32.as_float_rgb()), (Vol(spec_odd), fr32)], 8,
                 noalloc=True)
    + forward_case([(Vol(spec6), fr6)], 4, [spec6], noalloc=True))
tick("no-alloc")
# every compiled brick shape (paired by list position) on the odd-sized volume and the
# 6-frame scan: partial bricks on every axis, bit for bit with the oracle
n = C.c_int32(0)
shapes = []
for kind in (0, 1):
    check(lib.kf_brick_shapes(kind, None, 0, C.byref(n)))
    buf = np.zeros((n.value, 3), np.int32)
    check(lib.kf_brick_shapes(kind, buf.ctypes.data, n.value, C.byref(n)))
    shapes.append([tuple(int(x) for x in r) for r in buf])
out["shape_mismatches"] = 0
for q in range(1, max(len(shapes[0]), len(shapes[1]))):
    pair = (shapes[0][min(q, len(shapes[0]) - 1)], shapes[1][min(q, len(shapes[1]) - 1)])
    out["shape_mismatches"] += forward_case([(Vol(spec6), fr6), (Vol(spec_odd), fr32)], 8,
                                            [spec6, spec_odd], bricks=pair)
tick("brick shapes")
out["status_mismatches"] = status_case(spec6, fr6)
tick("status")
# nearest-pixel HD sampling: an 8-bit scan and a float one on the odd volume
import dataclasses  # noqa: E402
near6, near_odd = (dataclasses.replace(s_, hd_sampling="nearest") for s_ in (spec6, spec_odd))
out["nearest_mismatches"] = forward_case([(Vol(near6), fr6), (Vol(near_odd), fr32.as_float_rgb())], 8,
                                         [near6, near_odd])
out["nearest_status_mismatches"] = status_case(near6, fr6)
tick("nearest")
out["raycast_mismatches"] = raycast_case(spec6, fr6)
tick("raycast")
out["texture_mismatches"] = texture_case(spec6, fr6)
tick("texture")
out["mesh_mismatches"] = mesh_case(spec6, fr6, spec_odd)
tick("mesh")
# quadric-error decimation (host code of the library) of the oracle's marching-cubes mesh
# of the 6-frame scan, against the oracle's decimation, bit for bit
st = O.State(spec6, np.float32)
O.integrate(spec6, fr6, st)
V, T = O.marching_cubes(spec6, st.tsdf, st.wg, "f32")
out["decimate_mismatches"] = 0
for rate in (0.3, 0.05):
    ov = np.zeros_like(V)
    ot = np.zeros_like(T)
    nv, nt = C.c_int64(), C.c_int64()
    check(lib.kf_mesh_decimate(V.ctypes.data, len(V), T.ctypes.data, len(T), rate, ov.ctypes.data,
                               C.byref(nv), ot.ctypes.data, C.byref(nt)))
    wv, wt = O.decimate(V, T, rate)
    if (nv.value, nt.value) != (len(wv), len(wt)):
        out["decimate_mismatches"] += 1_000_000
    else:
        out["decimate_mismatches"] += int(np.count_nonzero(ov[:nv.value].view(np.uint32) != wv.view(np.uint32)))
        out["decimate_mismatches"] += int(np.count_nonzero(ot[:nt.value] != wt))
tick("decimation")
out["backward_6"] = backward_case(spec6, fr6, pose=True)
tick("backward 6")
out["backward_32"] = backward_case(spec32, fr32)
out["backward_odd"] = backward_case(spec_odd, fr6, pose=True)
tick("backward 32")
# the image gradient scattered with atomics for every update (no record buffer), and with a
# record buffer too small for the 32-frame scan (bricks past its end scatter directly)
for case, cap in (("backward_direct", "0"), ("backward_overflow", "3000")):
    os.environ["KF_BWD_RECORDS"] = cap
    try:
        out[case] = backward_case(spec32, fr32, pose=True)
    finally:
        del os.environ["KF_BWD_RECORDS"]
tick("backward direct / overflow")
# scans longer than one adjoint call: chunks of 12 (3 chunks of the 32-frame scan) and of 2
# (3 chunks of the 6-frame scan, every chunk after the first starting from stored weights)
for case, chunk, sp, f in (("backward_chunked", "12", spec32, fr32), ("backward_chunked_6", "2", spec6, fr6)):
    os.environ["KF_BWD_CHUNK"] = chunk
    try:
        out[case] = backward_case(sp, f, pose=True)
    finally:
        del os.environ["KF_BWD_CHUNK"]
tick("backward chunked")
print("JSON:" + json.dumps(out), flush=True)
