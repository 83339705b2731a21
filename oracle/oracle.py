"""ctypes wrapper of the C oracle (kf_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU-baseline
leg use this module to compute the reference results of the volumetric integration of
arXiv 1602.06645 (Sec. III TSDF volume; Sec. IV.B colour volume, Eq. 5-10; Sec. IV.A
depth-to-HD mapping, Eq. 1-4), the ray casting of the two volumes and the per-polygon
texture maps of Sec. IV.D (Eq. 11-14), marching cubes and the quadric-error decimation of
the mesh (Sec. IV.C).  The product library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_LIB_PATH = os.path.join(HERE, "liboracle.so")
# The mutation tests point this at a copy of the oracle built with a planted mistake.
LIB_PATH = os.environ.get("KF_ORACLE_LIB", DEFAULT_LIB_PATH)

ST_FRUSTUM, ST_NODEPTH, ST_BAND, ST_NORMAL, ST_GATE, ST_HD, ST_UPDATED = range(7)


def build(force: bool = True, src_dir: str = HERE, out: str = DEFAULT_LIB_PATH) -> str:
    """Compile liboracle.so with plain IEEE arithmetic (no contraction, no fast-math)."""
    if force or not os.path.exists(out):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-std=c11", "-Wall", "-shared", "-fPIC",
               "-o", out + ".tmp", os.path.join(src_dir, "kf_oracle.c"), "-lm"]
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)
    return out


class _Volume(C.Structure):
    _fields_ = [("gdim", C.c_int32 * 3), ("cdim", C.c_int32 * 3),
                ("origin", C.c_double * 3), ("extent", C.c_double * 3),
                ("sigma", C.c_double), ("gate", C.c_double), ("hd_nearest", C.c_int32)]


class _Frames(C.Structure):
    _fields_ = [("n_frames", C.c_int32), ("dw", C.c_int32), ("dh", C.c_int32),
                ("cw", C.c_int32), ("ch", C.c_int32),
                ("depth", C.c_void_p), ("rgb8", C.c_void_p), ("rgbf", C.c_void_p),
                ("K_d", C.c_void_p), ("K_rgb", C.c_void_p),
                ("T_rgb_from_d", C.c_void_p), ("T_world_from_cam", C.c_void_p),
                ("trunc", C.c_double), ("w_max", C.c_double)]


class _FC64(C.Structure):
    _fields_ = [(n, C.c_double * 9) if n.startswith("A") else
                (n, C.c_double * 3) if n.startswith("b") else (n, C.c_double)
                for n in ["Ag", "bg", "Ac", "bc", "Ah", "bh", "fx", "fy", "cx", "cy",
                          "inv_fx", "inv_fy", "fxr", "fyr", "cxr", "cyr", "trunc",
                          "inv_trunc", "w_max", "sigma2", "gate", "hd_nearest"]]


class _RC64(C.Structure):
    _fields_ = [(n, C.c_double * 3) for n in ["a", "Bu", "Bv", "B0", "ac", "Bcu", "Bcv", "Bc0",
                                               "Ru", "Rv", "R0", "tw", "inv_s", "gmax",
                                               "cmax"]] + [("delta", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False, out=LIB_PATH)
        L = C.CDLL(LIB_PATH)
        p = C.c_void_p
        L.or_frame_consts.argtypes = [C.POINTER(_Volume), C.POINTER(_Frames), C.c_int,
                                      C.POINTER(_FC64)]
        for name in ("or_integrate_f32", "or_integrate_f64"):
            fn = getattr(L, name)
            fn.argtypes = [C.POINTER(_Volume), C.POINTER(_Frames)] + [p] * 6 + \
                [C.c_int] * 6 + [p, p, p]
            fn.restype = None
        L.or_backward_f64.argtypes = [C.POINTER(_Volume), C.POINTER(_Frames), p, p,
                                      C.c_int, C.c_int, C.c_int, p, p, p]
        L.or_backward_f64.restype = None
        for name in ("or_raycast_f32", "or_raycast_f64"):
            fn = getattr(L, name)
            fn.argtypes = [C.POINTER(_Volume)] + [p] * 6 + [p, p, C.c_double, C.c_int, p,
                                                          C.c_int64, p, p, p, p]
            fn.restype = None
        L.or_raycast_consts.argtypes = [C.POINTER(_Volume), p, p, C.c_double,
                                        C.POINTER(_RC64)]
        L.or_raycast_consts.restype = None
        L.or_texture_layout.argtypes = [C.c_int32, p, C.c_double, C.c_int32, p]
        L.or_texture_layout.restype = C.c_int32
        for name in ("or_texture_generate_f32", "or_texture_generate_f64"):
            fn = getattr(L, name)
            fn.argtypes = [C.POINTER(_Volume)] + [p] * 4 + [C.c_int32, p, p, C.c_int32, p, p]
            fn.restype = None
        L.or_marching_cubes.argtypes = [C.POINTER(_Volume), p, p, p, p, C.c_int64, p,
                                        C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.or_marching_cubes.restype = C.c_int
        L.or_mc_cube_triangles.argtypes = [C.c_uint, p]
        L.or_mc_cube_triangles.restype = C.c_int
        L.or_decimate.argtypes = [p, C.c_int64, p, C.c_int64, C.c_double, p, p, p, p]
        L.or_decimate.restype = C.c_int64
        _lib = L
    return _lib


def _vol(vol) -> _Volume:
    v = _Volume()
    v.gdim[:] = [int(a) for a in vol.gdim]
    v.cdim[:] = [int(a) for a in vol.cdim]
    v.origin[:] = [float(a) for a in vol.origin]
    v.extent[:] = [float(a) for a in vol.extent]
    v.sigma = float(vol.sigma)
    v.gate = float(vol.gate)
    v.hd_nearest = 1 if getattr(vol, "hd_sampling", "bilinear") == "nearest" else 0
    return v


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _frames(fr, keep: list) -> _Frames:
    f = _Frames()
    depth = _c(fr.depth, np.float32)
    f.n_frames = depth.shape[0]
    f.dh, f.dw = depth.shape[1], depth.shape[2]
    f.depth = depth.ctypes.data
    keep.append(depth)
    f.rgb8 = f.rgbf = None
    rgb_in = np.asarray(fr.rgb)
    if rgb_in.dtype == np.uint8:
        rgb = _c(rgb_in, np.uint8)
        f.rgb8 = rgb.ctypes.data
    else:
        rgb = _c(rgb_in, np.float32)
        f.rgbf = rgb.ctypes.data
    keep.append(rgb)
    f.ch, f.cw = rgb.shape[1], rgb.shape[2]
    for name in ("K_d", "K_rgb", "T_rgb_from_d", "T_world_from_cam"):
        a = _c(getattr(fr, name), np.float64)
        keep.append(a)
        setattr(f, name, a.ctypes.data)
    f.trunc = float(fr.trunc)
    f.w_max = float(fr.w_max)
    return f


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    L = lib()
    L.or_num_threads.restype = C.c_int
    return int(L.or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops for the following calls."""
    L = lib()
    L.or_set_num_threads.argtypes = [C.c_int]
    L.or_set_num_threads.restype = None
    L.or_set_num_threads(int(n))


def frame_consts(vol, fr, frame: int) -> dict:
    keep: list = []
    out = _FC64()
    lib().or_frame_consts(C.byref(_vol(vol)), C.byref(_frames(fr, keep)), frame, C.byref(out))
    return {n: (np.array(getattr(out, n)) if isinstance(getattr(out, n), C.Array)
                else getattr(out, n)) for n, _ in _FC64._fields_}


class State:
    """Host copy of the six SoA arrays for z-slabs [gz0,gz1) and [cz0,cz1)."""

    def __init__(self, vol, dtype=np.float32, gz=None, cz=None):
        gz = gz or (0, vol.gdim[2])
        cz = cz or (0, vol.cdim[2])
        self.gz, self.cz = (int(gz[0]), int(gz[1])), (int(cz[0]), int(cz[1]))
        ng = vol.gdim[0] * vol.gdim[1] * (self.gz[1] - self.gz[0])
        nc = vol.cdim[0] * vol.cdim[1] * (self.cz[1] - self.cz[0])
        self.tsdf = np.zeros(ng, dtype)
        self.wg = np.zeros(ng, dtype)
        self.r = np.zeros(nc, dtype)
        self.g = np.zeros(nc, dtype)
        self.b = np.zeros(nc, dtype)
        self.wc = np.zeros(nc, dtype)

    @property
    def dtype(self):
        return self.tsdf.dtype

    def arrays(self):
        return [self.tsdf, self.wg, self.r, self.g, self.b, self.wc]


def integrate(vol, fr, state: State, frames_per_pass: int = 1, apply: bool = True,
              want_status: bool = False):
    """Apply every frame of `fr` to `state` in order; return counters (and statuses).

    Counters: [geometry updates, geometry voxels touched per pass, colour gate
    evaluations, colour voxels reaching the gate per pass, colour updates, colour voxels
    updated per pass].  Statuses are those of the last frame (OR_ST_* codes).
    """
    keep: list = []
    f = _frames(fr, keep)
    cnt = np.zeros(6, np.int64)
    gst = cst = None
    if want_status:
        gst = np.zeros(state.tsdf.size, np.uint8)
        cst = np.zeros(state.r.size, np.uint8)
    fn = lib().or_integrate_f32 if state.dtype == np.float32 else lib().or_integrate_f64
    fn(C.byref(_vol(vol)), C.byref(f), *[a.ctypes.data for a in state.arrays()],
       state.gz[0], state.gz[1], state.cz[0], state.cz[1], int(frames_per_pass), int(apply),
       None if gst is None else gst.ctypes.data, None if cst is None else cst.ctypes.data,
       cnt.ctypes.data)
    if want_status:
        return cnt, gst, cst
    return cnt


def status(vol, fr, state: State, frame: int):
    """Per-voxel status codes of one frame against the current state (no update)."""
    sub = fr.select(frame)
    _, gst, cst = integrate(vol, sub, state, apply=False, want_status=True)
    return gst, cst


def backward(vol, fr, g: np.ndarray, cz=None, wc0: np.ndarray | None = None,
             decide_f32: bool = False, pose: bool = False):
    """FP64 adjoint: d L / d RGB ([n][ch][cw][3]) and d L / d xi (6) for
    L = sum g[ch][v] C_N(v)_ch over colour slabs cz; g has shape (3, n_slab_voxels).
    decide_f32: take the integer decisions (pixel, masks, gate, bilinear cell) of the
    FP32 forward, as the GPU kernel does; otherwise everything is FP64.  pose: also
    return d L / d xi_n (n, 6) for the depth-camera poses (left perturbations in world
    coordinates, decisions held).  Defined for bilinear HD sampling only."""
    if getattr(vol, "hd_sampling", "bilinear") != "bilinear":
        raise ValueError("the adjoint is defined for bilinear HD sampling")
    keep: list = []
    f = _frames(fr, keep)
    cz = cz or (0, vol.cdim[2])
    g = _c(g, np.float64)
    d_rgb = np.zeros((f.n_frames, f.ch, f.cw, 3), np.float64)
    d_xi = np.zeros(6, np.float64)
    w0 = None if wc0 is None else _c(wc0, np.float64)
    d_pose = np.zeros((f.n_frames, 6), np.float64)
    lib().or_backward_f64(C.byref(_vol(vol)), C.byref(f),
                          None if w0 is None else w0.ctypes.data, g.ctypes.data,
                          int(cz[0]), int(cz[1]), int(decide_f32), d_rgb.ctypes.data,
                          d_xi.ctypes.data, d_pose.ctypes.data if pose else None)
    return (d_rgb, d_xi, d_pose) if pose else (d_rgb, d_xi)


def raycast_consts(vol, K, T_world_from_cam, delta: float) -> dict:
    """The per-camera constants of the ray caster, in double (exposed for tests)."""
    out = _RC64()
    Kc, Tc = _c(K, np.float64), _c(T_world_from_cam, np.float64)
    lib().or_raycast_consts(C.byref(_vol(vol)), Kc.ctypes.data, Tc.ctypes.data, float(delta),
                            C.byref(out))
    return {n: (np.array(getattr(out, n)) if isinstance(getattr(out, n), C.Array)
                else getattr(out, n)) for n, _ in _RC64._fields_}


def raycast(vol, state: State, K, T_world_from_cam, width: int, height: int, delta: float,
            pixels=None, precision: str = "f32") -> dict:
    """Ray cast a camera (intrinsics K, pose T_world_from_cam) through the whole volume
    held by `state` (it must cover every z-slab).  pixels: flat indices y * width + x to
    cast (default: the whole width x height image).  Returns float32 arrays depth [n],
    vertex, normal and colour [n, 3] (zeros where missing); the whole image is returned
    with shape [height, width(, 3)] when pixels is None."""
    if state.gz != (0, vol.gdim[2]) or state.cz != (0, vol.cdim[2]):
        raise ValueError("ray casting needs the whole volume")
    full = pixels is None
    pix = np.arange(width * height, dtype=np.int32) if full else _c(pixels, np.int32)
    n = pix.size
    depth = np.zeros(n, np.float32)
    vertex = np.zeros((n, 3), np.float32)
    normal = np.zeros((n, 3), np.float32)
    colour = np.zeros((n, 3), np.float32)
    arrs = [_c(a, np.float32) for a in state.arrays()]
    Kc, Tc = _c(K, np.float64), _c(T_world_from_cam, np.float64)
    fn = lib().or_raycast_f32 if precision == "f32" else lib().or_raycast_f64
    fn(C.byref(_vol(vol)), *[a.ctypes.data for a in arrs], Kc.ctypes.data, Tc.ctypes.data,
       float(delta), int(width), pix.ctypes.data, int(n), depth.ctypes.data,
       vertex.ctypes.data, normal.ctypes.data, colour.ctypes.data)
    out = {"depth": depth, "vertex": vertex, "normal": normal, "colour": colour}
    if full:
        out = {k: v.reshape((height, width) + v.shape[1:]) for k, v in out.items()}
    return out


def texture_layout(tri, size_pixel: float, atlas_height: int):
    """Texture-map sizes (Eq. 11-12, rounded up, at least 2 x 2) and their column-wise
    placement in an atlas of atlas_height texels (Sec. IV.D merging).  tri: [n, 3, 3]
    world vertices (V1, V2, V3).  Returns (rects int32 [n, 4] = x, y, w, h; atlas width),
    or raises ValueError when a map does not fit."""
    t = _c(tri, np.float32).reshape(-1, 9)
    rects = np.zeros((t.shape[0], 4), np.int32)
    width = lib().or_texture_layout(int(t.shape[0]), t.ctypes.data, float(size_pixel),
                                    int(atlas_height), rects.ctypes.data)
    if width < 0:
        raise ValueError("a texture map is larger than the atlas or 65535 texels")
    return rects, int(width)


def texture(vol, state: State, tri, rects, atlas_width: int, atlas_height: int,
            precision: str = "f32", atlas=None, atlas8=None):
    """Texel colours of every triangle's map (Eq. 13-14 and the colour-volume lookup),
    written at its rect of the atlas.  Returns (atlas float32 [H, W, 3], atlas8 uint8
    [H, W, 3]); texels outside every rect keep the given arrays' values (default zero)."""
    if state.cz != (0, vol.cdim[2]):
        raise ValueError("texture generation needs the whole colour volume")
    t = _c(tri, np.float32).reshape(-1, 9)
    rc = _c(rects, np.int32).reshape(-1, 4)
    if atlas is None:
        atlas = np.zeros((atlas_height, atlas_width, 3), np.float32)
    if atlas8 is None:
        atlas8 = np.zeros((atlas_height, atlas_width, 3), np.uint8)
    assert atlas.shape == (atlas_height, atlas_width, 3) and atlas.dtype == np.float32
    assert atlas8.shape == atlas.shape and atlas8.dtype == np.uint8
    assert atlas.flags.c_contiguous and atlas8.flags.c_contiguous
    r, g, b, wc = [_c(a, np.float32) for a in state.arrays()[2:]]
    fn = lib().or_texture_generate_f32 if precision == "f32" else lib().or_texture_generate_f64
    fn(C.byref(_vol(vol)), r.ctypes.data, g.ctypes.data, b.ctypes.data, wc.ctypes.data,
       int(t.shape[0]), t.ctypes.data, rc.ctypes.data, int(atlas_width),
       atlas.ctypes.data, atlas8.ctypes.data)
    return atlas, atlas8


def marching_cubes(vol, tsdf, wg, precision: str = "f32"):
    """Mesh of the geometry volume (tsdf, wg: flat or [Z,Y,X] float32 arrays).  Returns
    (vertices [nv, 3] float32 (FP32 arithmetic) or float64 (FP64 arithmetic), triangles
    [nt, 3] int32 vertex indices)."""
    f = _c(tsdf, np.float32).ravel()
    w = _c(wg, np.float32).ravel()
    assert f.size == w.size == int(np.prod(vol.gdim))
    nv, nt = C.c_int64(0), C.c_int64(0)
    L = lib()
    L.or_marching_cubes(C.byref(_vol(vol)), f.ctypes.data, w.ctypes.data, None, None, 0, None,
                        0, C.byref(nv), C.byref(nt))
    tris = np.zeros((nt.value, 3), np.int32)
    if precision == "f32":
        verts = np.zeros((nv.value, 3), np.float32)
        args = (verts.ctypes.data, None)
    else:
        verts = np.zeros((nv.value, 3), np.float64)
        args = (None, verts.ctypes.data)
    rc = L.or_marching_cubes(C.byref(_vol(vol)), f.ctypes.data, w.ctypes.data, *args,
                             nv.value, tris.ctypes.data, nt.value, C.byref(nv), C.byref(nt))
    assert rc == 0
    return verts, tris


def mc_cube_triangles(inside_mask: int) -> np.ndarray:
    """Triangles of one cube configuration as cube edge ids [n, 3]."""
    out = np.zeros((12, 3), np.int32)
    n = lib().or_mc_cube_triangles(int(inside_mask), out.ctypes.data)
    return out[:n].copy()


def decimate(vertices, triangles, rate: float):
    """Quadric-error decimation of a triangle mesh to round(rate * triangles) triangles
    (Sec. IV.C; see kf_decimate_body.h): returns (float32 [n][3], int32 [m][3])."""
    V = np.ascontiguousarray(vertices, np.float32).reshape(-1, 3)
    T = np.ascontiguousarray(triangles, np.int32).reshape(-1, 3)
    ov = np.zeros((max(len(V), 1), 3), np.float32)
    ot = np.zeros((max(len(T), 1), 3), np.int32)
    nv, nt = C.c_int64(), C.c_int64()
    r = lib().or_decimate(V.ctypes.data, len(V), T.ctypes.data, len(T), float(rate), ov.ctypes.data,
                          C.byref(nv), ot.ctypes.data, C.byref(nt))
    if r < 0:
        raise ValueError("bad mesh (index out of range or a triangle repeating a vertex)")
    return ov[:nv.value].copy(), ot[:nt.value].copy()
