"""Python face of libkfvol: torch tensors in, C ABI calls out.

Every step of the integration runs in the HIP library; this module only checks tensor
devices, dtypes and shapes, turns matrices into float64 host arrays, and passes pointers
and torch's current HIP stream to the C functions of include/kf.h.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _mat(a, shape) -> np.ndarray:
    m = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if m.shape != shape:
        raise ValueError(f"expected a matrix of shape {shape}, got {m.shape}")
    return m


def _ptr(a: np.ndarray) -> C.c_void_p:
    return C.c_void_p(a.ctypes.data)


def _dev(t: torch.Tensor, dtype, name: str, ndim: int | None = None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA/HIP tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _rgb(rgb, ndim: int, name: str = "rgb") -> torch.Tensor:
    """An HD image (ndim 3: [CH,CW,3]) or a stack of them (ndim 4: [n,CH,CW,3]): three
    interleaved channels per pixel, checked before the device so that no other layout
    (one or four channels, channel-first) ever reaches a kernel."""
    if not isinstance(rgb, torch.Tensor):
        raise ValueError(f"{name} must be a tensor")
    if rgb.dim() != ndim or rgb.shape[-1] != 3:
        want = "[CH,CW,3]" if ndim == 3 else "[n,CH,CW,3]"
        raise ValueError(f"{name} must be {want} with 3 interleaved channels, got shape "
                         f"{tuple(rgb.shape)}")
    _rgb_fmt(rgb)
    return _dev(rgb, rgb.dtype, name, ndim)


def _rgb_fmt(rgb: torch.Tensor) -> int:
    if rgb.dtype == torch.uint8:
        return L.KF_RGB8
    if rgb.dtype == torch.float32:
        return L.KF_RGBF32
    raise ValueError("rgb must be uint8 or float32")


def volume_desc(spec) -> L.VolumeDesc:
    d = L.VolumeDesc()
    d.geom_dim[:] = [int(x) for x in spec.gdim]
    d.colour_dim[:] = [int(x) for x in spec.cdim]
    d.origin[:] = [float(x) for x in spec.origin]
    d.extent[:] = [float(x) for x in spec.extent]
    d.colour_band = float(spec.sigma)
    d.colour_gate = float(spec.gate)
    mode = getattr(spec, "hd_sampling", "bilinear")
    if mode not in ("bilinear", "nearest"):
        raise ValueError(f"unknown HD sampling {mode!r}")
    d.hd_sampling = L.KF_HD_NEAREST if mode == "nearest" else L.KF_HD_BILINEAR
    return d


class Volume:
    """A geometry volume and its asymmetric colour volume in six float32 device arrays
    (tsdf, w_geom over geom_dim; r, g, b, w_col over colour_dim; x fastest), all zero."""

    def __init__(self, spec, device="cuda"):
        self.spec = spec
        dev = torch.device(device)
        ng = int(np.prod(spec.gdim))
        nc = int(np.prod(spec.cdim))
        z = lambda n: torch.zeros(n, dtype=torch.float32, device=dev)
        self.tsdf, self.w_geom = z(ng), z(ng)
        self.r, self.g, self.b, self.w_col = z(nc), z(nc), z(nc), z(nc)
        self._desc = volume_desc(spec)
        bufs = L.VolumeBuffers(*[t.data_ptr() for t in self.arrays()])
        h = C.c_void_p()
        L.check(L.load().kf_volume_create(C.byref(self._desc), C.byref(bufs), C.byref(h)))
        self._h = h

    def arrays(self):
        return [self.tsdf, self.w_geom, self.r, self.g, self.b, self.w_col]

    @property
    def handle(self) -> C.c_void_p:
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                L.load().kf_volume_destroy(h)
            except Exception:
                pass
            self._h = None

    def reset(self) -> None:
        L.check(L.load().kf_volume_reset(self._h, _stream()))

    def integrate(self, depth, rgb, K_d, K_rgb, T_rgb_from_d, T_world_from_cam,
                  trunc: float, w_max: float) -> None:
        """One frame: depth [H,W] float32 metres, rgb [CH,CW,3] uint8 or float32."""
        rgb = _rgb(rgb, 3)
        depth = _dev(depth, torch.float32, "depth", 2)
        Kd, Kr = _mat(K_d, (3, 3)), _mat(K_rgb, (3, 3))
        Trd, Twc = _mat(T_rgb_from_d, (4, 4)), _mat(T_world_from_cam, (4, 4))
        L.check(L.load().kf_integrate(
            self._h, C.c_void_p(depth.data_ptr()), depth.shape[1], depth.shape[0],
            C.c_void_p(rgb.data_ptr()), _rgb_fmt(rgb), rgb.shape[1], rgb.shape[0],
            _ptr(Kd), _ptr(Kr), _ptr(Trd), _ptr(Twc), float(trunc), float(w_max), _stream()))

    def raycast(self, K, T_world_from_cam, width: int, height: int, step_m: float,
                vertex: bool = True, normal: bool = True, rgb: bool = True) -> dict:
        """Ray cast the volumes from a camera (kf_raycast): float32 device tensors depth
        [H,W] (0 = no surface) and, if asked, vertex, normal and rgb [H,W,3]."""
        dev = self.tsdf.device
        out = {"depth": torch.empty((height, width), dtype=torch.float32, device=dev)}
        for name, want in (("vertex", vertex), ("normal", normal), ("rgb", rgb)):
            if want:
                out[name] = torch.empty((height, width, 3), dtype=torch.float32, device=dev)
        Kc, Tc = _mat(K, (3, 3)), _mat(T_world_from_cam, (4, 4))
        ptr = lambda n: C.c_void_p(out[n].data_ptr()) if n in out else None   # noqa: E731
        L.check(L.load().kf_raycast(self._h, int(width), int(height), _ptr(Kc), _ptr(Tc),
                                    float(step_m), ptr("depth"), ptr("vertex"), ptr("normal"),
                                    ptr("rgb"), _stream()))
        return out

    def texture(self, tri, rects, atlas_width: int, atlas_height: int, rgb: bool = True,
                rgb8: bool = True, out=None) -> dict:
        """Texel colours of every triangle's map (kf_texture_generate).  tri: [n,3,3]
        float32, rects: [n,4] int32 (from texture_layout), both on the volume's device.
        Returns float32 'rgb' and/or uint8 'rgb8' atlases [atlas_height, atlas_width, 3];
        texels outside every map are zero (or keep the values of the tensors in `out`)."""
        dev = self.r.device
        tri = _dev(tri, torch.float32, "tri", 3)
        rects = _dev(rects, torch.int32, "rects", 2)
        if tri.shape[1:] != (3, 3) or rects.shape != (tri.shape[0], 4):
            raise ValueError("tri must be [n,3,3] and rects [n,4]")
        res = dict(out or {})
        shape = (atlas_height, atlas_width, 3)
        for name, want, dt in (("rgb", rgb, torch.float32), ("rgb8", rgb8, torch.uint8)):
            if want and name not in res:
                res[name] = torch.zeros(shape, dtype=dt, device=dev)
            if name in res and (tuple(res[name].shape) != shape or res[name].dtype != dt
                                or not res[name].is_contiguous()):
                raise ValueError(f"{name} must be a contiguous {dt} tensor of shape {shape}")
        ptr = lambda n: C.c_void_p(res[n].data_ptr()) if n in res else None   # noqa: E731
        L.check(L.load().kf_texture_generate(
            self._h, int(tri.shape[0]), C.c_void_p(tri.data_ptr()), C.c_void_p(rects.data_ptr()),
            int(atlas_width), int(atlas_height), ptr("rgb"), ptr("rgb8"), _stream()))
        return res

    def mesh(self, capacity=None) -> tuple:
        """Marching cubes of the geometry volume (kf_mesh_extract): (vertices float32
        [n,3], triangles int32 [m,3]) device tensors.  Without `capacity` the counts are
        queried first; with capacity = (n, m) the outputs are allocated at that size and
        the mesh is extracted in one call (KfError if it does not fit)."""
        dev = self.tsdf.device
        counts = np.zeros(2, np.int64)
        if capacity is None:
            L.check(L.load().kf_mesh_extract(self._h, None, 0, None, 0,
                                             counts.ctypes.data_as(C.c_void_p), _stream()))
            capacity = (int(counts[0]), int(counts[1]))
        verts = torch.empty((max(capacity[0], 1), 3), dtype=torch.float32, device=dev)
        tris = torch.empty((max(capacity[1], 1), 3), dtype=torch.int32, device=dev)
        L.check(L.load().kf_mesh_extract(self._h, C.c_void_p(verts.data_ptr()), int(capacity[0]),
                                         C.c_void_p(tris.data_ptr()), int(capacity[1]),
                                         counts.ctypes.data_as(C.c_void_p), _stream()))
        return verts[:int(counts[0])], tris[:int(counts[1])]

    def status(self, depth, rgb, K_d, K_rgb, T_rgb_from_d, T_world_from_cam, trunc, w_max):
        """Per-voxel outcome codes of one frame (no update): (geometry, colour) uint8."""
        rgb = _rgb(rgb, 3)
        depth = _dev(depth, torch.float32, "depth", 2)
        gs = torch.empty(self.tsdf.numel(), dtype=torch.uint8, device=self.tsdf.device)
        cs = torch.empty(self.r.numel(), dtype=torch.uint8, device=self.r.device)
        Kd, Kr = _mat(K_d, (3, 3)), _mat(K_rgb, (3, 3))
        Trd, Twc = _mat(T_rgb_from_d, (4, 4)), _mat(T_world_from_cam, (4, 4))
        L.check(L.load().kf_debug_status(
            self._h, C.c_void_p(depth.data_ptr()), depth.shape[1], depth.shape[0],
            C.c_void_p(rgb.data_ptr()), _rgb_fmt(rgb), rgb.shape[1], rgb.shape[0],
            _ptr(Kd), _ptr(Kr), _ptr(Trd), _ptr(Twc), float(trunc), float(w_max),
            C.c_void_p(gs.data_ptr()), C.c_void_p(cs.data_ptr()), _stream()))
        return gs, cs


def decimate(vertices, triangles, rate: float):
    """Quadric-error decimation of a triangle mesh (kf_mesh_decimate, host-only): vertices
    [n,3] float32 and triangles [m,3] int32 (numpy arrays or tensors, e.g. Volume.mesh());
    returns numpy (vertices [n',3], triangles [m',3]) with at most round(rate * m)
    triangles."""
    V = np.ascontiguousarray(vertices.cpu().numpy() if isinstance(vertices, torch.Tensor)
                             else vertices, dtype=np.float32).reshape(-1, 3)
    T = np.ascontiguousarray(triangles.cpu().numpy() if isinstance(triangles, torch.Tensor)
                             else triangles, dtype=np.int32).reshape(-1, 3)
    ov = np.zeros((max(len(V), 1), 3), np.float32)
    ot = np.zeros((max(len(T), 1), 3), np.int32)
    nv, nt = C.c_int64(), C.c_int64()
    L.check(L.load().kf_mesh_decimate(V.ctypes.data_as(C.c_void_p), len(V),
                                      T.ctypes.data_as(C.c_void_p), len(T), float(rate),
                                      ov.ctypes.data_as(C.c_void_p), C.byref(nv),
                                      ot.ctypes.data_as(C.c_void_p), C.byref(nt)))
    return ov[:nv.value].copy(), ot[:nt.value].copy()


def texture_layout(tri, size_pixel: float, atlas_height: int):
    """Map sizes and atlas placement (kf_texture_layout, host-only): tri [n,3,3] world
    vertices.  Returns (rects int32 [n,4] = x, y, w, h; the atlas width)."""
    t = np.ascontiguousarray(tri.cpu().numpy() if isinstance(tri, torch.Tensor) else tri,
                             dtype=np.float32).reshape(-1, 3, 3)
    rects = np.zeros((t.shape[0], 4), np.int32)
    width = C.c_int32(0)
    L.check(L.load().kf_texture_layout(int(t.shape[0]), t.ctypes.data_as(C.c_void_p),
                                       float(size_pixel), int(atlas_height),
                                       rects.ctypes.data_as(C.c_void_p), C.byref(width)))
    return rects, int(width.value)


class Scan:
    """n frames for the batch call: depth [n,H,W] float32, rgb [n,CH,CW,3], one pose per
    frame (T_world_from_cam [n,4,4]); K_d, K_rgb 3x3; T_rgb_from_d 4x4."""

    def __init__(self, depth, rgb, K_d, K_rgb, T_rgb_from_d, T_world_from_cam, trunc, w_max):
        self.rgb = _rgb(rgb, 4)
        self.depth = _dev(depth, torch.float32, "depth", 3)
        self.fmt = _rgb_fmt(self.rgb)
        n = self.depth.shape[0]
        if self.rgb.shape[0] != n:
            raise ValueError("depth and rgb hold different numbers of frames")
        self.K_d, self.K_rgb = _mat(K_d, (3, 3)), _mat(K_rgb, (3, 3))
        self.T_rgb_from_d = _mat(T_rgb_from_d, (4, 4))
        self.T_world_from_cam = _mat(T_world_from_cam, (n, 4, 4))
        self.trunc, self.w_max = float(trunc), float(w_max)

    @staticmethod
    def from_frames(fr) -> "Scan":
        return Scan(fr.depth, fr.rgb, fr.K_d, fr.K_rgb, fr.T_rgb_from_d, fr.T_world_from_cam,
                    fr.trunc, fr.w_max)

    def scene(self, vol: Volume) -> L.Scene:
        s = L.Scene()
        s.vol = vol.handle.value
        s.n_frames = self.depth.shape[0]
        s.depth = self.depth.data_ptr()
        s.rgb = self.rgb.data_ptr()
        s.fmt = self.fmt
        s.dh, s.dw = self.depth.shape[1], self.depth.shape[2]
        s.ch, s.cw = self.rgb.shape[1], self.rgb.shape[2]
        s.K_d = self.K_d.ctypes.data
        s.K_rgb = self.K_rgb.ctypes.data
        s.T_rgb_from_d = self.T_rgb_from_d.ctypes.data
        s.T_world_from_cam = self.T_world_from_cam.ctypes.data
        s.trunc_m, s.w_max = self.trunc, self.w_max
        return s


def _scenes(pairs):
    arr = (L.Scene * max(1, len(pairs)))()
    for q, (vol, scan) in enumerate(pairs):
        arr[q] = scan.scene(vol)
    return arr


def brick_shapes() -> dict:
    """The brick shapes (x, y, z voxels) the library's integration kernels are compiled for:
    {"geometry": [...], "colour": [...]}, the default first (kf_brick_shapes)."""
    out = {}
    for kind, name in ((0, "geometry"), (1, "colour")):
        n = C.c_int32(0)
        L.check(L.load().kf_brick_shapes(kind, None, 0, C.byref(n)))
        buf = np.zeros((n.value, 3), np.int32)
        L.check(L.load().kf_brick_shapes(kind, buf.ctypes.data_as(C.c_void_p), n.value, C.byref(n)))
        out[name] = [tuple(int(x) for x in row) for row in buf]
    return out


def _bricks(bricks):
    """kf_bricks from {"geometry": (x, y, z), "colour": (x, y, z)} (either may be left out:
    the default shape), or None for the defaults."""
    if bricks is None:
        return None
    unknown = set(bricks) - {"geometry", "colour"}
    if unknown:
        raise ValueError(f"unknown brick kinds {sorted(unknown)}")
    defaults = brick_shapes()
    b = L.Bricks()
    for field, name in (("geom", "geometry"), ("colour", "colour")):
        shape = tuple(int(x) for x in bricks.get(name, defaults[name][0]))
        if len(shape) != 3:
            raise ValueError(f"{name} brick must be (x, y, z)")
        getattr(b, field)[:] = shape
    return C.byref(b)


def integrate_batch(pairs, frames_per_pass: int = 1, use_graph: bool = False,
                    bricks: dict | None = None) -> None:
    """Integrate [(Volume, Scan), ...]: every scan into its own volume, all together.
    bricks: brick shapes of the work items (brick_shapes(); None: the defaults), which
    change the time, never the result."""
    arr = _scenes(pairs)
    if bricks is None:
        L.check(L.load().kf_integrate_batch(arr, len(pairs), int(frames_per_pass), int(use_graph),
                                            _stream()))
    else:
        L.check(L.load().kf_integrate_batch_bricks(arr, len(pairs), int(frames_per_pass),
                                                   int(use_graph), _bricks(bricks), _stream()))


def release_graphs() -> tuple:
    """Drop every recorded batch graph and its workspace (kf_release_graphs): returns
    (graphs released, workspace bytes freed)."""
    n, b = C.c_int32(0), C.c_size_t(0)
    L.check(L.load().kf_release_graphs(C.byref(n), C.byref(b)))
    return int(n.value), int(b.value)


def integrate_batch_noalloc(pairs, frames_per_pass: int = 1) -> None:
    """integrate_batch through kf_integrate_batch_noalloc: the library allocates nothing
    (its workspace is a fixed 64 MiB device array per GPU, shared by all such calls)."""
    arr = _scenes(pairs)
    L.check(L.load().kf_integrate_batch_noalloc(arr, len(pairs), int(frames_per_pass),
                                                _stream()))


def integrate_batch_timed(pairs, frames_per_pass: int, events, bricks: dict | None = None) -> None:
    """integrate_batch that records each pair (start, end) or triple (start, mid, end) of
    `events` (torch.cuda.Event, enable_timing=True) around the integration launches of
    one pass, in order; mid is recorded between the geometry and the colour launch."""
    for ev in events:             # torch creates the HIP event on first record
        for e in ev:
            e.record()
    n = len(events)
    starts = (C.c_void_p * n)(*[ev[0].cuda_event for ev in events])
    ends = (C.c_void_p * n)(*[ev[-1].cuda_event for ev in events])
    mids = None
    if n and len(events[0]) == 3:
        mids = (C.c_void_p * n)(*[ev[1].cuda_event for ev in events])
    arr = _scenes(pairs)
    L.check(L.load().kf_integrate_batch_timed(arr, len(pairs), int(frames_per_pass),
                                              _bricks(bricks), starts, mids, ends, n, _stream()))


def integrate_batch_counted(pairs, frames_per_pass: int = 1, bricks: dict | None = None) -> np.ndarray:
    """Same as integrate_batch, and return the eight accounting counters (include/kf.h)."""
    arr = _scenes(pairs)
    dev = pairs[0][0].tsdf.device if pairs else torch.device("cuda")
    cnt = torch.zeros(8, dtype=torch.int64, device=dev)
    L.check(L.load().kf_integrate_batch_counted(arr, len(pairs), int(frames_per_pass),
                                                _bricks(bricks), C.c_void_p(cnt.data_ptr()),
                                                _stream()))
    return cnt.cpu().numpy()


def integrate_backward(spec, scan: Scan, grad: torch.Tensor, w_col0: torch.Tensor | None = None,
                       pose: bool = False):
    """dL/dRGB [n,CH,CW,3] float32 and dL/dxi [6] float64 (device) for
    L = sum grad[c][v] C_N(v)_c; scan.rgb must be float32.  pose: also dL/dxi_n [n,6]
    float64 for the depth-camera poses (left perturbations in world coordinates)."""
    if scan.fmt != L.KF_RGBF32:
        raise ValueError("the adjoint takes float32 images")
    nc = int(np.prod(spec.cdim))
    grad = _dev(grad, torch.float32, "grad", 2)
    if tuple(grad.shape) != (3, nc):
        raise ValueError(f"grad must have shape (3, {nc})")
    if w_col0 is not None:
        w_col0 = _dev(w_col0, torch.float32, "w_col0", 1)
        if w_col0.numel() != nc:
            raise ValueError(f"w_col0 must hold {nc} weights")
    n = scan.depth.shape[0]
    d_rgb = torch.empty_like(scan.rgb)
    d_xi = torch.empty(6, dtype=torch.float64, device=scan.rgb.device)
    d_pose = torch.empty((n, 6), dtype=torch.float64, device=scan.rgb.device) if pose else None
    desc = volume_desc(spec)
    L.check(L.load().kf_integrate_backward(
        C.byref(desc), None if w_col0 is None else C.c_void_p(w_col0.data_ptr()), n,
        C.c_void_p(scan.depth.data_ptr()), C.c_void_p(scan.rgb.data_ptr()),
        scan.depth.shape[2], scan.depth.shape[1], scan.rgb.shape[2], scan.rgb.shape[1],
        _ptr(scan.K_d), _ptr(scan.K_rgb), _ptr(scan.T_rgb_from_d), _ptr(scan.T_world_from_cam),
        C.c_void_p(grad.data_ptr()), C.c_void_p(d_rgb.data_ptr()), C.c_void_p(d_xi.data_ptr()),
        None if d_pose is None else C.c_void_p(d_pose.data_ptr()), _stream()))
    return (d_rgb, d_xi, d_pose) if pose else (d_rgb, d_xi)
