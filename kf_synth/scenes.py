"""Seeded synthetic RGB-D scans: the inputs of the volumetric integration.

The paper's captures (a lunch bag and a backpack scanned with a Kinect plus a rigidly
attached HD camera, Sec. V) are not available, so every workload is a seeded synthetic
stand-in with the same structure: a Kinect-class depth camera (640x480, noisy, with
holes), an HD RGB camera offset from it by a rigid extrinsic (Sec. IV.A), small objects
on a ground plane inside a cube-shaped volume, and a camera orbiting the objects.

This module only produces inputs (depth maps, RGB images, intrinsics, poses).  It holds
none of the integration arithmetic.  Rendering is an FP64 analytic ray cast written with
torch so it can run on the GPU for the large workloads; random numbers come from numpy's
seeded generator, so the same seed gives the same scan on any device.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

# Depth intrinsics by image size: f, cx, cy (pixel centres at integer coordinates).
DEPTH_INTRINSICS = {
    (640, 480): (525.0, 319.5, 239.5),
    (480, 360): (393.75, 239.5, 179.5),
    (320, 240): (262.5, 159.5, 119.5),
    (160, 120): (131.25, 79.5, 59.5),
}
RGB_INTRINSICS = {
    (1920, 1080): (1050.0, 959.5, 539.5),
    (1280, 720): (700.0, 639.5, 359.5),
    (960, 540): (525.0, 479.5, 269.5),
    (320, 240): (262.5, 159.5, 119.5),
}
MAX_RANGE = 3.0          # depth beyond this is reported as a hole (0)
BACKGROUND = 128         # RGB value where a ray hits nothing


def intrinsics(f: float, cx: float, cy: float) -> np.ndarray:
    return np.array([[f, 0.0, cx], [0.0, f, cy], [0.0, 0.0, 1.0]])


def rot_x(deg: float) -> np.ndarray:
    a = math.radians(deg)
    return np.array([[1, 0, 0], [0, math.cos(a), -math.sin(a)], [0, math.sin(a), math.cos(a)]])


def rot_y(deg: float) -> np.ndarray:
    a = math.radians(deg)
    return np.array([[math.cos(a), 0, math.sin(a)], [0, 1, 0], [-math.sin(a), 0, math.cos(a)]])


def rot_z(deg: float) -> np.ndarray:
    a = math.radians(deg)
    return np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])


def rigid(R: np.ndarray, t) -> np.ndarray:
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T


def rigid_inverse(T: np.ndarray) -> np.ndarray:
    R, t = T[:3, :3], T[:3, 3]
    return rigid(R.T, -R.T @ t)


def default_rgb_extrinsic() -> np.ndarray:
    """T_rgb_from_d: the HD camera sits 25 mm along +x of the depth camera, rotated 1 deg
    about y (a Kinect with an HD camera bolted beside it, Sec. IV.A)."""
    return rigid_inverse(rigid(rot_y(1.0), [0.025, 0.0, 0.0]))


def look_at_pose(position, target=(0.0, 0.0, 0.0)) -> np.ndarray:
    """T_world_from_cam for a camera at `position` looking at `target` in a z-up world;
    camera axes x right, y down, z forward."""
    c = np.asarray(position, float)
    f = np.asarray(target, float) - c
    f /= np.linalg.norm(f)
    x = np.cross(f, [0.0, 0.0, 1.0])
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    return rigid(np.stack([x, y, f], axis=1), c)


def orbit_poses(n: int, radius: float = 0.8, height: float = 0.3, jitter: float = 0.0,
                rng: np.random.Generator | None = None, sweep_deg: float = 360.0) -> np.ndarray:
    poses = np.zeros((n, 4, 4))
    for i in range(n):
        a = math.radians(sweep_deg) * i / n
        pos = np.array([radius * math.cos(a), radius * math.sin(a), height])
        if jitter > 0.0:
            pos = pos + rng.uniform(-jitter, jitter, 3)
        poses[i] = look_at_pose(pos)
    return poses


@dataclasses.dataclass
class VolumeSpec:
    """A geometry volume and the finer colour volume over the same cube (Sec. IV.B)."""
    gdim: tuple
    cdim: tuple
    origin: tuple
    extent: tuple
    sigma: float = 0.020    # colour distance threshold, 20 mm (Sec. IV.B)
    gate: float = 0.8       # colour weight gate (Sec. IV.B)
    hd_sampling: str = "bilinear"   # or "nearest": the HD pixel nearest the projection

    @staticmethod
    def cube(g: int, ratio: int, size: float, **kw) -> "VolumeSpec":
        return VolumeSpec((g, g, g), (g * ratio,) * 3, (-size / 2,) * 3, (size,) * 3, **kw)

    @property
    def n_geom(self) -> int:
        return int(np.prod(self.gdim))

    @property
    def n_colour(self) -> int:
        return int(np.prod(self.cdim))

    @property
    def geom_voxel(self) -> float:
        return self.extent[0] / self.gdim[0]


@dataclasses.dataclass
class Frames:
    """A scan: depth [n,H,W] float32 metres (0 = hole), RGB [n,CH,CW,3] uint8 or float32
    in [0,1], intrinsics, the depth-to-HD extrinsic and one camera pose per frame."""
    depth: object
    rgb: object
    K_d: np.ndarray
    K_rgb: np.ndarray
    T_rgb_from_d: np.ndarray
    T_world_from_cam: np.ndarray
    trunc: float
    w_max: float

    @property
    def n(self) -> int:
        return int(self.depth.shape[0])

    def select(self, idx) -> "Frames":
        if isinstance(idx, int):
            idx = slice(idx, idx + 1)
        return dataclasses.replace(self, depth=self.depth[idx], rgb=self.rgb[idx],
                                   T_world_from_cam=self.T_world_from_cam[idx])

    def to(self, device) -> "Frames":
        return dataclasses.replace(self, depth=_tensor(self.depth).to(device).contiguous(),
                                   rgb=_tensor(self.rgb).to(device).contiguous())

    def numpy(self) -> "Frames":
        return dataclasses.replace(self, depth=_array(self.depth), rgb=_array(self.rgb))

    def as_float_rgb(self) -> "Frames":
        """The same images as float32 in [0,1]: value = byte * float32(1/255)."""
        rgb = self.rgb
        if isinstance(rgb, torch.Tensor):
            if rgb.dtype == torch.uint8:
                rgb = rgb.to(torch.float32) * torch.tensor(np.float32(1.0 / 255.0), device=rgb.device)
        elif rgb.dtype == np.uint8:
            rgb = rgb.astype(np.float32) * np.float32(1.0 / 255.0)
        return dataclasses.replace(self, rgb=rgb)


def _tensor(a):
    return a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))


def _array(a):
    return a.detach().cpu().numpy() if isinstance(a, torch.Tensor) else np.asarray(a)


# ----------------------------------------------------------------------------- scene

@dataclasses.dataclass
class Scene:
    plane_z: float
    plane_colours: np.ndarray                    # (2,3) checker colour pair
    spheres: list = dataclasses.field(default_factory=list)   # (centre(3), r, colours(2,3))
    boxes: list = dataclasses.field(default_factory=list)     # (centre(3), half(3), yaw, colours)
    noise_seed: int = 0


def random_scene(rng: np.random.Generator, size: float, n_spheres: int, n_boxes: int) -> Scene:
    plane_z = -size / 2 + 0.05
    sc = Scene(plane_z, rng.uniform(0.15, 0.9, (2, 3)), noise_seed=int(rng.integers(1 << 30)))
    for _ in range(n_spheres):
        r = rng.uniform(0.05, 0.12)
        rad, ang = 0.2 * math.sqrt(rng.uniform()), rng.uniform(0, 2 * math.pi)
        c = np.array([rad * math.cos(ang), rad * math.sin(ang), plane_z + r])
        sc.spheres.append((c, r, rng.uniform(0.1, 0.95, (2, 3))))
    for _ in range(n_boxes):
        h = rng.uniform(0.04, 0.10, 3)
        yaw = rng.uniform(0, math.pi)
        rad, ang = 0.2 * math.sqrt(rng.uniform()), rng.uniform(0, 2 * math.pi)
        c = np.array([rad * math.cos(ang), rad * math.sin(ang), plane_z + h[2]])
        sc.boxes.append((c, h, yaw, rng.uniform(0.1, 0.95, (2, 3))))
    return sc


def _hash01(ix, iy, iz, seed: int):
    """Integer lattice hash -> [0,1) (int64 arithmetic kept below 2**63)."""
    m = 0xFFFFFFFF
    h = (ix * 73856093) & m
    h = h ^ ((iy * 19349663) & m)
    h = h ^ ((iz * 83492791) & m)
    h = h ^ (seed & m)
    h = (h ^ (h >> 16)) & m
    h = (h * 0x45D9F3B) & m
    h = (h ^ (h >> 16)) & m
    h = (h * 0x45D9F3B) & m
    h = (h ^ (h >> 16)) & m
    return h.to(torch.float64) / 4294967296.0


def value_noise(p: torch.Tensor, cell: float, seed: int) -> torch.Tensor:
    """Trilinear value noise on a `cell`-sized lattice with smoothstep fades."""
    q = p / cell
    i0 = torch.floor(q)
    f = q - i0
    s = f * f * (3.0 - 2.0 * f)
    i0 = i0.to(torch.int64) + (1 << 20)
    out = torch.zeros(p.shape[:-1], dtype=torch.float64, device=p.device)
    for dx in (0, 1):
        wx = s[..., 0] if dx else 1.0 - s[..., 0]
        for dy in (0, 1):
            wy = s[..., 1] if dy else 1.0 - s[..., 1]
            for dz in (0, 1):
                wz = s[..., 2] if dz else 1.0 - s[..., 2]
                out = out + wx * wy * wz * _hash01(i0[..., 0] + dx, i0[..., 1] + dy,
                                                   i0[..., 2] + dz, seed)
    return out


def _albedo(p: torch.Tensor, colours: torch.Tensor, seed: int) -> torch.Tensor:
    """Solid 2 cm checker between two colours, modulated by 5 mm value noise."""
    cells = torch.floor(p / 0.02).to(torch.int64).sum(-1)
    odd = (cells % 2).to(torch.float64)[..., None]
    base = colours[0] * (1.0 - odd) + colours[1] * odd
    return base * (0.7 + 0.3 * value_noise(p, 0.005, seed))[..., None]


def _cast(scene: Scene, o: torch.Tensor, d: torch.Tensor):
    """Nearest hit along rays o + t d (t > 0): returns t (inf = miss) and primitive id."""
    eps = 1e-9
    dev = d.device
    best = torch.full(d.shape[:-1], math.inf, dtype=torch.float64, device=dev)
    pid = torch.full(d.shape[:-1], -1, dtype=torch.int64, device=dev)

    def take(t, k):
        nonlocal best, pid
        better = t < best
        best = torch.where(better, t, best)
        pid = torch.where(better, torch.full_like(pid, k), pid)

    dz = d[..., 2]
    t = (scene.plane_z - o[2]) / torch.where(dz.abs() < 1e-300, torch.full_like(dz, 1e-300), dz)
    take(torch.where(t > eps, t, torch.full_like(t, math.inf)), 0)
    k = 1
    for c, r, _ in scene.spheres:
        oc = o - torch.as_tensor(c, device=dev)
        a = (d * d).sum(-1)
        b = (d * oc).sum(-1)
        cc = float(oc @ oc) - r * r
        disc = b * b - a * cc
        t = (-b - torch.sqrt(torch.clamp(disc, min=0.0))) / a
        take(torch.where((disc >= 0) & (t > eps), t, torch.full_like(t, math.inf)), k)
        k += 1
    for c, h, yaw, _ in scene.boxes:
        R = torch.as_tensor(rot_z(math.degrees(yaw)), device=dev)
        ol = R.T @ (o - torch.as_tensor(c, device=dev))
        dl = d @ R
        dl = torch.where(dl.abs() < 1e-12, torch.full_like(dl, 1e-12), dl)
        hh = torch.as_tensor(h, device=dev)
        t1 = (-hh - ol) / dl
        t2 = (hh - ol) / dl
        tmin = torch.minimum(t1, t2).amax(-1)
        tmax = torch.maximum(t1, t2).amin(-1)
        hit = (tmax >= tmin) & (tmin > eps)
        take(torch.where(hit, tmin, torch.full_like(tmin, math.inf)), k)
        k += 1
    return best, pid


def _colour(scene: Scene, p: torch.Tensor, pid: torch.Tensor) -> torch.Tensor:
    dev = p.device
    rgb = torch.full(p.shape, BACKGROUND / 255.0, dtype=torch.float64, device=dev)
    pairs = [scene.plane_colours] + [s[2] for s in scene.spheres] + [b[3] for b in scene.boxes]
    for k, pair in enumerate(pairs):
        m = pid == k
        if bool(m.any()):
            rgb[m] = _albedo(p[m], torch.as_tensor(pair, device=dev), scene.noise_seed + 7919 * k)
    return rgb


def _rays(K: np.ndarray, W: int, H: int, T_world_from_cam: np.ndarray, dev):
    """Per-pixel rays with camera-frame direction ((u-cx)/fx, (v-cy)/fy, 1), in world."""
    u = torch.arange(W, dtype=torch.float64, device=dev)
    v = torch.arange(H, dtype=torch.float64, device=dev)
    vv, uu = torch.meshgrid(v, u, indexing="ij")
    dc = torch.stack([(uu - K[0, 2]) / K[0, 0], (vv - K[1, 2]) / K[1, 1], torch.ones_like(uu)], -1)
    R = torch.as_tensor(T_world_from_cam[:3, :3], device=dev)
    return torch.as_tensor(T_world_from_cam[:3, 3], device=dev), dc @ R.T


def render_depth(scene: Scene, K: np.ndarray, W: int, H: int, T_world_from_cam: np.ndarray,
                 dev) -> torch.Tensor:
    """Noise-free depth (z along the optical axis), 0 where nothing is hit in range."""
    o, d = _rays(K, W, H, T_world_from_cam, dev)
    t, _ = _cast(scene, o, d)
    return torch.where(t <= MAX_RANGE, t, torch.zeros_like(t))


def render_rgb(scene: Scene, K: np.ndarray, W: int, H: int, T_world_from_rgb: np.ndarray,
               dev) -> torch.Tensor:
    """Unlit albedo seen by the HD camera, quantised to uint8 (round(255 clamp))."""
    o, d = _rays(K, W, H, T_world_from_rgb, dev)
    t, pid = _cast(scene, o, d)
    p = o + t[..., None] * d
    rgb = _colour(scene, p, pid)
    return torch.round(255.0 * torch.clamp(rgb, 0.0, 1.0)).to(torch.uint8)


def surface_triangles(scene: Scene, K: np.ndarray, W: int, H: int, poses: np.ndarray,
                      n_tri: int, edge_px: int, rng: np.random.Generator, box=None,
                      device="cpu") -> np.ndarray:
    """Triangles lying on the scene's surfaces, as a mesh of the scan would: from a random
    pose and a random pixel (x, y), the rays of pixels (x, y), (x + e, y) and (x, y + e)
    (e = edge_px) are cast, and the three hit points become V1, V2, V3 when all three rays
    hit the same primitive within range (and, given box = (lo, hi), inside that box, as a
    mesh extracted from a volume would be).  float32 [n_tri, 3, 3]."""
    dev = torch.device(device)
    out = []
    have = 0
    while have < n_tri:
        m = 4 * (n_tri - have) + 64
        pi = rng.integers(len(poses), size=m)
        x = rng.integers(0, W - edge_px, size=m).astype(np.float64)
        y = rng.integers(0, H - edge_px, size=m).astype(np.float64)
        px = np.stack([np.stack([x, y], 1), np.stack([x + edge_px, y], 1),
                       np.stack([x, y + edge_px], 1)], 1)                 # [m, 3, 2]
        dc = np.concatenate([(px[..., :1] - K[0, 2]) / K[0, 0], (px[..., 1:] - K[1, 2]) / K[1, 1],
                             np.ones(px.shape[:-1] + (1,))], -1)           # [m, 3, 3]
        R = poses[pi, :3, :3]
        o = torch.as_tensor(np.repeat(poses[pi, :3, 3][:, None], 3, 1).reshape(-1, 3), device=dev)
        d = torch.as_tensor(np.einsum("mij,mkj->mki", R, dc).reshape(-1, 3), device=dev)
        t, pid = _cast_batch(scene, o, d)
        t, pid = t.reshape(m, 3), pid.reshape(m, 3)
        ok = (pid[:, 0] >= 0) & (pid[:, 0] == pid[:, 1]) & (pid[:, 0] == pid[:, 2]) & \
             (t <= MAX_RANGE).all(1)
        pts = (o + t.reshape(-1, 1) * d).reshape(m, 3, 3)[ok].cpu().numpy()
        if box is not None:
            lo, hi = np.asarray(box[0]), np.asarray(box[1])
            pts = pts[((pts >= lo) & (pts <= hi)).all(axis=(1, 2))]
        out.append(pts[:n_tri - have])
        have += len(out[-1])
    return np.concatenate(out).astype(np.float32)


def _cast_batch(scene: Scene, o: torch.Tensor, d: torch.Tensor):
    """_cast for rays with per-ray origins (o: [n, 3])."""
    eps = 1e-9
    dev = d.device
    best = torch.full(d.shape[:-1], math.inf, dtype=torch.float64, device=dev)
    pid = torch.full(d.shape[:-1], -1, dtype=torch.int64, device=dev)

    def take(t, k):
        nonlocal best, pid
        better = t < best
        best = torch.where(better, t, best)
        pid = torch.where(better, torch.full_like(pid, k), pid)

    dz = d[:, 2]
    t = (scene.plane_z - o[:, 2]) / torch.where(dz.abs() < 1e-300, torch.full_like(dz, 1e-300), dz)
    take(torch.where(t > eps, t, torch.full_like(t, math.inf)), 0)
    k = 1
    for c, r, _ in scene.spheres:
        oc = o - torch.as_tensor(c, device=dev)
        a = (d * d).sum(-1)
        b = (d * oc).sum(-1)
        cc = (oc * oc).sum(-1) - r * r
        disc = b * b - a * cc
        t = (-b - torch.sqrt(torch.clamp(disc, min=0.0))) / a
        take(torch.where((disc >= 0) & (t > eps), t, torch.full_like(t, math.inf)), k)
        k += 1
    for c, h, yaw, _ in scene.boxes:
        R = torch.as_tensor(rot_z(math.degrees(yaw)), device=dev)
        ol = (o - torch.as_tensor(c, device=dev)) @ R
        dl = d @ R
        dl = torch.where(dl.abs() < 1e-12, torch.full_like(dl, 1e-12), dl)
        hh = torch.as_tensor(h, device=dev)
        t1 = (-hh - ol) / dl
        t2 = (hh - ol) / dl
        tmin = torch.minimum(t1, t2).amax(-1)
        tmax = torch.maximum(t1, t2).amin(-1)
        hit = (tmax >= tmin) & (tmin > eps)
        take(torch.where(hit, tmin, torch.full_like(tmin, math.inf)), k)
        k += 1
    return best, pid


def render_scan(scene: Scene, poses: np.ndarray, depth_size, rgb_size, noise_k: float,
                dropout: float, rng: np.random.Generator, trunc: float, w_max: float,
                device="cpu", T_rgb_from_d: np.ndarray | None = None) -> Frames:
    dw, dh = depth_size
    cw, ch = rgb_size
    K_d = intrinsics(*DEPTH_INTRINSICS[(dw, dh)])
    K_rgb = intrinsics(*RGB_INTRINSICS[(cw, ch)])
    T_rd = default_rgb_extrinsic() if T_rgb_from_d is None else T_rgb_from_d
    T_dr = rigid_inverse(T_rd)
    n = len(poses)
    dev = torch.device(device)
    depth = torch.empty((n, dh, dw), dtype=torch.float32, device=dev)
    rgb = torch.empty((n, ch, cw, 3), dtype=torch.uint8, device=dev)
    for i in range(n):
        z = render_depth(scene, K_d, dw, dh, poses[i], dev)
        if noise_k > 0.0:
            noise = torch.as_tensor(rng.standard_normal((dh, dw)), device=dev)
            z = torch.where(z > 0, z + noise * noise_k * z * z, z)
        if dropout > 0.0:
            holes = torch.as_tensor(rng.uniform(size=(dh, dw)) < dropout, device=dev)
            z = torch.where(holes, torch.zeros_like(z), z)
        z = torch.where((z > 0) & (z <= MAX_RANGE), z, torch.zeros_like(z))
        depth[i] = z.to(torch.float32)
        rgb[i] = render_rgb(scene, K_rgb, cw, ch, poses[i] @ T_dr, dev)
    return Frames(depth, rgb, K_d, K_rgb, T_rd, poses.copy(), float(trunc), float(w_max))
