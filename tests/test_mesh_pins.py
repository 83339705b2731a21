"""Pins of the oracle's marching cubes (CPU only).

The mesh extraction (Sec. III, after KinectFusion: the polygons of Sec. IV.C come from
it) is checked against properties that geometry and topology fix, not against its own
tables:
* one inside (or one outside) corner: one triangle on that corner's three edges, facing
  away from the inside;
* an ambiguous face (two diagonal inside corners) cuts off each inside corner;
* random sign fields over every cube configuration give a watertight, consistently
  oriented mesh: each edge away from the volume's boundary is used by exactly two
  triangles, once in each direction; every vertex is used;
* a sphere gives a closed surface of Euler characteristic 2 whose enclosed (signed)
  volume is 4/3 pi R^3 to the discretisation error, vertices on the sphere to the
  interpolation error; a torus gives Euler characteristic 0;
* an affine field (a plane) is reproduced exactly (up to the FP32 storage of the field):
  vertices on the plane, normals along its gradient, area of the plane inside the grid of
  voxel centres;
* F = 0 at voxel centres counts as outside (one sheet, not two);
* unobserved voxels (weight 0) remove exactly the cubes that touch them;
* vertices are numbered by (owning voxel, axis).
"""
import numpy as np
import pytest

from kf_synth.scenes import VolumeSpec

pytestmark = pytest.mark.usefixtures("oracle")

# cube corner c = x + 2y + 4z; edge id 4a + b0 + 2 b1 (other axes in increasing order)
CORNERS = np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], float)


def edge_point(e, t=0.5):
    a, b0, b1 = e >> 2, e & 1, (e >> 1) & 1
    others = [k for k in range(3) if k != a]
    p = np.zeros(3)
    p[others[0]], p[others[1]] = b0, b1
    p[a] = t
    return p


def centres(spec):
    s = np.asarray(spec.extent, float) / np.asarray(spec.gdim)
    ax = [spec.origin[k] + (np.arange(spec.gdim[k]) + 0.5) * s[k] for k in range(3)]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def index_coords(spec, p):
    s = np.asarray(spec.extent, float) / np.asarray(spec.gdim)
    return (p - np.asarray(spec.origin)) / s - 0.5


def edge_uses(tris):
    """Directed edge -> count, undirected edge -> count."""
    d = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    directed = {}
    for a, b in map(tuple, d):
        directed[(a, b)] = directed.get((a, b), 0) + 1
    undirected = {}
    for (a, b), n in directed.items():
        k = (min(a, b), max(a, b))
        undirected[k] = undirected.get(k, 0) + n
    return directed, undirected


def signed_volume(v, t):
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


# ---- single cubes

@pytest.mark.parametrize("c", range(8))
def test_single_inside_corner(oracle, c):
    for mask, sign in ((1 << c, 1.0), (0xFF ^ (1 << c), -1.0)):
        t = oracle.mc_cube_triangles(mask)
        assert t.shape == (1, 3)
        pts = np.array([edge_point(e) for e in t[0]])
        # the three edges of corner c
        assert all(np.abs(p - CORNERS[c]).sum() == 0.5 for p in pts)
        n = np.cross(pts[1] - pts[0], pts[2] - pts[0])
        # one inside corner: the normal points away from it; one outside corner: towards it
        assert sign * np.dot(n, pts.mean(0) - CORNERS[c]) > 0


def test_ambiguous_face_cuts_inside_corners(oracle):
    # corners 0 and 3 (diagonal on the face z = 0) inside: two separate triangles
    t = oracle.mc_cube_triangles((1 << 0) | (1 << 3))
    assert sorted(map(sorted, t.tolist())) == [[0, 4, 8], [1, 5, 11]]
    # the complement (0 and 3 outside): the face cuts off its inside corners 1 and 2, so
    # the two outside corners stay joined across it and one loop of six edges separates
    # them from the inside: 4 triangles fanned from one vertex
    t = oracle.mc_cube_triangles(0xFF ^ ((1 << 0) | (1 << 3)))
    assert len(t) == 4 and set(t.ravel().tolist()) == {0, 1, 4, 5, 8, 11}
    assert len(set(t[:, 0].tolist())) == 1


def faces_of(e):
    a, b0, b1 = e >> 2, e & 1, (e >> 1) & 1
    others = [k for k in range(3) if k != a]
    return {(others[0], b0), (others[1], b1)}


def test_no_triangle_edge_inside_a_face(oracle):
    """A triangle side joining two vertices on one cube face must be a segment of that face
    (both cubes sharing the face lay it, in opposite directions); a chord across a face
    would be laid by the neighbour too and break the mesh."""
    for mask in range(256):
        t = oracle.mc_cube_triangles(mask)
        uses = {}
        for tri in t.tolist():
            for a, b in ((tri[0], tri[1]), (tri[1], tri[2]), (tri[2], tri[0])):
                uses[(a, b)] = uses.get((a, b), 0) + 1
        for (a, b), n in uses.items():
            if faces_of(a) & faces_of(b):
                # a face segment: used once in this cube, not in reverse
                assert n == 1 and (b, a) not in uses, (mask, a, b)
            else:
                # an inner chord: once in each direction
                assert n == 1 and uses.get((b, a)) == 1, (mask, a, b)


def test_triangle_count_matches_loops(oracle):
    """Every crossed edge is used; triangles = crossed edges - 2 x loops (fans)."""
    for mask in range(256):
        t = oracle.mc_cube_triangles(mask)
        crossed = set()
        for e in range(12):
            p = edge_point(e, 0.0)
            q = edge_point(e, 1.0)
            c0 = int(p @ [1, 2, 4])
            c1 = int(q @ [1, 2, 4])
            if ((mask >> c0) & 1) != ((mask >> c1) & 1):
                crossed.add(e)
        used = set(t.ravel().tolist())
        assert used == crossed, mask
        if t.size:
            # each loop is fanned from its first edge: loops = distinct fan centres
            loops = len(set(t[:, 0].tolist()))
            assert len(t) == len(crossed) - 2 * loops


# ---- whole volumes

def mesh(oracle, spec, F, W=None, precision="f64"):
    W = np.ones_like(F) if W is None else W
    return oracle.marching_cubes(spec, F.astype(np.float32), W.astype(np.float32), precision)


def test_random_fields_watertight_and_oriented(oracle):
    spec = VolumeSpec((24, 22, 26), (48, 44, 52), (-0.5, -0.45, -0.55), (1.0, 0.9, 1.1))
    rng = np.random.default_rng(7)
    F = rng.uniform(-1, 1, int(np.prod(spec.gdim)))
    F[np.abs(F) < 1e-3] = 0.5
    # every configuration occurs
    X, Y, Z = spec.gdim
    G = (F.reshape(Z, Y, X) < 0).astype(int)
    cfg = sum(G[(c >> 2) & 1:Z - 1 + ((c >> 2) & 1), (c >> 1) & 1:Y - 1 + ((c >> 1) & 1),
                c & 1:X - 1 + (c & 1)] << c for c in range(8))
    assert len(np.unique(cfg)) == 256
    v, t = mesh(oracle, spec, F)
    directed, undirected = edge_uses(t)
    q = index_coords(spec, v)
    on_bd = (np.abs(q) < 1e-9) | (np.abs(q - (np.asarray(spec.gdim) - 1)) < 1e-9)
    for (a, b), n in undirected.items():
        if n == 1:      # only on the volume's boundary, both ends on a common boundary plane
            assert (on_bd[a] & on_bd[b]).any()
        else:
            assert n == 2 and directed.get((a, b), 0) == 1 and directed.get((b, a), 0) == 1
    assert np.array_equal(np.unique(t), np.arange(len(v)))      # every vertex used
    # vertices numbered by (owning voxel, axis): one fractional index coordinate each
    frac = np.abs(q - np.rint(q)) > 1e-9
    assert (frac.sum(1) == 1).all()
    axis = frac.argmax(1)
    own = np.floor(q + 1e-9).astype(np.int64)
    key = ((own[:, 2] * Y + own[:, 1]) * X + own[:, 0]) * 3 + axis
    assert (np.diff(key) > 0).all()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_sphere_closed_euler_volume(oracle, precision):
    spec = VolumeSpec((40, 36, 44), (80, 72, 88), (-0.5, -0.45, -0.55), (1.0, 0.9, 1.1))
    c, R = np.array([0.03, -0.02, 0.05]), 0.3
    p = centres(spec)
    F = np.clip((np.linalg.norm(p - c, axis=1) - R) / 0.08, -1, 1)
    v, t = mesh(oracle, spec, F, precision=precision)
    v = v.astype(np.float64)
    directed, undirected = edge_uses(t)
    assert all(n == 2 for n in undirected.values())
    assert all(n == 1 for n in directed.values())
    assert len(v) - len(undirected) + len(t) == 2
    vol = signed_volume(v - c, t)
    assert abs(vol / (4 / 3 * np.pi * R ** 3) - 1) < 0.01
    s = np.asarray(spec.extent) / np.asarray(spec.gdim)
    assert np.abs(np.linalg.norm(v - c, axis=1) - R).max() < 0.1 * s.min()


def test_torus_euler_zero(oracle):
    spec = VolumeSpec((48, 48, 32), (96, 96, 64), (-0.5, -0.5, -0.33), (1.0, 1.0, 0.66))
    p = centres(spec)
    Rt, rt = 0.3, 0.11
    d = np.sqrt((np.hypot(p[:, 0], p[:, 1]) - Rt) ** 2 + p[:, 2] ** 2) - rt
    v, t = mesh(oracle, spec, np.clip(d / 0.06, -1, 1))
    _, undirected = edge_uses(t)
    assert all(n == 2 for n in undirected.values())
    assert len(v) - len(undirected) + len(t) == 0
    assert signed_volume(v, t) > 0


@pytest.mark.parametrize("tilt", [0.0, 0.3])
def test_plane_exact(oracle, tilt):
    spec = VolumeSpec((20, 18, 22), (40, 36, 44), (-0.5, -0.45, -0.55), (1.0, 0.9, 1.1))
    n = np.array([tilt, -0.5 * tilt, 1.0])
    d0 = 0.0137
    p = centres(spec)
    F = (p @ n - d0) / np.linalg.norm(n)
    v, t = mesh(oracle, spec, F / 0.5)
    # exact up to the FP32 storage of the field (a relative 6e-8 of each sample)
    assert np.abs(v @ n - d0).max() < 1e-8
    nt = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    area = 0.5 * np.linalg.norm(nt, axis=1)
    assert (nt @ n > 0).all()                                    # towards positive F
    assert (np.linalg.norm(np.cross(nt, n), axis=1) <
            1e-5 * np.linalg.norm(nt, axis=1) * np.linalg.norm(n)).all()
    s = np.asarray(spec.extent) / np.asarray(spec.gdim)
    X, Y, _ = spec.gdim
    # the plane crosses the grid of centres over its whole x-y extent
    want = (X - 1) * s[0] * (Y - 1) * s[1] * np.linalg.norm(n) / abs(n[2])
    assert abs(area.sum() / want - 1) < 1e-6


def test_zero_at_centres_is_outside(oracle):
    spec = VolumeSpec((12, 10, 14), (24, 20, 28), (-0.5, -0.4, -0.55), (1.0, 0.8, 1.1))
    X, Y, Z = spec.gdim
    k = 6
    F = np.broadcast_to((np.arange(Z) - k)[:, None, None], (Z, Y, X)).astype(float).ravel()
    v, t = mesh(oracle, spec, F)
    q = index_coords(spec, v)
    assert np.allclose(q[:, 2], k, atol=1e-12)                  # one sheet, at layer k
    assert len(t) == 2 * (X - 1) * (Y - 1)
    assert np.array_equal(np.unique(t), np.arange(len(v)))      # valid, every vertex used


def test_unobserved_voxels_remove_their_cubes(oracle):
    spec = VolumeSpec((30, 28, 32), (60, 56, 64), (-0.5, -0.45, -0.55), (1.0, 0.9, 1.1))
    p = centres(spec)
    F = np.clip((np.linalg.norm(p, axis=1) - 0.3) / 0.08, -1, 1)
    v0, t0 = mesh(oracle, spec, F)
    X, Y, Z = spec.gdim
    W = np.ones(X * Y * Z)
    q0 = index_coords(spec, v0)
    # a voxel next to the surface
    i = np.argmin(np.abs(np.linalg.norm(p, axis=1) - 0.3))
    W[i] = 0.0
    v1, t1 = mesh(oracle, spec, F, W)
    ix, iy, iz = i % X, (i // X) % Y, i // (X * Y)
    # the cubes with lower corner in [i - 1, i] on every axis are gone: their triangles
    # are those whose 3 vertices lie in the closed 2x2x2-voxel region around voxel i
    lo, hi = np.array([ix - 1, iy - 1, iz - 1]), np.array([ix + 1, iy + 1, iz + 1])
    inside0 = ((q0[t0] >= lo - 1e-9) & (q0[t0] <= hi + 1e-9)).all(axis=(1, 2))
    kept = t0[~inside0]
    assert len(t1) == len(kept) and len(t1) < len(t0)
    # the rest of the mesh is the same triangles (by position)
    key = lambda v, t: sorted(map(tuple, np.round(v[t].reshape(-1, 9), 12)))   # noqa: E731
    assert key(v1, t1) == key(v0, kept)
    _, undirected = edge_uses(t1)
    assert sum(n == 1 for n in undirected.values()) >= 3          # a hole with a rim
    # vertices only where a remaining cube uses them
    assert np.array_equal(np.unique(t1), np.arange(len(v1)))
    assert len(v1) < len(v0)
    W[:] = 0.0
    v2, t2 = mesh(oracle, spec, F, W)
    assert len(v2) == 0 and len(t2) == 0
    # a single observed layer: its edges cross the sphere, but no cube is complete
    W.reshape(Z, Y, X)[Z // 2] = 1.0
    v3, t3 = mesh(oracle, spec, F, W)
    assert len(v3) == 0 and len(t3) == 0
