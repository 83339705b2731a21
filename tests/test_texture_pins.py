"""Pins of the oracle's per-polygon texture maps and atlas layout (CPU only).

Texture generation (Sec. IV.D, Eq. 11-14) is checked against results fixed by geometry and
by an independent interpolation routine rather than by its own formulas:
* map sizes of triangles with exactly representable edge lengths (Eq. 11-12, rounded up,
  at least 2);
* the worked example of the paper: the texel two steps along V_aV_b and three along V_aV_c
  sits at V_a + 2 V_aV_green + 3 V_aV_blue;
* an affine colour field is reproduced exactly by trilinear interpolation, so every texel
  equals the field at its closed-form world point (to the FP32 rounding of the stored voxel
  colours and of the output);
* on a random colour field, every texel equals scipy's linear interpolation
  (ndimage.map_coordinates, order 1) of the voxel grid at that point, with voxel centres at
  origin + (i + 1/2) s;
* texels whose cell touches a zero colour weight, or that lie outside the volume, are zero;
* constant fields fix the 8-bit conversion (rint of 255 min(max(c, 0), 1), ties to even);
* degenerate triangles give constant rows or a constant map;
* the layout: maps in the atlas, disjoint, column-wise from the top left, a new column
  only when the next map does not fit, and the width the rightmost column reaches.
"""
import numpy as np
import pytest
from scipy import ndimage

from kf_synth.scenes import VolumeSpec

pytestmark = pytest.mark.usefixtures("oracle")

U = 2.0 ** -10          # an exactly representable texel size


def colour_state(oracle, spec, fn, weight=1.0):
    """A state whose colour voxels hold fn(centre) and weight `weight` (geometry unused)."""
    st = oracle.State(spec, np.float32)
    s = np.asarray(spec.extent, float) / np.asarray(spec.cdim)
    ax = [spec.origin[k] + (np.arange(spec.cdim[k]) + 0.5) * s[k] for k in range(3)]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    rgb = fn(np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1))
    st.r[:], st.g[:], st.b[:] = [rgb[:, k].astype(np.float32) for k in range(3)]
    st.wc[:] = weight
    return st


def affine(p):
    return np.stack([0.2 + 0.3 * p[:, 0], 0.5 - 0.2 * p[:, 1], 0.1 + 0.4 * p[:, 2]], axis=1)


def texel_points(tri, rect):
    """World point of every texel of one map, FP64: V1 + i (V2-V1)/(w-1) + j (V3-V1)/(h-1)."""
    V = np.asarray(tri, np.float32).astype(np.float64).reshape(3, 3)
    w, h = int(rect[2]), int(rect[3])
    j, i = np.meshgrid(np.arange(h, dtype=float), np.arange(w, dtype=float), indexing="ij")
    g = (V[1] - V[0]) / (w - 1)
    b = (V[2] - V[0]) / (h - 1)
    return V[0] + i[..., None] * g + j[..., None] * b           # [h, w, 3]


def texels(atlas, rect):
    x, y, w, h = (int(v) for v in rect)
    return atlas[y:y + h, x:x + w]


def spec_aniso():
    return VolumeSpec((24, 20, 28), (48, 40, 56), (-0.5, -0.4, -0.55), (1.0, 0.8, 1.1))


def random_triangles(rng, n, spec, edge=(0.02, 0.08)):
    lo = np.asarray(spec.origin) + 0.1
    hi = np.asarray(spec.origin) + np.asarray(spec.extent) - 0.1
    V1 = rng.uniform(lo, hi, (n, 3))
    d2 = rng.normal(size=(n, 3))
    d3 = rng.normal(size=(n, 3))
    d2 *= (rng.uniform(*edge, n) / np.linalg.norm(d2, axis=1))[:, None]
    d3 *= (rng.uniform(*edge, n) / np.linalg.norm(d3, axis=1))[:, None]
    tri = np.stack([V1, np.clip(V1 + d2, lo, hi), np.clip(V1 + d3, lo, hi)], axis=1)
    return tri.astype(np.float32)


# ---- Eq. 11-12: map sizes

@pytest.mark.parametrize("e2,e3,wh", [
    ((30, 0, 0), (0, 40, 0), (30, 40)),          # axis edges of 30 and 40 texels
    ((18, 24, 0), (0, -24, 32), (30, 40)),       # 3-4-5 edges, 30 and 40 texels long
    ((30.5, 0, 0), (0, 0, 2.25), (31, 3)),       # fractions round up
    ((0.3, 0, 0), (0, 0, 1.0), (2, 2)),          # at least 2 texels per side
    ((0, 0, 0), (0, 0, 0), (2, 2)),              # degenerate
])
def test_map_size(oracle, e2, e3, wh):
    V1 = np.array([0.125, -0.25, 0.0625])
    tri = np.stack([V1, V1 + np.array(e2) * U, V1 + np.array(e3) * U])[None]
    rects, width = oracle.texture_layout(tri, U, 1024)
    assert tuple(rects[0, 2:]) == wh
    assert tuple(rects[0, :2]) == (0, 0) and width == wh[0]


# ---- Eq. 13-14 and the colour lookup

def test_worked_example(oracle):
    """The texel in column 2, row 3 of a map is V_a + 2 V_aV_green + 3 V_aV_blue."""
    spec = spec_aniso()
    st = colour_state(oracle, spec, affine)
    V1 = np.array([-0.2, 0.1, 0.05])
    tri = np.stack([V1, V1 + np.array([9, 3, 0]) * 8 * U, V1 + np.array([0, -4, 7]) * 8 * U])
    rects, width = oracle.texture_layout(tri[None], 8 * U, 64)
    w, h = rects[0, 2:]
    assert (w, h) == (10, 9)
    atlas, _ = oracle.texture(spec, st, tri[None], rects, width, 64, precision="f64")
    V = tri.astype(np.float32).astype(float)
    p23 = V[0] + 2 * (V[1] - V[0]) / (w - 1) + 3 * (V[2] - V[0]) / (h - 1)
    np.testing.assert_allclose(atlas[3, 2], affine(p23[None])[0], rtol=0, atol=2e-7)


@pytest.mark.parametrize("precision,tol", [("f64", 2e-7), ("f32", 3e-6)])
def test_affine_field_every_texel(oracle, precision, tol):
    spec = spec_aniso()
    st = colour_state(oracle, spec, affine)
    tri = random_triangles(np.random.default_rng(3), 40, spec)
    rects, width = oracle.texture_layout(tri, 0.004, 96)
    atlas, _ = oracle.texture(spec, st, tri, rects, width, 96, precision=precision)
    for t, r in zip(tri, rects):
        want = affine(texel_points(t, r).reshape(-1, 3)).reshape(int(r[3]), int(r[2]), 3)
        np.testing.assert_allclose(texels(atlas, r), want, rtol=0, atol=tol)


def test_random_field_matches_scipy_linear_interpolation(oracle):
    spec = spec_aniso()
    rng = np.random.default_rng(4)
    st = oracle.State(spec, np.float32)
    for a in (st.r, st.g, st.b):
        a[:] = rng.uniform(0, 1, a.size).astype(np.float32)
    st.wc[:] = 1.0
    tri = random_triangles(rng, 30, spec)
    rects, width = oracle.texture_layout(tri, 0.006, 64)
    atlas, _ = oracle.texture(spec, st, tri, rects, width, 64, precision="f64")
    s = np.asarray(spec.extent, float) / np.asarray(spec.cdim)
    cx, cy, cz = spec.cdim
    grids = [a.astype(np.float64).reshape(cz, cy, cx) for a in (st.r, st.g, st.b)]
    for t, r in zip(tri, rects):
        p = texel_points(t, r).reshape(-1, 3)
        q = (p - np.asarray(spec.origin)) / s - 0.5                    # index coordinates
        want = np.stack([ndimage.map_coordinates(G, q[:, ::-1].T, order=1) for G in grids], 1)
        got = texels(atlas, r).reshape(-1, 3)
        np.testing.assert_allclose(got, want, rtol=0, atol=1.5e-7)
        if (r == rects[0]).all():          # the three corners sit on V1, V2, V3
            w, h = int(r[2]), int(r[3])
            for k, idx in ((0, 0), (1, w - 1), (2, (h - 1) * w)):
                qv = (t[k].astype(float) - np.asarray(spec.origin)) / s - 0.5
                cv = [ndimage.map_coordinates(G, qv[::-1, None], order=1)[0] for G in grids]
                np.testing.assert_allclose(got[idx], cv, rtol=0, atol=1.5e-7)


def test_zero_weight_and_outside_texels_are_zero(oracle):
    """Colour weights vanish for voxels with x index below m: a texel is coloured iff its
    cell's lower x corner has index >= m, i.e. iff its point lies at or beyond the centre of
    voxel m; texels beyond the volume's last centres are zero too."""
    spec = spec_aniso()
    st = colour_state(oracle, spec, lambda p: 0.3 + 0.0 * p)
    cx, cy, cz = spec.cdim
    m = 20
    st.wc.reshape(cz, cy, cx)[:, :, :m] = 0.0
    s = np.asarray(spec.extent, float) / np.asarray(spec.cdim)
    x_m = spec.origin[0] + (m + 0.5) * s[0]
    z_top = spec.origin[2] + (cz - 0.5) * s[2]                    # the last centre in z
    V1 = np.array([x_m - 0.07, 0.01, z_top - 0.05])
    tri = np.stack([V1, V1 + [0.15, 0.0, 0.0], V1 + [0.0, 0.03, 0.1]]).astype(np.float32)
    rects, width = oracle.texture_layout(tri[None], 0.003, 64)
    atlas, atlas8 = oracle.texture(spec, st, tri[None], rects, width, 64, precision="f64")
    p = texel_points(tri, rects[0]).reshape(-1, 3)
    got = texels(atlas, rects[0]).reshape(-1, 3)
    inside = (p[:, 0] > x_m + 1e-9) & (p[:, 2] < z_top - 1e-9)
    outside = (p[:, 0] < x_m - 1e-9) | (p[:, 2] > z_top + 1e-9)
    assert inside.sum() > 50 and outside.sum() > 50
    np.testing.assert_allclose(got[inside], np.float32(0.3), rtol=0, atol=1e-7)
    assert not got[outside].any()
    assert not texels(atlas8, rects[0]).reshape(-1, 3)[outside].any()


def test_byte_conversion(oracle):
    """Constant fields: trilinear interpolation returns the constant exactly, so the bytes
    are rint(255 clamp(c)), with 127.5 -> 128 and 2.5 -> 2 (ties to even) in FP32."""
    spec = spec_aniso()
    consts = [(0.5, 1.2, -0.3), (0.25, float(np.float32(2.5 / 255)), 1.0)]
    want8 = [(128, 255, 0), (64, 2, 255)]
    for c, w8 in zip(consts, want8):
        st = colour_state(oracle, spec, lambda p: np.broadcast_to(np.array(c), p.shape))
        tri = random_triangles(np.random.default_rng(5), 3, spec)
        rects, width = oracle.texture_layout(tri, 0.01, 32)
        atlas, atlas8 = oracle.texture(spec, st, tri, rects, width, 32, precision="f32")
        for r in rects:
            assert (texels(atlas, r) == np.float32(c)).all()
            assert (texels(atlas8, r) == np.array(w8, np.uint8)).all()


def test_degenerate_triangles(oracle):
    spec = spec_aniso()
    st = colour_state(oracle, spec, affine)
    V1 = np.array([0.05, -0.02, 0.1])
    tri = np.stack([
        [V1, V1, V1 + [0.0, 0.05, 0.02]],          # V1 = V2: every row constant
        [V1, V1, V1],                                # a point: one colour
    ]).astype(np.float32)
    rects, width = oracle.texture_layout(tri, 0.004, 64)
    atlas, _ = oracle.texture(spec, st, tri, rects, width, 64, precision="f32")
    a = texels(atlas, rects[0])
    assert rects[0, 2] == 2 and (a == a[:, :1]).all()
    b = texels(atlas, rects[1])
    assert tuple(rects[1, 2:]) == (2, 2) and (b == b[0, 0]).all()
    np.testing.assert_allclose(b[0, 0], affine(V1[None].astype(np.float32).astype(float))[0],
                               atol=3e-6)


def test_untouched_texels_and_f32_vs_f64(oracle):
    spec = spec_aniso()
    rng = np.random.default_rng(6)
    st = colour_state(oracle, spec, lambda p: 0.5 + 0.3 * np.sin(9 * p))
    tri = random_triangles(rng, 25, spec)
    rects, width = oracle.texture_layout(tri, 0.005, 80)
    fill = np.full((80, width, 3), -7.0, np.float32)
    a32, _ = oracle.texture(spec, st, tri, rects, width, 80, atlas=fill.copy())
    a64, _ = oracle.texture(spec, st, tri, rects, width, 80, precision="f64")
    mask = np.zeros((80, width), bool)
    for r in rects:
        texels(mask, r)[:] = True
    assert (a32[~mask] == -7.0).all()
    np.testing.assert_allclose(a32[mask], a64[mask], rtol=0, atol=1e-5)


# ---- atlas layout (Sec. IV.D merging)

def check_layout(rects, width, H):
    x, y, w, h = rects.T.astype(np.int64)
    assert (x >= 0).all() and (y >= 0).all() and (y + h <= H).all() and (x + w <= width).all()
    paint = np.zeros((H, max(width, 1)), np.int32)
    for r in rects:
        texels(paint, r)[:] += 1
    assert paint.max(initial=0) <= 1, "maps overlap"
    col_x, col_w, yy = 0, 0, 0
    for n in range(len(rects)):
        if x[n] != col_x:                      # a new column: the map did not fit below
            assert yy + h[n] > H
            assert x[n] == col_x + col_w and y[n] == 0
            col_x, col_w, yy = x[n], 0, 0
        assert y[n] == yy                      # stacked top to bottom
        yy += h[n]
        col_w = max(col_w, w[n])
    assert width == (col_x + col_w if len(rects) else 0)


@pytest.mark.parametrize("H", [40, 64, 200])
def test_layout_column_wise(oracle, H):
    spec = spec_aniso()
    tri = random_triangles(np.random.default_rng(7), 120, spec, edge=(0.005, 0.1))
    rects, width = oracle.texture_layout(tri, 0.004, H)
    assert rects[:, 3].max() <= H
    check_layout(rects, width, H)
    ncol = len(np.unique(rects[:, 0]))
    assert ncol >= (2 if H < 200 else 1)


def test_layout_edges(oracle):
    rects, width = oracle.texture_layout(np.zeros((0, 3, 3), np.float32), 0.01, 16)
    assert rects.shape == (0, 4) and width == 0
    tall = np.array([[[0, 0, 0], [0.01, 0, 0], [0, 0.5, 0]]], np.float32)
    with pytest.raises(ValueError):
        oracle.texture_layout(tall, 0.01, 16)                   # 50 rows > 16
    rects, width = oracle.texture_layout(tall, 0.01, 50)        # exactly fits
    assert tuple(rects[0]) == (0, 0, 2, 50) and width == 2
    huge = np.array([[[0, 0, 0], [700.0, 0, 0], [0, 0.01, 0]]], np.float32)
    with pytest.raises(ValueError):
        oracle.texture_layout(huge, 0.01, 16)                   # 70000 columns
