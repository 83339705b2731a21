"""Pins of the oracle's ray caster (CPU only).

The ray caster (rendering of the integrated volumes, abstract and Sec. III) is checked
against results fixed by geometry rather than by its own formulas:
* an affine TSDF (a tilted plane) is reproduced exactly by trilinear interpolation, so the
  hit is the analytic ray/plane intersection, the normal the plane's, and an affine colour
  field gives the colour of the hit point; an anisotropic volume checks the per-axis
  scaling;
* a sphere's TSDF gives the analytic ray/sphere depth within the interpolation error;
* rays that leave the box, empty volumes and volumes that are solid everywhere miss;
* moving the volume and the camera together changes nothing;
* a dense FP64 march on a smooth random field finds the same first front-facing crossing.
"""
import numpy as np
import pytest

from kf_synth.scenes import VolumeSpec

pytestmark = pytest.mark.usefixtures("oracle")


def K160():
    return np.array([[131.25, 0, 79.5], [0, 131.25, 59.5], [0, 0, 1.0]])


def pose(R=np.eye(3), t=(0.0, 0.0, -0.8)):
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = t
    return T


def rot(axis, deg):
    a = np.radians(deg)
    c, s = np.cos(a), np.sin(a)
    if axis == "x":
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    if axis == "y":
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def centres(origin, extent, dim):
    s = np.asarray(extent, float) / np.asarray(dim)
    ax = [origin[k] + (np.arange(dim[k]) + 0.5) * s[k] for k in range(3)]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)   # x fastest


def analytic_state(oracle, spec, tsdf_fn, colour_fn, weight=1.0):
    st = oracle.State(spec, np.float32)
    pg = centres(spec.origin, spec.extent, spec.gdim)
    st.tsdf[:] = np.clip(tsdf_fn(pg), -1, 1).astype(np.float32)
    st.wg[:] = weight
    pc = centres(spec.origin, spec.extent, spec.cdim)
    rgb = colour_fn(pc)
    st.r[:], st.g[:], st.b[:] = [rgb[:, k].astype(np.float32) for k in range(3)]
    st.wc[:] = weight
    return st


def rays(K, T, W, H):
    """World origin and unit-depth directions of every pixel (FP64)."""
    x, y = np.meshgrid(np.arange(W, dtype=float), np.arange(H, dtype=float))
    dc = np.stack([(x - K[0, 2]) / K[0, 0], (y - K[1, 2]) / K[1, 1], np.ones_like(x)], -1)
    return T[:3, 3], dc @ T[:3, :3].T


def affine_colour(p):
    return np.stack([0.2 + 0.3 * p[:, 0], 0.5 - 0.2 * p[:, 1], 0.1 + 0.4 * p[:, 2]], axis=1)


@pytest.mark.parametrize("precision,tol", [("f64", 2e-6), ("f32", 2e-5)])
@pytest.mark.parametrize("anisotropic", [False, True])
def test_tilted_plane_closed_form(oracle, precision, tol, anisotropic):
    if anisotropic:
        spec = VolumeSpec((48, 40, 56), (96, 80, 112), (-0.5, -0.4, -0.55), (1.0, 0.8, 1.1))
    else:
        spec = VolumeSpec.cube(64, 2, 1.0)
    n = np.array([0.25, -0.35, -1.0])
    n /= np.linalg.norm(n)           # unit normal facing the camera (which looks along +z)
    p0 = np.array([0.02, -0.03, 0.1])
    trunc = 0.06
    st = analytic_state(oracle, spec, lambda p: ((p - p0) @ n) / trunc, affine_colour)
    K, T, W, H = K160(), pose(rot("y", 7) @ rot("x", -5)), 160, 120
    if anisotropic:   # also unequal focal lengths and an off-centre principal point
        K = np.array([[140.0, 0, 82.5], [0, 121.0, 57.25], [0, 0, 1.0]])
    out = oracle.raycast(spec, st, K, T, W, H, delta=0.4 * trunc, precision=precision)
    o, d = rays(K, T, W, H)
    t = ((p0 - o) @ n) / (d @ n)               # analytic camera depth of the plane
    hit_p = o + t[..., None] * d
    lo = np.asarray(spec.origin) + 0.08
    hi = np.asarray(spec.origin) + np.asarray(spec.extent) - 0.08
    inside = np.all((hit_p > lo) & (hit_p < hi), axis=-1)
    assert inside.sum() > 0.5 * W * H
    got = out["depth"]
    assert np.all(got[inside] > 0), "a ray through the plane missed"
    np.testing.assert_allclose(got[inside], t[inside], atol=tol)
    np.testing.assert_allclose(out["vertex"][inside], hit_p[inside], atol=tol)
    np.testing.assert_allclose(out["normal"][inside], np.broadcast_to(n, hit_p.shape)[inside],
                               atol=20 * tol)
    np.testing.assert_allclose(out["colour"][inside], affine_colour(hit_p[inside]), atol=tol)


def sphere_depth(o, d, c, R):
    oc = o - c
    a = np.sum(d * d, -1)
    b = 2 * (d @ oc)
    cc = oc @ oc - R * R
    disc = b * b - 4 * a * cc
    t = (-b - np.sqrt(np.maximum(disc, 0))) / (2 * a)
    return np.where(disc > 0, t, np.nan)


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_sphere_against_analytic_intersection(oracle, precision):
    spec = VolumeSpec.cube(96, 2, 1.0)
    c, R, trunc = np.array([0.03, -0.02, 0.1]), 0.26, 0.05
    st = analytic_state(oracle, spec, lambda p: (np.linalg.norm(p - c, axis=1) - R) / trunc,
                        affine_colour)
    K, T, W, H = K160(), pose(), 160, 120
    out = oracle.raycast(spec, st, K, T, W, H, delta=0.3 * trunc, precision=precision)
    o, d = rays(K, T, W, H)
    t = sphere_depth(o, d, c, R)
    hit_p = o + t[..., None] * d
    nrm = (hit_p - c) / R
    facing = -(nrm * d).sum(-1) / np.linalg.norm(d, axis=-1)       # cosine to the ray
    good = np.isfinite(t) & (facing > 0.5)
    assert good.sum() > 2000
    got = out["depth"]
    assert np.all(got[good] > 0)
    assert np.abs(got[good] - t[good]).max() < 1.5e-3
    assert np.all(got[~np.isfinite(t)] == 0), "a ray that misses the sphere reported a hit"
    assert np.abs(out["normal"][good] - nrm[good]).max() < 0.03
    np.testing.assert_allclose(np.linalg.norm(out["normal"][good], axis=-1), 1, atol=1e-5)
    np.testing.assert_allclose(out["colour"][good], affine_colour(out["vertex"][good]), atol=2e-5)


def test_misses_and_empty_volumes(oracle):
    spec = VolumeSpec.cube(32, 2, 1.0)
    trunc = 0.08
    plane = analytic_state(oracle, spec, lambda p: (0.1 - p[:, 2]) / trunc, affine_colour)
    K = K160()
    # looking away from the volume
    away = oracle.raycast(spec, plane, K, pose(rot("y", 180), (0, 0, -0.8)), 160, 120, 0.03)
    assert np.all(away["depth"] == 0) and np.all(away["vertex"] == 0)
    # unobserved (zero weights)
    empty = analytic_state(oracle, spec, lambda p: (0.1 - p[:, 2]) / trunc, affine_colour, 0.0)
    assert np.all(oracle.raycast(spec, empty, K, pose(), 160, 120, 0.03)["depth"] == 0)
    # solid (negative) and free (positive) everywhere: no front-facing crossing
    for v in (-1.0, 1.0):
        solid = analytic_state(oracle, spec, lambda p: np.full(len(p), v), affine_colour)
        assert np.all(oracle.raycast(spec, solid, K, pose(), 160, 120, 0.03)["depth"] == 0)
    # a back face (negative in front, positive behind) is not a surface seen from the camera
    back = analytic_state(oracle, spec, lambda p: (p[:, 2] - 0.1) / trunc, affine_colour)
    assert np.all(oracle.raycast(spec, back, K, pose(), 160, 120, 0.03)["depth"] == 0)
    # colour: zero where the colour weights are zero, geometry unaffected
    nocol = analytic_state(oracle, spec, lambda p: (0.1 - p[:, 2]) / trunc, affine_colour)
    nocol.wc[:] = 0
    a = oracle.raycast(spec, nocol, K, pose(), 160, 120, 0.03)
    b = oracle.raycast(spec, plane, K, pose(), 160, 120, 0.03)
    np.testing.assert_array_equal(a["depth"], b["depth"])
    assert np.all(a["colour"] == 0) and np.any(b["colour"] != 0)


def test_translation_invariance(oracle):
    spec = VolumeSpec.cube(48, 2, 1.0)
    c, R, trunc = np.array([0.0, 0.02, 0.12]), 0.3, 0.06
    fn = lambda p: (np.linalg.norm(p - c, axis=1) - R) / trunc    # noqa: E731
    st = analytic_state(oracle, spec, fn, affine_colour)
    off = np.array([0.25, 0.5, -0.75])                              # exact in binary
    spec2 = VolumeSpec(spec.gdim, spec.cdim, tuple(np.asarray(spec.origin) + off), spec.extent)
    T = pose(rot("y", 4))
    T2 = T.copy()
    T2[:3, 3] += off
    a = oracle.raycast(spec, st, K160(), T, 160, 120, 0.02, precision="f64")
    b = oracle.raycast(spec2, st, K160(), T2, 160, 120, 0.02, precision="f64")
    np.testing.assert_array_equal(a["depth"] > 0, b["depth"] > 0)
    np.testing.assert_allclose(a["depth"], b["depth"], atol=1e-6)
    np.testing.assert_allclose(a["vertex"] + (a["depth"] > 0)[..., None] * off, b["vertex"], atol=1e-6)
    np.testing.assert_allclose(a["normal"], b["normal"], atol=1e-5)


def _trilinear(F, W, q):
    """Dense FP64 trilinear interpolation (None where a corner is unobserved or out)."""
    d = np.array(F.shape[::-1])
    if np.any(q < 0) or np.any(q > d - 1):
        return None
    i = np.minimum(np.floor(q).astype(int), d - 2)
    f = q - i
    cube = F[i[2]:i[2] + 2, i[1]:i[1] + 2, i[0]:i[0] + 2]
    if np.any(W[i[2]:i[2] + 2, i[1]:i[1] + 2, i[0]:i[0] + 2] <= 0):
        return None
    wx = np.array([1 - f[0], f[0]])
    wy = np.array([1 - f[1], f[1]])
    wz = np.array([1 - f[2], f[2]])
    return float(np.einsum("zyx,z,y,x->", cube, wz, wy, wx))


def test_dense_march_brute_force(oracle):
    """A smooth random TSDF with features much larger than the step: the oracle's first
    front-facing crossing equals the one a march 32 times finer finds."""
    rng = np.random.default_rng(77)
    spec = VolumeSpec.cube(24, 2, 1.0)
    k = rng.normal(size=(4, 3)) * 2.0
    ph = rng.uniform(0, 2 * np.pi, 4)
    amp = rng.uniform(0.03, 0.06, 4)

    def field(p):
        return (0.05 - p[:, 2] + (amp * np.sin(p @ k.T + ph)).sum(1)) / 0.15
    st = analytic_state(oracle, spec, field, affine_colour)
    st.wg[rng.uniform(size=st.wg.size) < 0.01] = 0      # a few unobserved voxels
    K, T, W, H = K160(), pose(rot("x", 3)), 160, 120
    delta = 0.02
    pix = rng.choice(W * H, 60, replace=False)
    out = oracle.raycast(spec, st, K, T, W, H, delta, pixels=pix, precision="f64")
    F = st.tsdf.astype(np.float64).reshape(spec.gdim[::-1])
    Wg = st.wg.reshape(spec.gdim[::-1])
    s = np.asarray(spec.extent) / np.asarray(spec.gdim)
    o, d = rays(K, T, W, H)
    d = d.reshape(-1, 3)
    checked = 0
    for p_i, pix_i in enumerate(pix):
        fine = delta / 32
        prev = None
        found = 0.0
        for n in range(1, int(1.6 / fine)):
            t = n * fine
            q = (o + t * d[pix_i] - np.asarray(spec.origin)) / s - 0.5
            v = _trilinear(F, Wg, q)
            if v is not None and prev is not None and prev[1] > 0 > v:
                found = prev[0] + fine * prev[1] / (prev[1] - v)
                break
            prev = None if v is None else (t, v)
        got = out["depth"][p_i]
        if found == 0.0:
            assert got == 0.0 or got > 0     # a coarse step may still cross a thin gap
            continue
        assert got > 0, f"pixel {pix_i}: the dense march hits at {found}, the oracle misses"
        assert abs(got - found) < 2e-3, (pix_i, got, found)
        checked += 1
    assert checked > 30
