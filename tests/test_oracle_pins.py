"""Pins of the oracle against closed forms, invariants and an independent brute-force
implementation (CPU only).

Each pin is chosen so that a plausible mistake in the oracle (a dropped term, a wrong
sign or index, a transposed operand, a wrong rounding rule) fails at least one of them;
test_mutations.py checks that claim by planting such mistakes.
"""
import numpy as np
import pytest

import brute
from helpers import camera_volume, frames, intrinsics, plane_depth, posed, ramp_image
from kf_synth import configs
from kf_synth.scenes import VolumeSpec, default_rgb_extrinsic, rigid, rigid_inverse

K160 = intrinsics(131.25, 79.5, 59.5)
K320 = intrinsics(262.5, 159.5, 119.5)


def _run(O, vol, fr, dtype=np.float32, **kw):
    st = O.State(vol, dtype)
    cnt = O.integrate(vol, fr, st, **kw)
    return st, cnt


def _cam_coords(vol, dims, T_world_from_cam):
    pw = brute.voxel_centres(dims, vol.origin, vol.extent)
    T = np.linalg.inv(T_world_from_cam)
    return pw @ T[:3, :3].T + T[:3, 3]


# --------------------------------------------------------------------------- constants

def test_frame_constants_match_matrix_algebra(oracle):
    """The folded affine maps equal the 4x4 products of Eq. 5 and Eq. 3."""
    vol = camera_volume()
    T = posed()
    fr = frames(np.ones((120, 160)), np.zeros((240, 320, 3), np.uint8), K160, K320,
                default_rgb_extrinsic(), T, 0.03)
    fc = oracle.frame_consts(vol, fr, 0)
    s = np.asarray(vol.extent) / np.asarray(vol.gdim)
    T_cw = np.linalg.inv(T)
    for idx in [(0, 0, 0), (3, 17, 29), (31, 31, 31)]:
        pw = np.asarray(vol.origin) + (np.asarray(idx) + 0.5) * s
        pc = T_cw[:3, :3] @ pw + T_cw[:3, 3]
        np.testing.assert_allclose(fc["Ag"].reshape(3, 3) @ idx + fc["bg"], pc, atol=1e-14)
        sc = np.asarray(vol.extent) / np.asarray(vol.cdim)
        pw = np.asarray(vol.origin) + (np.asarray(idx) + 0.5) * sc
        pc = T_cw[:3, :3] @ pw + T_cw[:3, 3]
        np.testing.assert_allclose(fc["Ac"].reshape(3, 3) @ idx + fc["bc"], pc, atol=1e-14)
        q = fr.T_rgb_from_d[:3, :3] @ pc + fr.T_rgb_from_d[:3, 3]
        np.testing.assert_allclose(fc["Ah"].reshape(3, 3) @ idx + fc["bh"], q, atol=1e-14)
    assert fc["fx"] == 131.25 and fc["cy"] == 59.5 and fc["fxr"] == 262.5
    assert fc["sigma2"] == pytest.approx(0.02 ** 2, rel=1e-15)


# --------------------------------------------------------------------------- geometry

# FP32: the camera depth Z carries a few ulp(1) of rounding, amplified by 1/trunc.
@pytest.mark.parametrize("dtype,tol", [(np.float32, 1e-5), (np.float64, 1e-12)])
def test_plane_tsdf_closed_form(oracle, dtype, tol):
    """A fronto-parallel plane at d0 seen from a rotated, translated camera:
    F = min(1, (d0 - Z)/trunc) for every voxel in the band, weights count frames up to
    w_max, voxels behind the band or outside the frustum are never touched."""
    vol = camera_volume()
    T = posed()
    d0, trunc, n, w_max = 0.8, 0.0375, 7, 5
    fr = frames(np.full((n, 120, 160), d0), np.zeros((240, 320, 3), np.uint8), K160, K320,
                np.eye(4), T, trunc, w_max)
    st, cnt = _run(oracle, vol, fr, dtype)
    d0 = float(np.float32(d0))           # the depth map holds float32 metres
    pc = _cam_coords(vol, vol.gdim, T)
    x = 131.25 * pc[:, 0] / pc[:, 2] + 79.5
    y = 131.25 * pc[:, 1] / pc[:, 2] + 59.5
    inside = (np.rint(x) >= 0) & (np.rint(x) <= 159) & (np.rint(y) >= 0) & (np.rint(y) <= 119)
    clear = (np.abs(x - np.floor(x) - 0.5) > 1e-3) & (np.abs(y - np.floor(y) - 0.5) > 1e-3)
    sdf = d0 - pc[:, 2]
    band = inside & (sdf >= -trunc)
    sure = clear & (np.abs(sdf + trunc) > 1e-5)
    assert band.sum() > 1000 and (inside & ~band).sum() > 1000 and (~inside).sum() > 100
    np.testing.assert_array_equal(st.wg[band & sure], min(n, w_max))
    np.testing.assert_array_equal(st.wg[~band & sure], 0)
    np.testing.assert_allclose(st.tsdf[band & sure], np.minimum(1.0, sdf / trunc)[band & sure],
                               atol=tol, rtol=0)
    # repeats of the same frame leave F bit-equal to the single-frame value
    st1, _ = _run(oracle, vol, fr.select(0), dtype)
    np.testing.assert_array_equal(st.tsdf, st1.tsdf)
    assert cnt[0] == n * int((st.wg > 0).sum())


# --------------------------------------------------------------------------- colour

def _expected_plane_weight(vol, K, d0, W, H):
    """Closed form for the fronto-parallel plane at identity pose: w = Z/|P| at the
    voxel's depth pixel, i.e. 1/sqrt(((u-cx)/fx)^2 + ((v-cy)/fy)^2 + 1)."""
    pc = _cam_coords(vol, vol.cdim, np.eye(4))
    x = K[0, 0] * pc[:, 0] / pc[:, 2] + K[0, 2]
    y = K[1, 1] * pc[:, 1] / pc[:, 2] + K[1, 2]
    u, v = np.rint(x), np.rint(y)
    a = (u - K[0, 2]) / K[0, 0]
    b = (v - K[1, 2]) / K[1, 1]
    w = 1.0 / np.sqrt(a * a + b * b + 1.0)
    dist = np.sqrt((pc[:, 0] - a * d0) ** 2 + (pc[:, 1] - b * d0) ** 2 + (pc[:, 2] - d0) ** 2)
    ok = (u >= 0) & (u <= W - 2) & (v >= 0) & (v <= H - 2) & (dist <= 0.02)
    sure = (np.abs(x - np.floor(x) - 0.5) > 1e-3) & (np.abs(y - np.floor(y) - 0.5) > 1e-3) \
        & (np.abs(dist - 0.02) > 1e-5)
    return w, ok, sure


@pytest.mark.parametrize("dtype,tol", [(np.float32, 2e-5), (np.float64, 1e-12)])
def test_plane_colour_weight_recurrence(oracle, dtype, tol):
    """Static camera, fronto-parallel plane, wide field of view: W_m = 1 - (1 - w)^m while
    w > 0.8 W_{m-1}, and the colour weight freezes at the first frame that fails the gate
    (Eq. 8 normal, dot with the viewing direction, Eq. 10).  The slab-shaped volume is
    not a cube, which also exercises unequal dimensions."""
    K = intrinsics(60.0, 79.5, 59.5)
    Khd = intrinsics(60.0, 159.5, 119.5)
    vol = VolumeSpec((64, 48, 4), (128, 96, 8), (-0.8, -0.6, 0.76), (1.6, 1.2, 0.08))
    d0, m = 0.8, 6
    fr = frames(np.full((m, 120, 160), d0), np.full((240, 320, 3), 77, np.uint8), K, Khd,
                np.eye(4), np.eye(4), 0.05)
    st, _ = _run(oracle, vol, fr, dtype)
    w, ok, sure = _expected_plane_weight(vol, K, float(np.float32(d0)), 160, 120)
    W = np.zeros_like(w)
    for _ in range(m):
        W = np.where(w > 0.8 * W, W + w * (1.0 - W), W)
    # keep voxels whose HD sample is inside the HD image (identity extrinsic)
    pc = _cam_coords(vol, vol.cdim, np.eye(4))
    xh = 60.0 * pc[:, 0] / pc[:, 2] + 159.5
    yh = 60.0 * pc[:, 1] / pc[:, 2] + 119.5
    hd = (np.floor(xh) >= 0) & (np.floor(xh) <= 318) & (np.floor(yh) >= 0) & (np.floor(yh) <= 238)
    sel = ok & sure & hd
    assert sel.sum() > 500
    assert (w[sel] < 0.8).sum() > 50 and (w[sel] > 0.8).sum() > 50   # both regimes present
    frozen = sel & (W < 1.0 - (1.0 - w) ** m - 1e-3)
    assert frozen.sum() > 50                                          # the gate stopped them
    np.testing.assert_allclose(st.wc[sel], W[sel], atol=tol, rtol=0)
    np.testing.assert_array_equal(st.wc[~ok & sure], 0)


def test_tilted_plane_weight_orientation(oracle):
    """A plane tilted by 40 deg: the first colour weight is the cosine between the plane
    normal and the viewing ray, positive for a surface facing the camera."""
    th = np.radians(40.0)
    n = np.array([0.0, np.sin(th), np.cos(th)])
    d0 = 0.8
    vol = camera_volume(g=16, ratio=2, z0=0.55, size=0.5)
    D = plane_depth(K160, 160, 120, n, d0 * np.cos(th))
    D = np.where((D > 0) & (D < 3), D, 0)
    fr = frames(D, np.full((240, 320, 3), 50, np.uint8), K160, K320, np.eye(4), np.eye(4), 0.05)
    st, _ = _run(oracle, vol, fr, np.float32)
    bc = brute.colour(vol, fr.numpy(), brute.FP32_MARGINS)
    pc = _cam_coords(vol, vol.cdim, np.eye(4))
    upd = st.wc > 0
    assert upd.sum() > 300
    # expected: n . P / |P| with P the back-projected depth pixel of each voxel
    x = 131.25 * pc[:, 0] / pc[:, 2] + 79.5
    y = 131.25 * pc[:, 1] / pc[:, 2] + 59.5
    r = np.stack([(np.rint(x) - 79.5) / 131.25, (np.rint(y) - 59.5) / 131.25,
                  np.ones_like(x)], -1)
    w = (r @ n) / np.linalg.norm(r, axis=1)
    np.testing.assert_allclose(st.wc[upd], w[upd], atol=2e-4)
    assert (st.wc[upd] > 0.5).all()
    np.testing.assert_array_equal(upd[~bc["ambiguous"]], (bc["wc"] > 0)[~bc["ambiguous"]])


def test_constant_colour_is_exact(oracle):
    """A constant RGB8 image gives exactly byte * float32(1/255) in every observed voxel
    (lerp of equal values, then C + alpha * 0)."""
    vol, fr = configs.tiny()
    fr = fr.numpy()
    fr.rgb = np.empty_like(fr.rgb)
    fr.rgb[...] = np.array([200, 17, 99], np.uint8)
    st, _ = _run(oracle, vol, fr, np.float32)
    seen = st.wc > 0
    assert seen.sum() > 10000
    for arr, c in zip((st.r, st.g, st.b), (200, 17, 99)):
        np.testing.assert_array_equal(arr[seen], np.float32(c) * np.float32(1.0 / 255.0))
        np.testing.assert_array_equal(arr[~seen], 0)


# The image itself is stored in float32 (rounding <= 3e-8 per pixel).
@pytest.mark.parametrize("dtype,tol", [(np.float32, 1e-6), (np.float64, 1e-7)])
def test_ramp_image_pins_hd_projection(oracle, dtype, tol):
    """An affine F32 image R(x, y) is reproduced exactly by bilinear sampling, so each
    observed colour voxel equals R at the HD projection of its own centre (Eq. 3-5),
    not at the projection of the back-projected surface point."""
    T_rd = default_rgb_extrinsic()
    vol = camera_volume(g=16, ratio=3, z0=0.7, size=0.25)
    img = ramp_image(320, 240)
    fr = frames(np.full((3, 120, 160), 0.8), img, K160, K320, T_rd, np.eye(4), 0.05)
    st, _ = _run(oracle, vol, fr, dtype)
    pc = _cam_coords(vol, vol.cdim, np.eye(4))
    q = pc @ T_rd[:3, :3].T + T_rd[:3, 3]
    xh = 262.5 * q[:, 0] / q[:, 2] + 159.5
    yh = 262.5 * q[:, 1] / q[:, 2] + 119.5
    expect = 0.2 + 0.001 * xh + 0.0015 * yh
    seen = st.wc > 0
    assert seen.sum() > 500
    np.testing.assert_allclose(st.r[seen], expect[seen], atol=tol, rtol=0)
    # the surface-point reading would differ by much more than the tolerance
    x = 131.25 * pc[:, 0] / pc[:, 2] + 79.5
    y = 131.25 * pc[:, 1] / pc[:, 2] + 59.5
    P = np.stack([(np.rint(x) - 79.5) / 131.25 * 0.8, (np.rint(y) - 59.5) / 131.25 * 0.8,
                  np.full_like(x, 0.8)], -1)
    qs = P @ T_rd[:3, :3].T + T_rd[:3, 3]
    alt = 0.2 + 0.001 * (262.5 * qs[:, 0] / qs[:, 2] + 159.5) + 0.0015 * (262.5 * qs[:, 1] / qs[:, 2] + 119.5)
    assert np.abs(alt[seen] - expect[seen]).max() > 1e-3


def test_rgb8_and_float_inputs_agree_bitwise(oracle):
    """RGB8 is converted per pixel before interpolation, so the equivalent float image
    (byte * float32(1/255)) gives a bit-identical volume."""
    vol, fr = configs.tiny(n_frames=4)
    fr = fr.numpy()
    a, _ = _run(oracle, vol, fr, np.float32)
    b, _ = _run(oracle, vol, fr.as_float_rgb(), np.float32)
    for x, y in zip(a.arrays(), b.arrays()):
        np.testing.assert_array_equal(x, y)


# --------------------------------------------------------------------------- brute force

def _small_scan(n=3, g=16, ratio=2):
    vol, fr = configs.tiny(n_frames=n)
    vol = VolumeSpec.cube(g, ratio, 1.0)
    return vol, fr.numpy()


@pytest.mark.parametrize("g,ratio", [(16, 2), (24, 2), (16, 3)])
def test_brute_force_fp64(oracle, g, ratio):
    vol, fr = _small_scan(3, g, ratio)
    st, cnt = _run(oracle, vol, fr, np.float64)
    bg = brute.geometry(vol, fr)
    bc = brute.colour(vol, fr)
    okg, okc = ~bg["ambiguous"], ~bc["ambiguous"]
    assert okg.mean() > 0.99 and okc.mean() > 0.99
    assert (bg["wg"] > 0).sum() > 1000 and (bc["wc"] > 0).sum() > 300
    np.testing.assert_array_equal(st.wg[okg], bg["wg"][okg])
    np.testing.assert_allclose(st.tsdf[okg], bg["tsdf"][okg], atol=1e-9)
    for k in ("r", "g", "b", "wc"):
        np.testing.assert_allclose(getattr(st, k)[okc], bc[k][okc], atol=1e-9)
    # counters agree with the brute-force statuses
    assert cnt[0] == int((bg["status"] == 6).sum())
    assert cnt[2] == int((bc["status"] >= 4).sum())
    assert cnt[4] == int((bc["status"] == 6).sum())


def test_brute_force_fp32(oracle):
    vol, fr = _small_scan(3, 24, 2)
    st, _ = _run(oracle, vol, fr, np.float32)
    bg = brute.geometry(vol, fr, brute.FP32_MARGINS)
    bc = brute.colour(vol, fr, brute.FP32_MARGINS)
    okg, okc = ~bg["ambiguous"], ~bc["ambiguous"]
    assert okg.mean() > 0.95 and okc.mean() > 0.95
    np.testing.assert_array_equal(st.wg[okg], bg["wg"][okg])
    np.testing.assert_allclose(st.tsdf[okg], bg["tsdf"][okg], atol=1e-5)
    np.testing.assert_array_equal((st.wc > 0)[okc], (bc["wc"] > 0)[okc])
    np.testing.assert_allclose(st.wc[okc], bc["wc"][okc], atol=2e-3)
    for k in ("r", "g", "b"):
        np.testing.assert_allclose(getattr(st, k)[okc], bc[k][okc], atol=2e-3)


def test_status_codes_match_brute_force(oracle):
    vol, fr = _small_scan(3, 16, 3)
    bg = brute.geometry(vol, fr)
    bc = brute.colour(vol, fr)
    st = oracle.State(vol, np.float64)
    for f in range(fr.n):
        gs, cs = oracle.status(vol, fr, st, f)
        okg, okc = ~bg["ambiguous"], ~bc["ambiguous"]
        np.testing.assert_array_equal(gs[okg], bg["status"][f][okg])
        np.testing.assert_array_equal(cs[okc], bc["status"][f][okc])
        oracle.integrate(vol, fr.select(f), st)
    assert len(set(bc["status"].ravel().tolist())) >= 5


def test_world_translation_invariance(oracle):
    """Shifting the volume origin and every camera by the same vector changes nothing."""
    vol, fr = _small_scan(3, 16, 2)
    a, _ = _run(oracle, vol, fr, np.float64)
    tau = np.array([0.31, -0.17, 0.05])
    vol2 = VolumeSpec(vol.gdim, vol.cdim, tuple(np.asarray(vol.origin) + tau), vol.extent)
    fr2 = fr.select(slice(0, fr.n))
    fr2.T_world_from_cam = fr.T_world_from_cam.copy()
    fr2.T_world_from_cam[:, :3, 3] += tau
    b, _ = _run(oracle, vol2, fr2, np.float64)
    amb_g = brute.geometry(vol, fr)["ambiguous"]
    amb_c = brute.colour(vol, fr)["ambiguous"]
    np.testing.assert_allclose(a.tsdf[~amb_g], b.tsdf[~amb_g], atol=1e-9)
    np.testing.assert_array_equal(a.wg[~amb_g], b.wg[~amb_g])
    for k in ("r", "g", "b", "wc"):
        np.testing.assert_allclose(getattr(a, k)[~amb_c], getattr(b, k)[~amb_c], atol=1e-9)


def test_pass_union_counters(oracle):
    """Per-pass counters: with one pass over all frames, the touched counts equal the
    number of voxels with non-zero weight; with one frame per pass they equal the
    per-frame totals."""
    vol, fr = _small_scan(5, 16, 2)
    _, c1 = _run(oracle, vol, fr, np.float32, frames_per_pass=1)
    st, cn = _run(oracle, vol, fr, np.float32, frames_per_pass=fr.n)
    _, c2 = _run(oracle, vol, fr, np.float32, frames_per_pass=2)
    assert c1[1] == c1[0] and c1[3] == c1[2] and c1[5] == c1[4]
    assert cn[1] == int((st.wg > 0).sum()) and cn[5] == int((st.wc > 0).sum())
    assert cn[1] <= c2[1] <= c1[1] and cn[5] <= c2[5] <= c1[5]
    assert (c1[[0, 2, 4]] == cn[[0, 2, 4]]).all()


def test_slab_subset_equals_full(oracle):
    """Voxels are independent: integrating a z-slab range alone gives the same values."""
    vol, fr = _small_scan(3, 16, 2)
    full, _ = _run(oracle, vol, fr, np.float32)
    part = oracle.State(vol, np.float32, gz=(5, 11), cz=(9, 23))
    oracle.integrate(vol, fr, part)
    ng = 16 * 16
    nc = 32 * 32
    np.testing.assert_array_equal(part.tsdf, full.tsdf[5 * ng:11 * ng])
    np.testing.assert_array_equal(part.wc, full.wc[9 * nc:23 * nc])
    np.testing.assert_array_equal(part.g, full.g[9 * nc:23 * nc])


def test_holes_and_invalid_depth_are_skipped(oracle):
    """Zero, negative, NaN and infinite depth pixels are holes: no voxel reading one is
    updated (Sec. IV.B only uses non-zero depth)."""
    vol = camera_volume(g=16, ratio=2)
    D = np.full((120, 160), 0.8, np.float32)
    D[:, :50] = 0.0
    D[:, 50:60] = np.nan
    D[:, 60:70] = -1.0
    D[:, 70:80] = np.inf
    fr = frames(D, np.full((240, 320, 3), 9, np.uint8), K160, K320, np.eye(4), np.eye(4), 0.03)
    st, _ = _run(oracle, vol, fr, np.float32)
    pc = _cam_coords(vol, vol.gdim, np.eye(4))
    u = np.rint(131.25 * pc[:, 0] / pc[:, 2] + 79.5)
    assert (st.wg[u < 79] == 0).all() and (st.wg[u > 81] > 0).any()
    pcc = _cam_coords(vol, vol.cdim, np.eye(4))
    uc = np.rint(131.25 * pcc[:, 0] / pcc[:, 2] + 79.5)
    assert (st.wc[uc < 80] == 0).all() and (st.wc[uc > 81] > 0).any()


def test_brute_force_anisotropic_intrinsics(oracle):
    """Unequal focal lengths and an off-centre principal point on both cameras, so that a
    swapped x/y intrinsic anywhere shows up (the scan itself need not be consistent
    with them: the integration only reads the numbers)."""
    vol, fr = _small_scan(3, 16, 3)
    fr.K_d = np.array([[140.0, 0.0, 83.25], [0.0, 124.0, 57.75], [0.0, 0.0, 1.0]])
    fr.K_rgb = np.array([[281.0, 0.0, 150.5], [0.0, 246.5, 124.0], [0.0, 0.0, 1.0]])
    st, _ = _run(oracle, vol, fr, np.float64)
    bg = brute.geometry(vol, fr)
    bc = brute.colour(vol, fr)
    okg, okc = ~bg["ambiguous"], ~bc["ambiguous"]
    assert (bc["wc"] > 0).sum() > 300
    np.testing.assert_array_equal(st.wg[okg], bg["wg"][okg])
    np.testing.assert_allclose(st.tsdf[okg], bg["tsdf"][okg], atol=1e-9)
    for k in ("r", "g", "b", "wc"):
        np.testing.assert_allclose(getattr(st, k)[okc], bc[k][okc], atol=1e-9)
