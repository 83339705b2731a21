"""Pins of the oracle's FP64 adjoint of the colour update (CPU only).

L = sum_v sum_ch g[ch][v] C_N(v)_ch.  Eq. 9 makes C_N linear in the HD pixel values
with weights that do not depend on them, and Eq. 3-4 make it smooth in the RGB
extrinsic away from bilinear cell borders; the pins below check the adjoint against
exact linearity, conservation, a constant image and FP64 central differences.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import brute
from helpers import frames, ramp_image
from kf_synth import configs
from kf_synth.scenes import VolumeSpec


def hat(xi):
    """4x4 twist of xi = (rho, phi)."""
    rho, phi = xi[:3], xi[3:]
    M = np.zeros((4, 4))
    M[:3, :3] = [[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]]
    M[:3, 3] = rho
    return M


def _scan(n=4, g=16, ratio=2):
    vol, fr = configs.tiny(n_frames=n)
    vol = VolumeSpec.cube(g, ratio, 1.0)
    return vol, fr.numpy().as_float_rgb()


def _loss(O, vol, fr, g):
    st = O.State(vol, np.float64)
    O.integrate(vol, fr, st)
    return float(np.sum(g[0] * st.r) + np.sum(g[1] * st.g) + np.sum(g[2] * st.b)), st


def test_rgb_gradient_is_exact_linearity(oracle):
    vol, fr = _scan()
    rng = np.random.default_rng(7)
    g = rng.standard_normal((3, vol.n_colour))
    d_rgb, _ = oracle.backward(vol, fr, g)
    L0, _ = _loss(oracle, vol, fr, g)
    nz = np.argwhere(np.abs(d_rgb) > 1e-3)
    assert len(nz) > 100
    for f, y, x, c in nz[rng.choice(len(nz), 6, replace=False)]:
        fr2 = fr.select(slice(0, fr.n))
        fr2.rgb = fr.rgb.copy()
        old = np.float64(fr2.rgb[f, y, x, c])
        fr2.rgb[f, y, x, c] = np.float32(old + 0.25)
        delta = np.float64(fr2.rgb[f, y, x, c]) - old
        L1, _ = _loss(oracle, vol, fr2, g)
        assert (L1 - L0) / delta == pytest.approx(d_rgb[f, y, x, c], rel=1e-9, abs=1e-12)
    # untouched pixels have exactly zero gradient
    assert (d_rgb == 0).mean() > 0.5


def test_rgb_gradient_conservation(oracle):
    """The first update of a voxel has alpha = 1, so the beta_n of a voxel sum to one and
    the image gradient of each channel sums to the g of the observed voxels."""
    vol, fr = _scan()
    rng = np.random.default_rng(8)
    g = rng.standard_normal((3, vol.n_colour))
    d_rgb, _ = oracle.backward(vol, fr, g)
    _, st = _loss(oracle, vol, fr, g)
    seen = st.wc > 0
    for c in range(3):
        assert d_rgb[..., c].sum() == pytest.approx(g[c][seen].sum(), rel=1e-10, abs=1e-10)


def test_constant_image_has_zero_pose_gradient(oracle):
    vol, fr = _scan()
    fr.rgb = np.full_like(fr.rgb, 0.4)
    g = np.random.default_rng(9).standard_normal((3, vol.n_colour))
    _, d_xi = oracle.backward(vol, fr, g)
    assert (d_xi == 0).all()


def _loss_at(oracle, vol, fr, g, xi):
    fr2 = fr.select(slice(0, fr.n))
    fr2.T_rgb_from_d = expm(hat(xi)) @ fr.T_rgb_from_d
    return _loss(oracle, vol, fr2, g)[0]


def _fd(oracle, vol, fr, g, h=1e-4):
    out = np.zeros(6)
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        out[k] = (_loss_at(oracle, vol, fr, g, e) - _loss_at(oracle, vol, fr, g, -e)) / (2 * h)
    return out


def test_pose_gradient_ramp_image_central_differences(oracle):
    """On an affine image bilinear sampling is globally affine, so L is smooth in xi
    except at the HD border; the adjoint must match FP64 central differences."""
    vol, fr = _scan(n=3)
    fr.rgb = np.repeat(ramp_image(320, 240, 0.1, 0.0021, -0.0013)[None], fr.n, axis=0)
    fr.rgb[..., 1] = ramp_image(320, 240, 0.3, -0.0007, 0.0017)[..., 0]
    g = np.random.default_rng(10).standard_normal((3, vol.n_colour))
    # keep the HD border out of reach of the perturbation
    rec = brute.colour(vol, fr, record=True)["frames"]
    margin = np.zeros(vol.n_colour, bool)
    for r in rec:
        near = (r["xh"] < 3) | (r["xh"] > 316) | (r["yh"] < 3) | (r["yh"] > 236)
        margin |= near
    g[:, margin] = 0.0
    _, d_xi = oracle.backward(vol, fr, g)
    fd = _fd(oracle, vol, fr, g)
    assert np.abs(fd).max() > 1e-2
    np.testing.assert_allclose(d_xi, fd, rtol=1e-3, atol=1e-3 * np.abs(fd).max())


def test_pose_gradient_textured_image_central_differences(oracle):
    """64 seeded voxels whose HD samples keep their bilinear cell, update mask and border
    status under every +-h perturbation (h = 1e-4 per se(3) component)."""
    vol, fr = _scan(n=4, g=24, ratio=2)
    h = 1e-4
    base = brute.colour(vol, fr, record=True)
    keep = base["wc"] > 0
    for k in range(6):
        for sgn in (-1, 1):
            e = np.zeros(6)
            e[k] = sgn * h
            fr2 = fr.select(slice(0, fr.n))
            fr2.T_rgb_from_d = expm(hat(e)) @ fr.T_rgb_from_d
            rec = brute.colour(vol, fr2, record=True)["frames"]
            for r0, r1 in zip(base["frames"], rec):
                keep &= (r0["upd"] == r1["upd"])
                keep &= ~r0["upd"] | ((r0["x0"] == r1["x0"]) & (r0["y0"] == r1["y0"]))
    for r0 in base["frames"]:
        keep &= ~r0["upd"] | ((r0["ax"] > 0.02) & (r0["ax"] < 0.98) & (r0["ay"] > 0.02) & (r0["ay"] < 0.98))
    cand = np.flatnonzero(keep)
    assert len(cand) >= 64
    rng = np.random.default_rng(5005)
    sel = rng.choice(cand, 64, replace=False)
    g = np.zeros((3, vol.n_colour))
    g[:, sel] = rng.standard_normal((3, 64))
    _, d_xi = oracle.backward(vol, fr, g)
    fd = _fd(oracle, vol, fr, g, h)
    assert np.abs(fd).max() > 1e-3
    np.testing.assert_allclose(d_xi, fd, rtol=1e-3, atol=1e-3 * np.abs(fd).max())


def test_backward_from_nonzero_initial_weights(oracle):
    """Starting weights change alpha of the first update (no longer 1): the adjoint
    still matches exact linearity in the pixels."""
    vol, fr = _scan(n=3)
    rng = np.random.default_rng(11)
    wc0 = rng.uniform(0.0, 0.6, vol.n_colour)
    g = rng.standard_normal((3, vol.n_colour))
    d_rgb, _ = oracle.backward(vol, fr, g, wc0=wc0)

    def loss(rgb):
        fr2 = fr.select(slice(0, fr.n))
        fr2.rgb = rgb
        st = oracle.State(vol, np.float64)
        st.wc[:] = wc0
        oracle.integrate(vol, fr2, st)
        return float(np.sum(g[0] * st.r) + np.sum(g[1] * st.g) + np.sum(g[2] * st.b))

    L0 = loss(fr.rgb)
    nz = np.argwhere(np.abs(d_rgb) > 1e-3)
    for f, y, x, c in nz[rng.choice(len(nz), 4, replace=False)]:
        rgb = fr.rgb.copy()
        old = np.float64(rgb[f, y, x, c])
        rgb[f, y, x, c] = np.float32(old + 0.25)
        delta = np.float64(rgb[f, y, x, c]) - old
        assert (loss(rgb) - L0) / delta == pytest.approx(d_rgb[f, y, x, c], rel=1e-9, abs=1e-12)


def test_fp32_decision_mode_agrees_away_from_ties(oracle):
    """The adjoint with the FP32 forward's integer decisions equals the all-FP64 adjoint
    on voxels whose decisions are not within rounding of a threshold in any frame."""
    vol, fr = _scan(n=5, g=24, ratio=2)
    amb = brute.colour(vol, fr, brute.FP32_MARGINS)["ambiguous"]
    g = np.random.default_rng(12).standard_normal((3, vol.n_colour))
    g[:, amb] = 0.0
    r64, x64 = oracle.backward(vol, fr, g)
    r32, x32 = oracle.backward(vol, fr, g, decide_f32=True)
    assert np.abs(x64).max() > 1e-2
    np.testing.assert_allclose(x32, x64, rtol=1e-3, atol=1e-3 * np.abs(x64).max())
    np.testing.assert_allclose(r32, r64, rtol=1e-3, atol=1e-3 * np.abs(r64).max())


# ---- depth-camera poses: T_world_from_cam[n] <- exp(xi_n^) T_world_from_cam[n]

def _pose_perturbed(fr, f, xi):
    fr2 = fr.select(slice(0, fr.n))
    fr2.T_world_from_cam = fr.T_world_from_cam.copy()
    fr2.T_world_from_cam[f] = expm(hat(xi)) @ fr.T_world_from_cam[f]
    return fr2


def test_depth_pose_gradient_central_differences(oracle):
    """64 seeded voxels whose depth pixels, update masks and bilinear cells stay put under
    every +-h perturbation of every frame's pose; per-frame gradients against FP64 central
    differences."""
    vol, fr = _scan(n=3, g=24, ratio=2)
    h = 1e-4
    base = brute.colour(vol, fr, record=True)
    keep = base["wc"] > 0
    for f in range(fr.n):
        for k in range(6):
            for sgn in (-1, 1):
                e = np.zeros(6)
                e[k] = sgn * h
                rec = brute.colour(vol, _pose_perturbed(fr, f, e), record=True)["frames"]
                for r0, r1 in zip(base["frames"], rec):
                    keep &= r0["upd"] == r1["upd"]
                    keep &= ~r0["upd"] | ((r0["x0"] == r1["x0"]) & (r0["y0"] == r1["y0"]) &
                                          (r0["u"] == r1["u"]) & (r0["v"] == r1["v"]))
    for r0 in base["frames"]:
        keep &= ~r0["upd"] | ((r0["ax"] > 0.02) & (r0["ax"] < 0.98) & (r0["ay"] > 0.02) & (r0["ay"] < 0.98))
    cand = np.flatnonzero(keep)
    assert len(cand) >= 64
    rng = np.random.default_rng(5006)
    sel = rng.choice(cand, 64, replace=False)
    g = np.zeros((3, vol.n_colour))
    g[:, sel] = rng.standard_normal((3, 64))
    _, _, d_pose = oracle.backward(vol, fr, g, pose=True)
    fd = np.zeros((fr.n, 6))
    for f in range(fr.n):
        for k in range(6):
            e = np.zeros(6)
            e[k] = h
            lp = _loss(oracle, vol, _pose_perturbed(fr, f, e), g)[0]
            lm = _loss(oracle, vol, _pose_perturbed(fr, f, -e), g)[0]
            fd[f, k] = (lp - lm) / (2 * h)
    assert np.abs(fd).max() > 1e-3
    np.testing.assert_allclose(d_pose, fd, rtol=1e-3, atol=1e-3 * np.abs(fd).max())


def test_depth_pose_and_extrinsic_adjoints_agree(oracle):
    """With one frame, perturbing the pose by xi moves the HD-camera point as perturbing the
    extrinsic by -Ad(T_hd_from_world) xi: d_pose = -Ad^T d_xi (two derivations of the same
    chain: through the world point, and through the HD-camera point)."""
    vol, fr = _scan(n=1, g=24, ratio=2)
    g = np.random.default_rng(12).standard_normal((3, vol.n_colour))
    _, d_xi, d_pose = oracle.backward(vol, fr, g, pose=True)
    T = fr.T_rgb_from_d @ np.linalg.inv(fr.T_world_from_cam[0])
    R, t = T[:3, :3], T[:3, 3]
    tx = np.array([[0, -t[2], t[1]], [t[2], 0, -t[0]], [-t[1], t[0], 0]])
    Ad = np.block([[R, tx @ R], [np.zeros((3, 3)), R]])
    assert np.abs(d_xi).max() > 1e-2
    np.testing.assert_allclose(d_pose[0], -Ad.T @ d_xi, rtol=1e-9, atol=1e-9 * np.abs(d_xi).max())


def test_constant_image_has_zero_depth_pose_gradient(oracle):
    vol, fr = _scan()
    fr.rgb = np.full_like(fr.rgb, 0.4)
    g = np.random.default_rng(9).standard_normal((3, vol.n_colour))
    _, _, d_pose = oracle.backward(vol, fr, g, pose=True)
    assert d_pose.shape == (fr.n, 6) and (d_pose == 0).all()
