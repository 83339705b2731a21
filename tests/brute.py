"""Brute-force FP64 implementation of the integration, written independently of the C
oracle and used only to pin it.

It takes the paper's equations literally on whole arrays of voxels with NumPy:
4x4 homogeneous transforms and an explicit inverse of K_c (Eq. 1, 5, 7), the
homogeneous projection (x, y, z) = K (X, Y, Z) followed by the division (Eq. 4, 6),
the normal as an explicit cross product (Eq. 8), the colour update in its fractional
form (C W_pre + W HD) / (W_pre + W) (Eq. 9), the weight update of Eq. 10, and the TSDF
running average (F W + t) / (W + 1) of KinectFusion (Sec. III).  Bilinear sampling is
written as the four-weight sum.

Besides the final state it reports, per voxel, whether any decision of any frame came
within a margin of its threshold (a rounding tie of the pixel, the truncation or sigma
boundary, the weight gate, an HD cell border); such voxels may legitimately differ
between precisions and are excluded from element-wise comparisons.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Margins:
    px: float = 1e-6       # pixel coordinate distance to a rounding / flooring boundary
    dist: float = 1e-9     # metres, for the truncation and sigma tests
    w: float = 1e-9        # the weight gate


FP32_MARGINS = Margins(px=2e-3, dist=2e-5, w=2e-3)


def voxel_centres(dim, origin, extent):
    """World coordinates of every voxel centre, x fastest: shape (N, 3)."""
    s = np.asarray(extent, float) / np.asarray(dim, float)
    k, j, i = np.indices((dim[2], dim[1], dim[0])).reshape(3, -1)
    idx = np.stack([i, j, k], axis=1).astype(float)
    return np.asarray(origin, float) + (idx + 0.5) * s


def _homog(p):
    return np.concatenate([p, np.ones((p.shape[0], 1))], axis=1)


def _near_half(x, m):
    """True where x lies within m of a rint tie (k + 1/2)."""
    return np.abs((x - np.floor(x)) - 0.5) < m


def _near_int(x, m):
    return np.abs(x - np.round(x)) < m


def _depth_lookup(D, u, v, ok):
    H, W = D.shape
    uu = np.where(ok, u, 0).astype(np.int64)
    vv = np.where(ok, v, 0).astype(np.int64)
    return np.where(ok, D[np.clip(vv, 0, H - 1), np.clip(uu, 0, W - 1)], 0.0)


def _valid(d):
    return np.isfinite(d) & (d > 0)


def project_depth(K, pc, W, H, m: Margins):
    """Eq. 6 then the perspective division and nearest pixel; returns (u, v, inside, amb)."""
    hom = (K @ pc.T).T
    with np.errstate(divide="ignore", invalid="ignore"):
        x = hom[:, 0] / hom[:, 2]
        y = hom[:, 1] / hom[:, 2]
    u, v = np.rint(x), np.rint(y)
    front = pc[:, 2] > 0
    inside = front & (u >= 0) & (u <= W - 1) & (v >= 0) & (v <= H - 1)
    amb = front & (_near_half(x, m.px) | _near_half(y, m.px))
    return u, v, inside, amb


def geometry(vol, fr, m: Margins = Margins()):
    with np.errstate(all="ignore"):
        return _geometry(vol, fr, m)


def _geometry(vol, fr, m):
    pw = voxel_centres(vol.gdim, vol.origin, vol.extent)
    n = pw.shape[0]
    F = np.zeros(n)
    Wg = np.zeros(n)
    amb = np.zeros(n, bool)
    status = np.zeros((fr.n, n), np.uint8)
    D_all = np.asarray(fr.depth, np.float64)
    for f in range(fr.n):
        T_cw = np.linalg.inv(fr.T_world_from_cam[f])
        pc = (T_cw @ _homog(pw).T).T[:, :3]
        H, W = D_all[f].shape
        u, v, inside, a = project_depth(fr.K_d, pc, W, H, m)
        d = _depth_lookup(D_all[f], u, v, inside)
        ok = inside & _valid(d)
        sdf = d - pc[:, 2]
        upd = ok & (sdf >= -fr.trunc)
        a |= ok & (np.abs(sdf + fr.trunc) < m.dist)
        amb |= a
        t = np.minimum(1.0, sdf / fr.trunc)
        Fn = (F * Wg + t) / (Wg + 1.0)
        F = np.where(upd, Fn, F)
        Wg = np.where(upd, np.minimum(Wg + 1.0, fr.w_max), Wg)
        st = np.where(~inside, 0, np.where(~_valid(d), 1, np.where(upd, 6, 2)))
        status[f] = st
    return dict(tsdf=F, wg=Wg, ambiguous=amb, status=status)


def bilinear(img, xh, yh):
    """Four-weight bilinear sample of an (H, W, 3) image at (xh, yh); returns (N, 3),
    the cell, the fractions and the spatial gradient (d/dx, d/dy)."""
    x0 = np.floor(xh).astype(np.int64)
    y0 = np.floor(yh).astype(np.int64)
    ax = (xh - x0)[:, None]
    ay = (yh - y0)[:, None]
    p00 = img[y0, x0]
    p10 = img[y0, x0 + 1]
    p01 = img[y0 + 1, x0]
    p11 = img[y0 + 1, x0 + 1]
    s = (1 - ax) * (1 - ay) * p00 + ax * (1 - ay) * p10 + (1 - ax) * ay * p01 + ax * ay * p11
    gx = (1 - ay) * (p10 - p00) + ay * (p11 - p01)
    gy = (1 - ax) * (p01 - p00) + ax * (p11 - p10)
    return s, x0, y0, ax[:, 0], ay[:, 0], gx, gy


def colour(vol, fr, m: Margins = Margins(), wc0=None, record=False):
    """Colour volume after all frames.  With record=True also returns, per frame, the
    update mask, alpha, HD coordinates, HD-camera point q and the image gradient."""
    with np.errstate(all="ignore"):
        return _colour(vol, fr, m, wc0, record)


def _colour(vol, fr, m, wc0, record):
    pw = voxel_centres(vol.cdim, vol.origin, vol.extent)
    n = pw.shape[0]
    C = np.zeros((n, 3))
    Wc = np.zeros(n) if wc0 is None else np.asarray(wc0, float).copy()
    amb = np.zeros(n, bool)
    status = np.zeros((fr.n, n), np.uint8)
    Kinv = np.linalg.inv(fr.K_d)
    D_all = np.asarray(fr.depth, np.float64)
    rgb = np.asarray(fr.rgb)
    imgs = rgb.astype(np.float64) * (1.0 / 255.0) if rgb.dtype == np.uint8 else rgb.astype(np.float64)
    rec = []
    for f in range(fr.n):
        D = D_all[f]
        H, W = D.shape
        CH, CW = imgs[f].shape[:2]
        T_cw = np.linalg.inv(fr.T_world_from_cam[f])
        pc = (T_cw @ _homog(pw).T).T[:, :3]
        u, v, inside, a = project_depth(fr.K_d, pc, W, H, m)
        d = _depth_lookup(D, u, v, inside)
        okd = inside & _valid(d)
        # Eq. 7: back-projection of the integer depth pixel.
        P = (Kinv @ np.stack([u, v, np.ones(n)])).T * d[:, None]
        dist = np.linalg.norm(pc - P, axis=1)
        band = okd & (dist <= vol.sigma)
        a |= okd & (np.abs(dist - vol.sigma) < m.dist)
        nb = band & (u + 1 <= W - 1) & (v + 1 <= H - 1)
        d1 = _depth_lookup(D, u + 1, v, nb)
        d2 = _depth_lookup(D, u, v + 1, nb)
        nb &= _valid(d1) & _valid(d2)
        P1 = (Kinv @ np.stack([u + 1, v, np.ones(n)])).T * d1[:, None]
        P2 = (Kinv @ np.stack([u, v + 1, np.ones(n)])).T * d2[:, None]
        N = np.cross(P1 - P, P2 - P)            # Eq. 8
        nN = np.linalg.norm(N, axis=1)
        nb &= nN > 0
        with np.errstate(divide="ignore", invalid="ignore"):
            w = np.einsum("ij,ij->i", N, P) / (nN * np.linalg.norm(P, axis=1))
        gate = nb & (w > vol.gate * Wc)
        a |= nb & (np.abs(w - vol.gate * Wc) < m.w)
        # Eq. 3 then Eq. 4 on the voxel centre.
        q = (fr.T_rgb_from_d @ _homog(pc).T).T[:, :3]
        hom = (fr.K_rgb @ q.T).T
        with np.errstate(divide="ignore", invalid="ignore"):
            xh = hom[:, 0] / hom[:, 2]
            yh = hom[:, 1] / hom[:, 2]
        hd = gate & (q[:, 2] > 0) & (np.floor(xh) >= 0) & (np.floor(xh) <= CW - 2) \
            & (np.floor(yh) >= 0) & (np.floor(yh) <= CH - 2)
        a |= gate & (_near_int(xh, m.px) | _near_int(yh, m.px))
        amb |= a
        xs = np.where(hd, xh, 0.0)
        ys = np.where(hd, yh, 0.0)
        s, x0, y0, ax, ay, gx, gy = bilinear(imgs[f], xs, ys)
        wn = np.where(hd, w, 0.0)
        alpha = np.where(hd, wn / np.where(hd, Wc + wn, 1.0), 0.0)
        Cn = (C * Wc[:, None] + wn[:, None] * s) / np.where(hd, Wc + wn, 1.0)[:, None]
        C = np.where(hd[:, None], Cn, C)
        Wc = np.where(hd, Wc + wn * (1.0 - Wc), Wc)
        st = np.where(~inside, 0, np.where(~_valid(d), 1, np.where(~band, 2, np.where(
            ~nb, 3, np.where(~gate, 4, np.where(~hd, 5, 6))))))
        status[f] = st
        if record:
            rec.append(dict(upd=hd, alpha=alpha, xh=xh, yh=yh, q=q, gx=gx, gy=gy,
                            x0=x0, y0=y0, ax=ax, ay=ay, u=u, v=v))
    out = dict(r=C[:, 0], g=C[:, 1], b=C[:, 2], wc=Wc, ambiguous=amb, status=status)
    if record:
        out["frames"] = rec
    return out
