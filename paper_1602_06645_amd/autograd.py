"""torch.autograd wrapper of the colour-volume integration and its hand-written adjoint.

KFColourFn.apply(rgb, xi, depth, spec, K_d, K_rgb, T_rgb_from_d, T_world_from_cam)
returns the colour volume (3 x N_colour, float32) obtained by integrating the float32 HD
images `rgb` [n,CH,CW,3] with the extrinsic exp(xi^) T_rgb_from_d (xi = (rho, phi) in
se(3), float64, 6).  Gradients flow to `rgb` and `xi`; both come from the library's
backward kernel, which returns the gradient for a left perturbation at the current
extrinsic; kf_se3_pullback maps it to xi itself (the SE(3) left Jacobian) and
kf_se3_compose forms the perturbed extrinsic.  Any number of frames: the library takes
a longer scan in chunks of 64 frames.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .api import Scan, Volume, integrate_backward, integrate_batch


def _ptr(a: np.ndarray) -> C.c_void_p:
    return C.c_void_p(a.ctypes.data)


def se3_exp_times(xi, T) -> np.ndarray:
    """exp(xi^) T (kf_se3_compose); T rigid 4x4."""
    x = np.ascontiguousarray(xi, np.float64).reshape(6)
    Ti = np.ascontiguousarray(T, np.float64).reshape(4, 4)
    out = np.zeros((4, 4), np.float64)
    L.check(L.load().kf_se3_compose(_ptr(x), _ptr(Ti), _ptr(out)))
    return out


def se3_exp(xi) -> np.ndarray:
    """exp(xi^) as a 4x4 matrix."""
    return se3_exp_times(xi, np.eye(4))


def se3_pullback(xi, d_eps) -> np.ndarray:
    """J_l(xi)^T d_eps (kf_se3_pullback)."""
    x = np.ascontiguousarray(xi, np.float64).reshape(6)
    d = np.ascontiguousarray(d_eps, np.float64).reshape(6)
    out = np.zeros(6, np.float64)
    L.check(L.load().kf_se3_pullback(_ptr(x), _ptr(d), _ptr(out)))
    return out


def se3_left_jacobian(xi) -> np.ndarray:
    """J_l(xi) (6 x 6), column by column through kf_se3_pullback."""
    return np.stack([se3_pullback(xi, e) for e in np.eye(6)], axis=0)


class KFColourFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rgb, xi, depth, spec, K_d, K_rgb, T_rgb_from_d, T_world_from_cam,
                trunc=0.01, w_max=128.0):
        xi_np = xi.detach().double().cpu().numpy()
        T = se3_exp_times(xi_np, T_rgb_from_d)
        vol = Volume(spec, device=rgb.device)
        scan = Scan(depth, rgb.detach().contiguous(), K_d, K_rgb, T, T_world_from_cam, trunc, w_max)
        integrate_batch([(vol, scan)], frames_per_pass=max(1, scan.depth.shape[0]))
        ctx.spec, ctx.scan, ctx.xi = spec, scan, xi_np
        ctx.xi_meta = (xi.dtype, xi.device)
        return torch.stack([vol.r, vol.g, vol.b])

    @staticmethod
    def backward(ctx, grad):
        d_rgb, d_eps = integrate_backward(ctx.spec, ctx.scan, grad.contiguous().float())
        d_xi = se3_pullback(ctx.xi, d_eps.double().cpu().numpy())
        dtype, device = ctx.xi_meta
        return (d_rgb, torch.as_tensor(d_xi, dtype=dtype, device=device),
                None, None, None, None, None, None, None, None)
