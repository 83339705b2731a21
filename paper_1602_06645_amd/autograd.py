"""torch.autograd wrapper of the colour-volume integration and its hand-written adjoint.

KFColourFn.apply(rgb, xi, depth, spec, K_d, K_rgb, T_rgb_from_d, T_world_from_cam)
returns the colour volume (3 x N_colour, float32) obtained by integrating the float32 HD
images `rgb` [n,CH,CW,3] with the extrinsic exp(xi^) T_rgb_from_d (xi = (rho, phi) in
se(3), float64, 6).  Gradients flow to `rgb` and `xi`; both come from the library's
backward kernel, which returns the gradient for a left perturbation at the current
extrinsic.  The chain rule to xi itself is the SE(3) left Jacobian (a 6x6 host product).
"""
from __future__ import annotations

import numpy as np
import torch

from .api import Scan, Volume, integrate_backward, integrate_batch


def _hat3(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def se3_hat(xi) -> np.ndarray:
    M = np.zeros((4, 4))
    M[:3, :3] = _hat3(xi[3:])
    M[:3, 3] = xi[:3]
    return M


def _series(A, coeff, terms=40):
    out = np.zeros_like(A)
    P = np.eye(A.shape[0])
    for k in range(terms):
        out = out + coeff(k) * P
        P = P @ A
    return out


def se3_exp(xi) -> np.ndarray:
    """exp of the 4x4 twist (power series, converges for any xi)."""
    fact = [1.0]
    for k in range(1, 45):
        fact.append(fact[-1] * k)
    return _series(se3_hat(np.asarray(xi, float)), lambda k: 1.0 / fact[k])


def se3_left_jacobian(xi) -> np.ndarray:
    """J_l(xi) = sum_k ad_xi^k / (k+1)!, with ad_xi = [[phi^, rho^], [0, phi^]]."""
    xi = np.asarray(xi, float)
    ad = np.zeros((6, 6))
    ad[:3, :3] = _hat3(xi[3:])
    ad[:3, 3:] = _hat3(xi[:3])
    ad[3:, 3:] = _hat3(xi[3:])
    fact = [1.0]
    for k in range(1, 45):
        fact.append(fact[-1] * k)
    return _series(ad, lambda k: 1.0 / fact[k + 1])


class KFColourFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rgb, xi, depth, spec, K_d, K_rgb, T_rgb_from_d, T_world_from_cam,
                trunc=0.01, w_max=128.0):
        xi_np = xi.detach().double().cpu().numpy()
        T = se3_exp(xi_np) @ np.asarray(T_rgb_from_d, float)
        vol = Volume(spec, device=rgb.device)
        scan = Scan(depth, rgb.detach().contiguous(), K_d, K_rgb, T, T_world_from_cam, trunc, w_max)
        integrate_batch([(vol, scan)], frames_per_pass=max(1, scan.depth.shape[0]))
        ctx.spec, ctx.scan, ctx.xi = spec, scan, xi_np
        ctx.xi_meta = (xi.dtype, xi.device)
        return torch.stack([vol.r, vol.g, vol.b])

    @staticmethod
    def backward(ctx, grad):
        d_rgb, d_eps = integrate_backward(ctx.spec, ctx.scan, grad.contiguous().float())
        J = se3_left_jacobian(ctx.xi)
        d_xi = J.T @ d_eps.double().cpu().numpy()
        dtype, device = ctx.xi_meta
        return (d_rgb, torch.as_tensor(d_xi, dtype=dtype, device=device),
                None, None, None, None, None, None, None, None)
