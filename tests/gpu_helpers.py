"""Shared pieces of the GPU parity tests."""
from __future__ import annotations

import sys

import numpy as np
import torch

import paper_1602_06645_amd as kf

STATE_NAMES = ["tsdf", "w_geom", "r", "g", "b", "w_col"]


def say(msg: str) -> None:
    """Name the case before a GPU step, so a failure that ends the process is attributed."""
    print(msg, flush=True)
    sys.stdout.flush()


def to_host(vol: kf.Volume):
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in vol.arrays()]


def integrate_plain(vol: kf.Volume, fr) -> None:
    """Frame by frame through kf_integrate."""
    for f in range(fr.n):
        vol.integrate(fr.depth[f], fr.rgb[f], fr.K_d, fr.K_rgb, fr.T_rgb_from_d,
                      fr.T_world_from_cam[f], fr.trunc, fr.w_max)


def assert_matches_oracle(got, want, tol=1e-5, where=""):
    """Weights bit-exact; TSDF and colour within tol (absolute)."""
    for name, g, w in zip(STATE_NAMES, got, want):
        assert g.shape == w.shape, (name, g.shape, w.shape)
        if name.startswith("w"):
            bad = np.flatnonzero(g != w)
            assert bad.size == 0, (f"{where}{name}: {bad.size} weights differ, first at "
                                   f"{bad[:5]}: gpu {g[bad[:5]]} oracle {w[bad[:5]]}")
        else:
            err = np.abs(g.astype(np.float64) - w.astype(np.float64))
            assert err.max() <= tol, f"{where}{name}: max error {err.max()} at {err.argmax()}"


def assert_bitwise(a, b, where=""):
    for name, x, y in zip(STATE_NAMES, a, b):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), f"{where}{name} differs"
