"""Choose the launch configuration of a workload on the current GPU: the brick shape of
each volume kind and the frames per pass (K).

No candidate may change the result (the per-voxel operations and frame order do not depend
on them): every one is checked bit for bit against the default configuration.  The search
first times the brick shapes at a fixed K, both kinds in the same runs (the geometry and
colour launches of each pass are timed apart with HIP events), and keeps the fastest shape
of each kind; it then times whole scans (HIP-graph replay, volume resets included) over K
with those shapes.  The result is written to tuning.json next to this file, keyed by the
GPU architecture and the workload's name, with the volume and image sizes it was measured
on.

Usage: python -m paper_1602_06645_amd.autotune --workload {kinect,fused,many_scenes}
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING = os.path.join(HERE, "tuning.json")
K_CANDIDATES = (8, 16, 32, 48, 64)
SHAPE_K = 64          # frames per pass while the brick shapes are compared


def gpu_arch() -> str:
    """The gfx architecture of device 0 (e.g. 'gfx950'), without feature suffixes."""
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _load(path: str | None = None) -> dict:
    try:
        with open(path or TUNING) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def entry(workload: str, arch: str | None = None, path: str | None = None) -> dict | None:
    """The tuned entry of a workload for an architecture (default: device 0's), or None."""
    if arch is None:
        try:
            arch = gpu_arch()
        except Exception:
            return None
    return _load(path).get(arch, {}).get(workload)


def frames_per_pass(workload: str, default: int = 64, arch: str | None = None,
                    path: str | None = None) -> int:
    e = entry(workload, arch, path)
    return int(e["frames_per_pass"]) if e else default


def bricks(workload: str, arch: str | None = None, path: str | None = None) -> dict | None:
    """The tuned brick shapes {"geometry": (x, y, z), "colour": (x, y, z)} of a workload,
    or None (the library's defaults) when it has not been tuned on this architecture."""
    e = entry(workload, arch, path)
    if not e or "bricks" not in e:
        return None
    return {k: tuple(int(x) for x in v) for k, v in e["bricks"].items()}


def _state(pairs):
    return [[t.clone() for t in v.arrays()] for v, _ in pairs]


def _same(ref, pairs, what):
    import torch
    for sa, (v, _) in zip(ref, pairs):
        for a, b in zip(sa, v.arrays()):
            if not torch.equal(a.view(torch.int32), b.view(torch.int32)):
                raise RuntimeError(f"{what} changed the result")


def _time_shapes(pairs, K, shape_pair, reps):
    """Mean geometry and colour launch times (ms per scan: summed over the passes) of
    reps timed scans with bricks shape_pair."""
    import numpy as np
    import torch

    from .api import integrate_batch_timed
    n_pass = max((scan.depth.shape[0] + K - 1) // K for _, scan in pairs)
    g_ms, c_ms = [], []
    for r in range(reps + 1):
        for v, _ in pairs:
            v.reset()
        ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(n_pass)]
        integrate_batch_timed(pairs, K, ev, bricks=shape_pair)
        torch.cuda.synchronize()
        if r > 0:      # the first run warms up
            g_ms.append(sum(a.elapsed_time(b) for a, b, _ in ev))
            c_ms.append(sum(b.elapsed_time(c) for _, b, c in ev))
    return float(np.mean(g_ms)), float(np.mean(c_ms))


def _time_scan(pairs, K, shape_pair, reps):
    import torch

    from .api import integrate_batch
    for v, _ in pairs:
        v.reset()
    integrate_batch(pairs, frames_per_pass=K, use_graph=True, bricks=shape_pair)   # records
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for v, _ in pairs:
            v.reset()
        integrate_batch(pairs, frames_per_pass=K, use_graph=True, bricks=shape_pair)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / reps


def tune(pairs, k_candidates, reps: int = 3, shape_k: int = SHAPE_K) -> dict:
    """Search the brick shapes (at K = shape_k), then K (with the chosen shapes), for a
    batch of (Volume, Scan) pairs; every candidate must reproduce the default
    configuration's volumes bit for bit.  Returns the entry written to tuning.json."""
    import torch

    from .api import brick_shapes, integrate_batch
    shapes = brick_shapes()
    n_max = max(scan.depth.shape[0] for _, scan in pairs)
    shape_k = min(shape_k, n_max)
    for v, _ in pairs:
        v.reset()
    integrate_batch(pairs, frames_per_pass=shape_k)
    torch.cuda.synchronize()
    ref = _state(pairs)
    n = max(len(shapes["geometry"]), len(shapes["colour"]))
    shape_ms = []
    for q in range(n):
        pair = {"geometry": shapes["geometry"][min(q, len(shapes["geometry"]) - 1)],
                "colour": shapes["colour"][min(q, len(shapes["colour"]) - 1)]}
        g, c = _time_shapes(pairs, shape_k, pair, reps)
        _same(ref, pairs, f"bricks {pair}")
        shape_ms.append({"geometry": list(pair["geometry"]), "colour": list(pair["colour"]),
                         "geometry_ms": g, "colour_ms": c})
        print(f"[autotune] bricks {pair}: geometry {g:.2f} ms, colour {c:.2f} ms per scan",
              file=sys.stderr, flush=True)
    best = {"geometry": tuple(min(shape_ms, key=lambda r: r["geometry_ms"])["geometry"]),
            "colour": tuple(min(shape_ms, key=lambda r: r["colour_ms"])["colour"])}
    ks = sorted({min(K, n_max) for K in k_candidates})
    scan_ms = {}
    for K in ks:
        scan_ms[K] = _time_scan(pairs, K, best, reps)
        _same(ref, pairs, f"frames_per_pass={K} with bricks {best}")
        print(f"[autotune] K={K} with {best}: {scan_ms[K]:.2f} ms per scan", file=sys.stderr,
              flush=True)
    K = min(scan_ms, key=scan_ms.get)
    return {"frames_per_pass": K, "bricks": {k: list(v) for k, v in best.items()},
            "shape_k": shape_k, "brick_ms": shape_ms,
            "ms_per_batch": {str(k): v for k, v in scan_ms.items()}}


def _workload(name: str):
    sys.path.insert(0, os.path.dirname(HERE))
    from kf_synth import configs
    if name == "kinect":
        return [configs.kinect(device="cuda")]
    if name == "fused":
        return [configs.fused(device="cuda")]
    if name == "many_scenes":
        return configs.multi_scene(device="cuda")
    raise ValueError(f"unknown workload {name!r}")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="kinect", choices=("kinect", "fused", "many_scenes"))
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    import torch

    from . import api

    scans = _workload(args.workload)
    pairs = [(api.Volume(s), api.Scan.from_frames(f)) for s, f in scans]
    res = tune(pairs, K_CANDIDATES, args.reps)
    arch = gpu_arch()
    res.update({"device": torch.cuda.get_device_name(0), "arch": arch,
                "shapes": [{"geometry": list(s.gdim), "colour": list(s.cdim),
                            "depth": [int(f.depth.shape[2]), int(f.depth.shape[1])],
                            "rgb": [int(f.rgb.shape[2]), int(f.rgb.shape[1])], "frames": f.n}
                           for s, f in scans]})
    table = _load()
    table.setdefault(arch, {})[args.workload] = res
    with open(TUNING + ".tmp", "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(TUNING + ".tmp", TUNING)
    print(json.dumps({args.workload: res}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
