"""Choose the launch configuration of a workload on the current GPU: frames per pass (K).

Every candidate must produce a bit-identical volume (the per-voxel frame order does not
depend on it); the fastest is written to tuning.json next to this file, keyed by the GPU
architecture and the workload's name, with the shapes it was measured on.

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
CANDIDATES = (4, 8, 16, 32, 48, 64)


def gpu_arch() -> str:
    """The gfx architecture of device 0 (e.g. 'gfx950'), without feature suffixes."""
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _load() -> dict:
    try:
        with open(TUNING) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def entry(workload: str, arch: str | None = None) -> dict | None:
    """The tuned entry of a workload for an architecture (default: device 0's), or None."""
    if arch is None:
        try:
            arch = gpu_arch()
        except Exception:
            return None
    return _load().get(arch, {}).get(workload)


def frames_per_pass(workload: str, default: int = 64, arch: str | None = None) -> int:
    e = entry(workload, arch)
    return int(e["frames_per_pass"]) if e else default


def _time_batch(pairs, K, reps):
    import torch

    from .api import integrate_batch
    for v, _ in pairs:
        v.reset()
    integrate_batch(pairs, frames_per_pass=K, use_graph=True)       # records the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for v, _ in pairs:
            v.reset()
        integrate_batch(pairs, frames_per_pass=K, use_graph=True)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / reps


def tune(pairs, candidates, reps: int = 3) -> dict:
    """Time a batch of (Volume, Scan) pairs at each K; every K must give the volumes of
    the first one bit for bit.  Returns {K: ms per batch (resets included)}."""
    import torch

    results, ref = {}, None
    for K in candidates:
        ms = _time_batch(pairs, K, reps)
        state = [[t.clone() for t in v.arrays()] for v, _ in pairs]
        if ref is None:
            ref = state
        else:
            for sa, sb in zip(ref, state):
                for a, b in zip(sa, sb):
                    if not torch.equal(a.view(torch.int32), b.view(torch.int32)):
                        raise RuntimeError(f"frames_per_pass={K} changed the result")
        del state
        results[K] = ms
        print(f"[autotune] K={K}: {ms:.2f} ms", file=sys.stderr, flush=True)
    return results


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
    n_max = max(f.n for _, f in scans)
    cands = sorted({min(K, n_max) for K in CANDIDATES})
    res = tune(pairs, cands, args.reps)
    best = min(res, key=res.get)
    arch = gpu_arch()
    table = _load()
    table.setdefault(arch, {})[args.workload] = {
        "frames_per_pass": best, "ms_per_batch": {str(k): v for k, v in res.items()},
        "device": torch.cuda.get_device_name(0),
        "shapes": [{"geometry": list(s.gdim), "colour": list(s.cdim),
                    "depth": [int(f.depth.shape[2]), int(f.depth.shape[1])],
                    "rgb": [int(f.rgb.shape[2]), int(f.rgb.shape[1])], "frames": f.n}
                   for s, f in scans]}
    with open(TUNING + ".tmp", "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(TUNING + ".tmp", TUNING)
    print(json.dumps({args.workload: table[arch][args.workload]}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
