"""Choose frames_per_pass (K) for a workload on the current GPU.

Every candidate K must produce a bit-identical volume (per-voxel frame order does not
depend on K); the fastest is written to tuning.json next to this file under the
workload's name.  Usage: python -m paper_1602_06645_amd.autotune [--frames N]
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


def tune(vol, scan_passes, reps: int = 3) -> dict:
    """scan_passes: {K: [Scan, ...]} splitting the same frames into passes of K."""
    import torch

    from .api import integrate_batch

    results, ref = {}, None
    for K, passes in scan_passes.items():
        def run():
            vol.reset()
            for ps in passes:
                integrate_batch([(vol, ps)], frames_per_pass=K, use_graph=True)
        run()
        torch.cuda.synchronize()
        state = [t.clone() for t in vol.arrays()]
        if ref is None:
            ref = state
        else:
            for a, b in zip(ref, state):
                if not torch.equal(a.view(torch.int32), b.view(torch.int32)):
                    raise RuntimeError(f"frames_per_pass={K} changed the result")
        t0 = time.perf_counter()
        for _ in range(reps):
            run()
        torch.cuda.synchronize()
        results[K] = 1e3 * (time.perf_counter() - t0) / reps
        print(f"[autotune] K={K}: {results[K]:.2f} ms per scan", file=sys.stderr, flush=True)
    return results


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=300)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    import torch

    from kf_synth import configs

    from . import api

    spec, fr = configs.kinect(device="cuda", n_frames=args.frames)
    vol = api.Volume(spec)
    passes = {}
    for K in CANDIDATES:
        passes[K] = [api.Scan(fr.depth[p:p + K], fr.rgb[p:p + K], fr.K_d, fr.K_rgb,
                              fr.T_rgb_from_d, fr.T_world_from_cam[p:p + K], fr.trunc, fr.w_max)
                     for p in range(0, fr.n, K)]
    res = tune(vol, passes)
    best = min(res, key=res.get)
    table = {}
    if os.path.exists(TUNING):
        with open(TUNING) as f:
            table = json.load(f)
    table["kinect"] = {"frames_per_pass": best, "ms_per_scan": res,
                       "device": torch.cuda.get_device_name(0)}
    with open(TUNING + ".tmp", "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(TUNING + ".tmp", TUNING)
    print(json.dumps(table["kinect"]))
    return 0


if __name__ == "__main__":
    sys.exit(main())
