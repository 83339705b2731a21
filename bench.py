#!/usr/bin/env python3
"""Benchmark of the per-frame volumetric integration (TSDF geometry volume + asymmetric
colour volume, arXiv 1602.06645 Sec. III and IV.B) on one MI355X.

Workload (synthetic, seeded): geometry 256^3 + colour 512^3 over a 0.75 m cube, a
300-frame orbit of 640x480 float depth (noisy, 1 % holes) and 1920x1080 RGB8 images of
3 spheres and 2 boxes on a plane; trunc = 4 geometry voxels, w_max = 128.

One step = one whole scan: reset the volume, then integrate all 300 frames in passes of
K frames (one call: depth pyramids for all frames, then per pass a culling launch and two
persistent integration launches, geometry bricks then colour bricks).  The metric counts
every voxel of both volumes once per frame (the swept voxel updates of KinectFusion-style
integration).  Besides the headline line the JSON carries: the plain frame-by-frame path
and the fused/plain speedup, forward + backward time of the differentiable form on the
first 32 frames, the roofline of the dominant kernels (VALU-bound: algorithmic operations
per pass over the pass's measured duration, with the HBM fraction of the algorithmic bytes
beside it; both from units of work counted by the kernels' counting instantiation), and the
CPU oracle timed on a sample.

Usage: python bench.py [--steps K] [--warmup W] [--frames N] [--frames-per-pass K]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel updates/s (geometry+colour) & % HBM roofline; fused-vs-plain; fwd+bwd ms"
HBM_PEAK_GBS = 8000.0
# FP32 vector issue peak of one MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, counting
# one operation per lane per instruction (a fused multiply-add is one operation, packed
# FP32 is not used); the 157.3 TFLOP/s headline counts FMA twice and packed FP32 twice.
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# Arithmetic operations of the method per unit of work, counted on the single-precision
# operation sequence of the integration (each add, multiply, FMA, division, square root,
# rounding, comparison or conversion is one operation):
OPS = {
    # a geometry voxel-frame in a live brick: Eq. 5 z term (3 FMA; the column terms,
    # 6 FMA, shared by 8 voxels), 1/Z, 2 mul + 2 FMA + 2 rint, 5 frustum comparisons,
    # pixel index, 2 validity comparisons, sdf, band comparison
    "geom_voxel_frame": 21,
    # a geometry update: min(1, sdf / trunc) (2), W + 1, F + (t - F) / (W + 1) (3), min
    "geom_update": 7,
    # a colour voxel-frame in a live brick: as the geometry one up to the depth sample,
    # then Eq. 7 (6), the difference to the voxel (3), its squared norm (3), comparison
    "colour_voxel_frame": 32,
    # a colour gate evaluation (Eq. 10's W against gate * W_pre): mul + comparison
    "colour_gate": 2,
    # a colour update: HD pixel (Eq. 2-4 as 9 FMA, 1/q_z, 2 mul + 2 FMA, 2 floor, 5
    # comparisons, cell index 3), bilinear sample of 3 channels of 8-bit pixels (12
    # conversions, 12 scalings, 9 lerps of 2), Eq. 9 (alpha: 2, 3 x 2) and Eq. 10 (2)
    "colour_update": 24 + 12 + 12 + 18 + 2 + 6 + 2,
    # a depth pixel of the weight map (Eq. 7 at the pixel and 2 neighbours, Eq. 8 cross
    # product, norms, dot product, square root and division): its own launch
    "weight_map_pixel": 59,
}
WORKLOAD = ("kinect-like scan: geometry 256^3 + colour 512^3 (2x per axis) over 0.75 m, "
            "300 frames of 640x480 float32 depth + 1920x1080 RGB8")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def default_frames_per_pass() -> int:
    path = os.path.join(ROOT, "paper_1602_06645_amd", "tuning.json")
    try:
        with open(path) as f:
            return int(json.load(f)["kinect"]["frames_per_pass"])
    except (OSError, KeyError, ValueError):
        return 8


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in ("kf_integrate.hip", "kf_device.h", "kf_cull.h"):
        with open(os.path.join(ROOT, "paper_1602_06645_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(K: int):
    """HBM bytes per pass of the integrate kernels from the rocprofv3 FETCH_SIZE and
    WRITE_SIZE runs recorded under profiles/ (scaled by the same counters on a plain copy
    of known size); None when the kernel source or the pass length changed since."""
    path = os.path.join(ROOT, "profiles", "integrate_kernel_kinect_traffic.txt")
    try:
        with open(path) as f:
            rec = json.loads(f.read().split("JSON:", 1)[1])
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash() or rec.get("frames_per_pass") != K:
        return None
    return rec.get("bytes_per_launch")


def pass_scans(kf, fr, K):
    out = []
    for p in range(0, fr.n, K):
        q = min(fr.n, p + K)
        out.append(kf.Scan(fr.depth[p:q], fr.rgb[p:q], fr.K_d, fr.K_rgb, fr.T_rgb_from_d,
                           fr.T_world_from_cam[p:q], fr.trunc, fr.w_max))
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=300)
    ap.add_argument("--frames-per-pass", type=int, default=0, help="0: tuned default")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extras", action="store_true",
                    help="time only the fused scan (for profiling runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device to device three times (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters against a known byte count)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(the integration runs on one GPU per process)",
              file=sys.stderr, flush=True)
        return 2

    import numpy as np
    import torch

    import paper_1602_06645_amd as kf
    from kf_synth import configs

    if not torch.cuda.is_available():
        log("no GPU visible")
        return 1
    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_per_dispatch": 4 << 28}), flush=True)
        return 0
    K = args.frames_per_pass or default_frames_per_pass()

    t = time.perf_counter()
    spec, fr = configs.kinect(device="cuda", n_frames=args.frames)
    torch.cuda.synchronize()
    log(f"generated {fr.n} frames on the GPU in {time.perf_counter() - t:.1f} s")
    n_vox = spec.n_geom + spec.n_colour
    vol = kf.Volume(spec)
    passes = pass_scans(kf, fr, K)
    frame_bytes = fr.depth[0].numel() * 4 + fr.rgb[0].numel()

    # ---- algorithmic bytes of the fused scan (counting instantiation, not timed)
    vol.reset()
    cnt = kf.integrate_batch_counted([(vol, kf.Scan.from_frames(fr))], frames_per_pass=K)
    alg_bytes = 16 * int(cnt[1]) + 4 * int(cnt[3]) + 28 * int(cnt[5]) + fr.n * frame_bytes
    log(f"counters {list(map(int, cnt))}; algorithmic bytes per scan {alg_bytes / 1e9:.3f} GB")

    # ---- fused scan: warmup, then the timed steps.  A step integrates the whole scan in
    # one call (passes of K frames); HIP events recorded by the library around each
    # integration launch give the dominant kernel's duration.
    scan = kf.Scan.from_frames(fr)
    n_pass = len(passes)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n_pass * args.steps)]

    def scan_step(events=None):
        vol.reset()
        if events is None:
            kf.integrate_batch([(vol, scan)], frames_per_pass=K, use_graph=True)
        else:
            kf.integrate_batch_timed([(vol, scan)], K, events)

    for _ in range(args.warmup):
        scan_step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} scans, K={K}, {n_pass} passes per scan)")
    t0 = time.perf_counter()
    for s in range(args.steps):
        scan_step(ev[s * n_pass:(s + 1) * n_pass])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ms_step = 1e3 * wall / args.steps
    value = n_vox * fr.n * args.steps / wall
    launch_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    log(f"fused: {ms_step:.2f} ms per scan, {value:.4g} voxel updates/s, "
        f"integrate kernels {launch_ms:.3f} ms per pass")
    per_launch_bytes = alg_bytes / len(passes)
    achieved_gbs = per_launch_bytes / (launch_ms * 1e-3) / 1e9
    # algorithmic operations of the two integration launches of one pass (the weight maps
    # are computed by their own launch and are not part of it)
    alg_ops = (OPS["geom_voxel_frame"] * 512 * int(cnt[6]) + OPS["geom_update"] * int(cnt[0])
               + OPS["colour_voxel_frame"] * 512 * int(cnt[7]) + OPS["colour_gate"] * int(cnt[2])
               + OPS["colour_update"] * int(cnt[4]))
    per_launch_ops = alg_ops / len(passes)
    achieved_tops = per_launch_ops / (launch_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "voxel updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "frames": fr.n, "frames_per_pass": K,
                   "geometry_dim": list(spec.gdim), "colour_dim": list(spec.cdim),
                   "depth": [fr.depth.shape[2], fr.depth.shape[1]],
                   "rgb": [fr.rgb.shape[2], fr.rgb.shape[1]], "rgb_format": "u8",
                   "trunc_m": fr.trunc, "w_max": fr.w_max, "sigma_m": spec.sigma,
                   "gate": spec.gate},
        "roofline": {"bound": "alu", "achieved": achieved_tops, "peak": ALU_PEAK_TOPS,
                     "unit": "Top/s (FP32 vector operations)",
                     "frac": achieved_tops / ALU_PEAK_TOPS, "traffic": measured_traffic(K),
                     "algorithmic_ops_per_launch": per_launch_ops,
                     "hbm": {"achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": achieved_gbs / HBM_PEAK_GBS},
                     "kernel": "integrate_kernel<0,0> + integrate_kernel<0,1> (geometry and "
                               "colour persistent launches of one fused pass)",
                     "launch_ms": launch_ms, "algorithmic_bytes_per_launch": per_launch_bytes},
        "counters": {"geom_updates": int(cnt[0]), "geom_touched_per_pass": int(cnt[1]),
                     "colour_gate_evals": int(cnt[2]), "colour_read_per_pass": int(cnt[3]),
                     "colour_updates": int(cnt[4]), "colour_touched_per_pass": int(cnt[5]),
                     "geom_brick_frames": int(cnt[6]), "colour_brick_frames": int(cnt[7]),
                     "geom_live_fraction": int(cnt[6]) * 512 / (spec.n_geom * fr.n),
                     "colour_live_fraction": int(cnt[7]) * 512 / (spec.n_colour * fr.n)},
        "effective_voxel_updates_per_s": (int(cnt[0]) + int(cnt[4])) * args.steps / wall,
    }

    if not args.no_extras:
        # ---- plain frame-by-frame path over the same scan
        def plain_step():
            vol.reset()
            for f in range(fr.n):
                vol.integrate(fr.depth[f], fr.rgb[f], fr.K_d, fr.K_rgb, fr.T_rgb_from_d,
                              fr.T_world_from_cam[f], fr.trunc, fr.w_max)
        plain_step()
        torch.cuda.synchronize()
        tp = time.perf_counter()
        n_plain = max(1, min(args.steps, 3))
        for _ in range(n_plain):
            plain_step()
        torch.cuda.synchronize()
        plain_wall = (time.perf_counter() - tp) / n_plain
        out["plain_ms_per_step"] = 1e3 * plain_wall
        out["plain_voxel_updates_per_s"] = n_vox * fr.n / plain_wall
        out["fused_vs_plain"] = plain_wall / (wall / args.steps)
        log(f"plain: {1e3 * plain_wall:.2f} ms per scan; fused speedup {out['fused_vs_plain']:.2f}x")

        # ---- the nearest-pixel HD sampling variant: the same scan and launch configuration
        import dataclasses
        spec_n = dataclasses.replace(spec, hd_sampling="nearest")
        vol_n = kf.Volume(spec_n)

        def nearest_step():
            vol_n.reset()
            kf.integrate_batch([(vol_n, scan)], frames_per_pass=K, use_graph=True)
        nearest_step()
        torch.cuda.synchronize()
        tn = time.perf_counter()
        for _ in range(3):
            nearest_step()
        torch.cuda.synchronize()
        out["nearest_ms_per_step"] = 1e3 * (time.perf_counter() - tn) / 3
        log(f"nearest-pixel HD sampling: {out['nearest_ms_per_step']:.2f} ms per scan")
        del vol_n

        # ---- ray casting of the integrated volumes (the scan's poses, depth resolution)
        step = 0.8 * fr.trunc
        rc_poses = fr.T_world_from_cam[::10]
        H, W = fr.depth.shape[1], fr.depth.shape[2]
        vol.raycast(fr.K_d, rc_poses[0], W, H, step)
        torch.cuda.synchronize()
        rc_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(len(rc_poses))]
        hits = []
        for (e0, e1), T in zip(rc_ev, rc_poses):
            e0.record()
            img = vol.raycast(fr.K_d, T, W, H, step)
            e1.record()
            hits.append(img["depth"])
        torch.cuda.synchronize()
        rc_ms = float(np.mean([a.elapsed_time(b) for a, b in rc_ev]))
        hit_frac = float(np.mean([float((d > 0).float().mean()) for d in hits]))
        out["raycast"] = {"ms_per_image": rc_ms, "rays_per_s": W * H / (rc_ms * 1e-3),
                          "image": [W, H], "step_m": step, "poses": len(rc_poses),
                          "hit_fraction": hit_frac,
                          "outputs": "depth, vertex, normal, rgb (float32)"}
        log(f"ray cast: {rc_ms:.3f} ms per {W}x{H} image, {hit_frac:.2f} of the rays hit")
        del hits

        # ---- marching cubes of the integrated geometry volume
        verts, tris = vol.mesh()
        cap = (verts.shape[0], tris.shape[0])
        torch.cuda.synchronize()
        mc_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(10)]
        tm = time.perf_counter()
        for e0, e1 in mc_ev:
            e0.record()
            vol.mesh(capacity=cap)
            e1.record()
        torch.cuda.synchronize()
        mc_wall = (time.perf_counter() - tm) / len(mc_ev)
        mc_ms = float(np.mean([a.elapsed_time(b) for a, b in mc_ev]))
        out["mesh"] = {"ms_per_mesh": mc_ms, "wall_ms_per_call": 1e3 * mc_wall,
                       "vertices": cap[0], "triangles": cap[1],
                       "voxels_per_s": spec.n_geom / (mc_ms * 1e-3),
                       "note": "one kf_mesh_extract call: classify, count, scan, read the "
                               "counts back (one synchronisation), write the mesh"}
        log(f"marching cubes: {mc_ms:.3f} ms on the GPU ({1e3 * mc_wall:.3f} ms per call), "
            f"{cap[0]} vertices, {cap[1]} triangles")
        del verts, tris

        # ---- per-polygon texture maps from the integrated colour volume (Sec. IV.C)
        tri, size_pixel = configs.kinect_triangles(n_frames=fr.n)
        AH = 4096
        rects, AW = kf.texture_layout(tri, size_pixel, AH)
        tri_d = torch.as_tensor(tri, device="cuda")
        rects_d = torch.as_tensor(rects, device="cuda")
        atlas = vol.texture(tri_d, rects_d, AW, AH)
        torch.cuda.synchronize()
        tx_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(10)]
        for e0, e1 in tx_ev:
            e0.record()
            vol.texture(tri_d, rects_d, AW, AH, out=atlas)
            e1.record()
        torch.cuda.synchronize()
        tx_ms = float(np.mean([a.elapsed_time(b) for a, b in tx_ev]))
        n_texels = int((rects[:, 2].astype(np.int64) * rects[:, 3]).sum())
        nonzero = float(atlas["rgb8"].reshape(-1, 3).amax(1).gt(0).sum()) / n_texels
        out["texture"] = {"ms_per_atlas": tx_ms, "texels_per_s": n_texels / (tx_ms * 1e-3),
                          "triangles": len(tri), "texels": n_texels, "atlas": [AW, AH],
                          "size_pixel_m": size_pixel, "nonzero_fraction": nonzero,
                          "outputs": "float32 RGB + 8-bit RGB atlases",
                          "output_GBps": 15 * n_texels / (tx_ms * 1e-3) / 1e9}
        log(f"texture maps: {tx_ms:.3f} ms for {len(tri)} triangles, {n_texels / 1e6:.1f} M texels "
            f"({nonzero:.3f} non-zero)")
        del atlas, tri_d, rects_d

        # ---- differentiable form: first 32 frames as float images, forward + backward
        nb = min(32, fr.n)
        rgbf = fr.rgb[:nb].to(torch.float32) * torch.tensor(np.float32(1.0 / 255.0), device="cuda")
        scan32 = kf.Scan(fr.depth[:nb], rgbf.contiguous(), fr.K_d, fr.K_rgb, fr.T_rgb_from_d,
                         fr.T_world_from_cam[:nb], fr.trunc, fr.w_max)
        g = configs.gradient_weights(spec.n_colour, device="cuda")

        def fwd_bwd():
            vol.reset()
            kf.integrate_batch([(vol, scan32)], frames_per_pass=nb)
            return kf.integrate_backward(spec, scan32, g)
        fwd_bwd()
        torch.cuda.synchronize()
        tb = time.perf_counter()
        reps = 3
        for _ in range(reps):
            fwd_bwd()
        torch.cuda.synchronize()
        out["fwd_bwd_ms"] = 1e3 * (time.perf_counter() - tb) / reps
        out["fwd_bwd_config"] = f"first {nb} frames, float32 RGB, full volume, g ~ N(0,1) on every colour voxel"
        log(f"forward+backward ({nb} frames): {out['fwd_bwd_ms']:.2f} ms")

        def fwd_bwd_pose():
            vol.reset()
            kf.integrate_batch([(vol, scan32)], frames_per_pass=nb)
            return kf.integrate_backward(spec, scan32, g, pose=True)
        fwd_bwd_pose()
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for _ in range(reps):
            fwd_bwd_pose()
        torch.cuda.synchronize()
        out["fwd_bwd_pose_ms"] = 1e3 * (time.perf_counter() - tb) / reps
        log(f"forward+backward with the {nb} depth-pose gradients: {out['fwd_bwd_pose_ms']:.2f} ms")
        del rgbf, scan32, g

    if not args.no_cpu:
        from oracle import oracle as O
        # a bounded sample: consecutive frames of the same scan, one call each, until about
        # 10 s of oracle time
        st = O.State(spec, np.float32)
        n_cpu, t_cpu = 0, 0.0
        while n_cpu < fr.n and t_cpu < 10.0:
            one = fr.select(slice(n_cpu, n_cpu + 1)).numpy()
            tc = time.perf_counter()
            O.integrate(spec, one, st)
            t_cpu += time.perf_counter() - tc
            n_cpu += 1
        out["cpu_baseline"] = {"value": n_vox * n_cpu / t_cpu, "unit": "voxel updates/s",
                               "cores": O.num_threads(), "kind": "oracle",
                               "sample": f"frames 0-{n_cpu - 1} of the same scan, whole volume "
                                         f"(plain C oracle, OpenMP over z), {t_cpu:.1f} s"}
        log(f"cpu oracle: {out['cpu_baseline']['value']:.4g} voxel updates/s on {O.num_threads()} threads")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
