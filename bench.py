#!/usr/bin/env python3
"""Benchmark of the per-frame volumetric integration (TSDF geometry volume + asymmetric
colour volume, arXiv 1602.06645 Sec. III and IV.B) on one MI355X.

Headline workload (synthetic, seeded): the fused multi-frame scan, geometry 512^3 +
colour 1024^3 over a 1 m cube (18.3 GB of state), a 256-frame orbit of 640x480 float
depth (noisy, 1 % holes) and 1920x1080 RGB8 images of 4 spheres and 4 boxes on a plane;
trunc = 4 geometry voxels, w_max = 128.

One step = one whole scan: reset the volume, then integrate all 256 frames in passes of
K frames (K from the autotuner; one call: depth pyramids and pixel maps for all frames,
then per pass a culling launch and two persistent integration launches, geometry bricks
then colour bricks).  The metric counts every voxel of both volumes once per frame (the
swept voxel updates of KinectFusion-style integration).

Besides the headline the JSON line carries: the plain frame-by-frame path on the same
scan and the fused/plain speedup; the roofline of the dominant kernel (the colour
integration launch, VALU-bound: algorithmic operations per launch over its duration
measured with HIP events on the launch stream, with the HBM fraction of its algorithmic
bytes beside it); the many-uneven-scenes batch (16 scans, 86 GB of state) against the
same scans integrated one by one; a device copy giving the achievable HBM bandwidth;
the Kinect-like scan (256^3 / 512^3, 300 frames) with ray casting, marching cubes, the
quadric-error decimation of the mesh and texture maps of the decimated mesh; forward + backward of the differentiable form on its first
32 frames; and the CPU oracle timed on a sample of the headline scan's z-slabs on all
host threads and on one.

Usage: python bench.py [--steps K] [--warmup W] [--frames-per-pass K] [--legs a,b,...]
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
    # then the difference to Eq. 7's P (3), its squared norm (3), comparison (P itself
    # depends only on the depth pixel and is counted with the pixel map)
    "colour_voxel_frame": 26,
    # a colour gate evaluation (Eq. 10's W against gate * W_pre): mul + comparison
    "colour_gate": 2,
    # a colour update: HD pixel (Eq. 2-4 as 9 FMA, 1/q_z, 2 mul + 2 FMA, 2 floor, 5
    # comparisons, cell index 3), bilinear sample of 3 channels of 8-bit pixels (12
    # conversions, 12 scalings, 9 lerps of 2), Eq. 9 (alpha: 2, 3 x 2) and Eq. 10 (2)
    "colour_update": 24 + 12 + 12 + 18 + 2 + 6 + 2,
    # a depth pixel of the pixel map (Eq. 7 at the pixel and 2 neighbours, Eq. 8 cross
    # product, norms, dot product, square root and division): its own launch
    "pixel_map_pixel": 59,
}
WORKLOAD = ("fused multi-frame scan: geometry 512^3 + colour 1024^3 (2x per axis) over 1.0 m, "
            "256 frames of 640x480 float32 depth + 1920x1080 RGB8, 4 spheres + 4 boxes")
ALL_LEGS = ("plain", "copy", "many", "kinect", "backward", "cpu")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(sources=None) -> str:
    """Hash of the integration kernels' code: their sources with comments and blank space
    taken out, so that a change of comments alone keeps the recorded traffic valid.
    `sources`: the three files' texts (default: read from the package)."""
    import hashlib
    import re
    names = ("kf_integrate.hip", "kf_device.h", "kf_cull.h")
    if sources is None:
        sources = []
        for name in names:
            with open(os.path.join(ROOT, "paper_1602_06645_amd", "csrc", name)) as f:
                sources.append(f.read())
    h = hashlib.sha256()
    for text in sources:
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(K: int):
    """HBM bytes per launch of the integration kernels on the headline scan from the
    rocprofv3 FETCH_SIZE and WRITE_SIZE runs recorded under profiles/ (scaled by the same
    counters on a plain copy of known size): {"colour": B, "geometry": B}; None when the
    kernel source or the pass length changed since."""
    path = os.path.join(ROOT, "profiles", "integrate_kernels_fused_traffic.txt")
    try:
        with open(path) as f:
            rec = json.loads(f.read().split("JSON:", 1)[1])
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash() or rec.get("frames_per_pass") != K:
        return None
    return rec.get("bytes_per_launch")


def alg_counts(cnt, n_frames, frame_bytes):
    """Algorithmic bytes and operations of a whole scan from the counting instantiation's
    counters, split by launch kind (the frame inputs are charged to the colour launch,
    which reads the HD images, and the geometry launch, which reads the depth maps)."""
    g_bytes = 16 * int(cnt[1])
    c_bytes = 4 * int(cnt[3]) + 28 * int(cnt[5])
    g_ops = OPS["geom_voxel_frame"] * int(cnt[6]) + OPS["geom_update"] * int(cnt[0])
    c_ops = (OPS["colour_voxel_frame"] * int(cnt[7]) + OPS["colour_gate"] * int(cnt[2])
             + OPS["colour_update"] * int(cnt[4]))
    return {"geometry": {"bytes": g_bytes + n_frames * frame_bytes[0], "ops": g_ops},
            "colour": {"bytes": c_bytes + n_frames * (frame_bytes[0] + frame_bytes[1]),
                       "ops": c_ops}}


def counters_dict(cnt, spec, n):
    return {"geom_updates": int(cnt[0]), "geom_touched_per_pass": int(cnt[1]),
            "colour_gate_evals": int(cnt[2]), "colour_read_per_pass": int(cnt[3]),
            "colour_updates": int(cnt[4]), "colour_touched_per_pass": int(cnt[5]),
            "geom_voxel_frames_in_live_bricks": int(cnt[6]),
            "colour_voxel_frames_in_live_bricks": int(cnt[7]),
            "geom_live_fraction": int(cnt[6]) / (spec.n_geom * n),
            "colour_live_fraction": int(cnt[7]) / (spec.n_colour * n)}


def timed_reps(fn, reps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames-per-pass", type=int, default=0, help="0: tuned default")
    ap.add_argument("--legs", default=",".join(ALL_LEGS),
                    help="extra legs after the headline, comma-separated, from "
                         + ",".join(ALL_LEGS) + " ('' for none)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extras", action="store_true", help="time only the headline scan")
    ap.add_argument("--plain-only", action="store_true",
                    help="only run the plain frame-by-frame path twice (for profiling it)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device to device three times (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters against a known byte count)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(the integration runs on one GPU per process)",
              file=sys.stderr, flush=True)
        return 2
    legs = set() if args.no_extras else {x for x in args.legs.split(",") if x}
    if args.no_cpu:
        legs.discard("cpu")
    unknown = legs - set(ALL_LEGS)
    if unknown:
        print(f"unknown legs {sorted(unknown)}", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1602_06645_amd as kf
    from kf_synth import configs
    from paper_1602_06645_amd import autotune

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
    K = args.frames_per_pass or autotune.frames_per_pass("fused", default=64)
    bricks = autotune.bricks("fused")
    bricks_cfg = bricks or {k: v[0] for k, v in kf.brick_shapes().items()}

    t = time.perf_counter()
    spec, fr = configs.fused(device="cuda")
    torch.cuda.synchronize()
    log(f"generated the fused scan ({fr.n} frames) on the GPU in {time.perf_counter() - t:.1f} s")
    n_vox = spec.n_geom + spec.n_colour
    vol = kf.Volume(spec)
    scan = kf.Scan.from_frames(fr)

    def plain_scan():
        vol.reset()
        for f in range(fr.n):
            vol.integrate(fr.depth[f], fr.rgb[f], fr.K_d, fr.K_rgb, fr.T_rgb_from_d,
                          fr.T_world_from_cam[f], fr.trunc, fr.w_max)

    if args.plain_only:
        for _ in range(2):
            log(f"plain scan: {1e3 * timed_reps(plain_scan, 1):.1f} ms")
        return 0

    frame_bytes = (fr.depth[0].numel() * 4, fr.rgb[0].numel())
    n_pass = (fr.n + K - 1) // K

    # ---- algorithmic bytes and operations (counting instantiation, not timed)
    vol.reset()
    cnt = kf.integrate_batch_counted([(vol, scan)], frames_per_pass=K, bricks=bricks)
    alg = alg_counts(cnt, fr.n, frame_bytes)
    log(f"counters {list(map(int, cnt))}; algorithmic bytes per scan "
        f"{(alg['geometry']['bytes'] + alg['colour']['bytes']) / 1e9:.3f} GB")

    # ---- headline: warmup through the recorded graph, then the timed steps; HIP events
    # recorded by the library around each launch give the kernels' durations
    def graph_scan():
        vol.reset()
        kf.integrate_batch([(vol, scan)], frames_per_pass=K, use_graph=True, bricks=bricks)

    for _ in range(args.warmup):
        graph_scan()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} scans, K={K}, {n_pass} passes per scan)")
    ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3))
          for _ in range(n_pass * args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        vol.reset()
        kf.integrate_batch_timed([(vol, scan)], K, ev[s * n_pass:(s + 1) * n_pass], bricks=bricks)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    value = n_vox * fr.n * args.steps / wall
    geom_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    col_ms = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    log(f"fused: {ms_step:.2f} ms per scan, {value:.4g} voxel updates/s; per pass geometry "
        f"launch {geom_ms:.3f} ms, colour launch {col_ms:.3f} ms")

    def launch_roof(kind, ms):
        ops = alg[kind]["ops"] / n_pass
        byts = alg[kind]["bytes"] / n_pass
        tops = ops / (ms * 1e-3) / 1e12
        gbs = byts / (ms * 1e-3) / 1e9
        return {"launch_ms": ms, "algorithmic_ops_per_launch": ops, "achieved_tops": tops,
                "frac": tops / ALU_PEAK_TOPS, "algorithmic_bytes_per_launch": byts,
                "hbm": {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS}}

    colour = launch_roof("colour", col_ms)
    geom = launch_roof("geometry", geom_ms)
    both_ms = geom_ms + col_ms
    both_tops = (alg["geometry"]["ops"] + alg["colour"]["ops"]) / n_pass / (both_ms * 1e-3) / 1e12
    traffic = measured_traffic(K)
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
                   "bricks": {k: list(v) for k, v in bricks_cfg.items()},
                   "geometry_dim": list(spec.gdim), "colour_dim": list(spec.cdim),
                   "depth": [fr.depth.shape[2], fr.depth.shape[1]],
                   "rgb": [fr.rgb.shape[2], fr.rgb.shape[1]], "rgb_format": "u8",
                   "trunc_m": fr.trunc, "w_max": fr.w_max, "sigma_m": spec.sigma,
                   "gate": spec.gate, "graph": "warmup only (timed steps record events)"},
        "roofline": {"bound": "alu", "achieved": colour["achieved_tops"], "peak": ALU_PEAK_TOPS,
                     "unit": "Top/s (FP32 vector operations)", "frac": colour["frac"],
                     "traffic": None if traffic is None else traffic.get("colour"),
                     "kernel": "integrate_kernel<0,1> (colour bricks, persistent launch of one "
                               "fused pass)",
                     "launch_ms": col_ms,
                     "algorithmic_ops_per_launch": colour["algorithmic_ops_per_launch"],
                     "algorithmic_bytes_per_launch": colour["algorithmic_bytes_per_launch"],
                     "hbm": colour["hbm"],
                     "geometry_launch": dict(geom, traffic=None if traffic is None
                                             else traffic.get("geometry")),
                     "both_launches": {"launch_ms": both_ms, "achieved_tops": both_tops,
                                       "frac": both_tops / ALU_PEAK_TOPS}},
        "counters": counters_dict(cnt, spec, fr.n),
        "effective_voxel_updates_per_s": (int(cnt[0]) + int(cnt[4])) * args.steps / wall,
    }

    if "plain" in legs:
        # ---- the plain frame-by-frame path on the same scan (one call per frame)
        plain_scan()
        plain_wall = timed_reps(plain_scan, 1)
        out["plain_ms_per_step"] = 1e3 * plain_wall
        out["plain_voxel_updates_per_s"] = n_vox * fr.n / plain_wall
        out["fused_vs_plain"] = plain_wall / (wall / args.steps)
        log(f"plain: {1e3 * plain_wall:.1f} ms per scan; fused speedup {out['fused_vs_plain']:.2f}x")

    cpu_frames = fr.numpy() if "cpu" in legs else None
    del scan, fr, vol
    torch.cuda.empty_cache()

    if "copy" in legs:
        # ---- achievable HBM bandwidth: a 4 GiB device-to-device copy (read + write)
        n = 1 << 30
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        out["hbm_copy"] = {"GBps": 2 * 4 * n / (ms * 1e-3) / 1e9, "bytes": 2 * 4 * n,
                           "ms": ms, "note": "torch copy_ of 4 GiB float32, read + write"}
        log(f"HBM copy: {out['hbm_copy']['GBps']:.0f} GB/s")
        del src, dst
        torch.cuda.empty_cache()

    if "many" in legs:
        # ---- 16 uneven scans in one batch call against the same scans one by one
        t = time.perf_counter()
        scans = configs.multi_scene(device="cuda")
        torch.cuda.synchronize()
        log(f"generated the many-scenes batch ({len(scans)} scans) in {time.perf_counter() - t:.1f} s")
        vols = [kf.Volume(s) for s, _ in scans]
        pairs = [(v, kf.Scan.from_frames(f)) for v, (_, f) in zip(vols, scans)]
        Km = autotune.frames_per_pass("many_scenes", default=32)
        Bm = autotune.bricks("many_scenes")

        def batched():
            for v in vols:
                v.reset()
            kf.integrate_batch(pairs, frames_per_pass=Km, use_graph=True, bricks=Bm)

        def one_by_one_fused():
            for p in pairs:
                p[0].reset()
                kf.integrate_batch([p], frames_per_pass=Km, use_graph=True, bricks=Bm)

        def one_by_one_plain():
            for v, (s, f) in zip(vols, scans):
                v.reset()
                for q in range(f.n):
                    v.integrate(f.depth[q], f.rgb[q], f.K_d, f.K_rgb, f.T_rgb_from_d,
                                f.T_world_from_cam[q], f.trunc, f.w_max)
        batched()
        one_by_one_fused()
        b_s = timed_reps(batched, 3)
        f_s = timed_reps(one_by_one_fused, 3)
        one_by_one_plain()
        p_s = timed_reps(one_by_one_plain, 1)
        nv = sum((s.n_geom + s.n_colour) * f.n for s, f in scans)
        out["many_scenes"] = {
            "scenes": len(scans), "state_GB": sum(4 * 2 * s.n_geom + 4 * 4 * s.n_colour
                                                  for s, _ in scans) / 1e9,
            "frames_per_scene": scans[0][1].n, "frames_per_pass": Km,
            "batched_ms": 1e3 * b_s, "batched_voxel_updates_per_s": nv / b_s,
            "sequential_fused_ms": 1e3 * f_s, "sequential_plain_ms": 1e3 * p_s,
            "batched_vs_sequential_plain": p_s / b_s, "batched_vs_sequential_fused": f_s / b_s,
            "note": "resets of all volumes included in every figure"}
        log(f"many scenes: batched {1e3 * b_s:.1f} ms, one by one fused {1e3 * f_s:.1f} ms, "
            f"one by one plain {1e3 * p_s:.1f} ms")
        del vols, pairs, scans
        torch.cuda.empty_cache()

    if legs & {"kinect", "backward"}:
        kinect_legs(out, legs, kf, configs, np, torch)

    if "cpu" in legs:
        out["cpu_baseline"], out["cpu_baseline_1core"] = cpu_legs(spec, cpu_frames, np)
    print(json.dumps(out), flush=True)
    return 0


def kinect_legs(out, legs, kf, configs, np, torch):
    """The Kinect-like scan (256^3 / 512^3, 300 frames): fused scan time, ray casting,
    marching cubes, decimation of the mesh and texture maps of the decimated mesh; forward +
    backward on its first 32 frames."""
    from paper_1602_06645_amd import autotune
    t = time.perf_counter()
    spec, fr = configs.kinect(device="cuda")
    torch.cuda.synchronize()
    log(f"generated the Kinect-like scan ({fr.n} frames) in {time.perf_counter() - t:.1f} s")
    vol = kf.Volume(spec)
    scan = kf.Scan.from_frames(fr)
    res = {"workload": "geometry 256^3 + colour 512^3 over 0.75 m, 300 frames of 640x480 "
                       "depth + 1920x1080 RGB8"}
    if "kinect" in legs:
        K = autotune.frames_per_pass("kinect", default=64)
        Bk = autotune.bricks("kinect")

        def scan_step():
            vol.reset()
            kf.integrate_batch([(vol, scan)], frames_per_pass=K, use_graph=True, bricks=Bk)
        scan_step()
        s = timed_reps(scan_step, 5)
        res.update({"frames_per_pass": K, "ms_per_scan": 1e3 * s,
                    "voxel_updates_per_s": (spec.n_geom + spec.n_colour) * fr.n / s})
        log(f"kinect scan: {1e3 * s:.2f} ms")

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
        res["raycast"] = {"ms_per_image": rc_ms, "rays_per_s": W * H / (rc_ms * 1e-3),
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
        res["mesh"] = {"ms_per_mesh": mc_ms, "wall_ms_per_call": 1e3 * mc_wall,
                       "vertices": cap[0], "triangles": cap[1],
                       "voxels_per_s": spec.n_geom / (mc_ms * 1e-3),
                       "note": "one kf_mesh_extract call: classify, count, scan, read the "
                               "counts back (one synchronisation), write the mesh"}
        log(f"marching cubes: {mc_ms:.3f} ms on the GPU ({1e3 * mc_wall:.3f} ms per call), "
            f"{cap[0]} vertices, {cap[1]} triangles")
        del verts, tris

        # ---- quadric-error decimation of the marching-cubes mesh (Sec. IV.C), host code
        verts, tris = vol.mesh(capacity=cap)
        vh, th = verts.cpu().numpy(), tris.cpu().numpy()
        rate = 0.02
        td = time.perf_counter()
        dv, dt_ = kf.decimate(vh, th, rate)
        dec_s = time.perf_counter() - td
        res["decimation"] = {"rate": rate, "triangles_in": int(len(th)), "triangles_out": int(len(dt_)),
                             "vertices_out": int(len(dv)), "ms": 1e3 * dec_s,
                             "triangles_per_s": len(th) / dec_s,
                             "note": "kf_mesh_decimate on the host (one thread), mesh copied from "
                                     "the GPU first"}
        log(f"decimation: {len(th)} -> {len(dt_)} triangles in {1e3 * dec_s:.0f} ms")
        del verts, tris

        # ---- per-polygon texture maps of the decimated mesh from the integrated colour
        # volume (Sec. IV.D): V1, V2, V3 of each map are the triangle's vertices in order
        tri = np.ascontiguousarray(dv[dt_], np.float32)
        size_pixel = 0.8 / 1050.0   # one HD pixel at the scanning distance
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
        res["texture"] = {"ms_per_atlas": tx_ms, "texels_per_s": n_texels / (tx_ms * 1e-3),
                          "mesh": f"marching cubes of the scanned volume decimated to {rate:g}",
                          "triangles": len(tri), "texels": n_texels, "atlas": [AW, AH],
                          "size_pixel_m": size_pixel, "nonzero_fraction": nonzero,
                          "outputs": "float32 RGB + 8-bit RGB atlases",
                          "output_GBps": 15 * n_texels / (tx_ms * 1e-3) / 1e9}
        log(f"texture maps: {tx_ms:.3f} ms for {len(tri)} triangles, {n_texels / 1e6:.1f} M texels "
            f"({nonzero:.3f} non-zero)")
        del atlas, tri_d, rects_d

    if "backward" in legs:
        # ---- differentiable form: first 32 frames as float images, forward + backward
        nb = min(32, fr.n)
        rgbf = fr.rgb[:nb].to(torch.float32) * torch.tensor(np.float32(1.0 / 255.0), device="cuda")
        scan32 = kf.Scan(fr.depth[:nb], rgbf.contiguous(), fr.K_d, fr.K_rgb, fr.T_rgb_from_d,
                         fr.T_world_from_cam[:nb], fr.trunc, fr.w_max)
        g = configs.gradient_weights(spec.n_colour, device="cuda")
        Bb = autotune.bricks("kinect")   # the forward with the kinect scan's tuned shapes

        def fwd_bwd():
            vol.reset()
            kf.integrate_batch([(vol, scan32)], frames_per_pass=nb, bricks=Bb)
            return kf.integrate_backward(spec, scan32, g)

        def fwd_bwd_pose():
            vol.reset()
            kf.integrate_batch([(vol, scan32)], frames_per_pass=nb, bricks=Bb)
            return kf.integrate_backward(spec, scan32, g, pose=True)
        fwd_bwd()
        res["fwd_bwd_ms"] = 1e3 * timed_reps(fwd_bwd, 3)
        res["fwd_bwd_config"] = (f"first {nb} frames, float32 RGB, full volume, g ~ N(0,1) on "
                                 "every colour voxel; forward with the kinect scan's tuned bricks")
        log(f"forward+backward ({nb} frames): {res['fwd_bwd_ms']:.2f} ms")
        fwd_bwd_pose()
        res["fwd_bwd_pose_ms"] = 1e3 * timed_reps(fwd_bwd_pose, 3)
        log(f"forward+backward with the {nb} depth-pose gradients: {res['fwd_bwd_pose_ms']:.2f} ms")
        out["fwd_bwd_ms"] = res["fwd_bwd_ms"]
        del rgbf, scan32, g
    out["kinect"] = res
    del vol, scan, fr
    torch.cuda.empty_cache()


def cpu_legs(spec, frames, np):
    """The oracle (plain C, OpenMP over z) on a seeded sample of the headline scan's
    z-slabs, all 256 frames: on every host thread, and on one.  Voxels are independent,
    so the rate on a sample of slabs is the rate of the whole volume's work per slab."""
    from oracle import oracle as O
    rng = np.random.default_rng(1003)
    ratio = spec.cdim[2] // spec.gdim[2]

    def run(n_slabs, thick):
        # slabs of `thick` geometry slices and the colour slices over the same z range
        starts = sorted(rng.choice(spec.gdim[2] // thick, n_slabs, replace=False) * thick)
        vox, secs = 0, 0.0
        for g0 in starts:
            gz, cz = (int(g0), int(g0) + thick), (int(g0) * ratio, (int(g0) + thick) * ratio)
            st = O.State(spec, np.float32, gz=gz, cz=cz)
            t = time.perf_counter()
            O.integrate(spec, frames, st)
            secs += time.perf_counter() - t
            vox += st.tsdf.size + st.r.size
        return vox * frames.n / secs, secs, starts

    threads = O.num_threads()
    v_all, s_all, sl = run(3, 4)          # 12 of 512 geometry slices: 3/128 of the volume
    res_all = {"value": v_all, "unit": "voxel updates/s", "cores": threads, "kind": "oracle",
               "sample": f"3 seeded z-slabs of 4 geometry / {4 * ratio} colour slices at "
                         f"geometry z {[int(s) for s in sl]} (3/128 of the volume), all "
                         f"{frames.n} frames, {s_all:.1f} s on {threads} threads; plain C "
                         "oracle, OpenMP over z"}
    log(f"cpu oracle: {v_all:.4g} voxel updates/s on {threads} threads ({s_all:.1f} s)")
    O.set_num_threads(1)
    try:
        v_one, s_one, sl = run(1, 1)      # 1 of 512 geometry slices: 1/512 of the volume
    finally:
        O.set_num_threads(threads)
    res_one = {"value": v_one, "unit": "voxel updates/s", "cores": 1, "kind": "oracle",
               "sample": f"1 seeded z-slab of 1 geometry / {ratio} colour slices at geometry "
                         f"z {int(sl[0])} (1/512 of the volume), all {frames.n} frames, "
                         f"{s_one:.1f} s on one thread"}
    log(f"cpu oracle: {v_one:.4g} voxel updates/s on 1 thread ({s_one:.1f} s)")
    return res_all, res_one


if __name__ == "__main__":
    sys.exit(main())
