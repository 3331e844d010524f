"""Benchmark of the SG-Splatting rasteriser on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sg-3m-1600]

Workload: 3M clustered Gaussians, 1600x1060, SG form (SH degree 1 + 4
lobes) beside the degree-3 SH form on the same geometry.  Prints one JSON
line: forward frames/s of the SG form (value), forward+backward ms (L1
loss against a seeded target), the SH-3 form's frames/s, per-stage times
from HIP events inside the timed loops, the roofline of the dominant
kernel, and the FP64 oracle's throughput on a bounded sample of the same
frame on the host CPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# fp32 vector peak: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (non-packed lane ops)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sg-3m-1600")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sh3", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many forward+backward steps (for rocprofv3)")
    return ap.parse_args()


def stage_bytes(name, n, nvis, P, tiles, fpg, tile_passes, npix):
    """Algorithmic HBM bytes of each stage for one frame."""
    return {
        "fwd.preprocess": n * (4 * fpg) + n * (4 + 8) + nvis * 64,
        "fwd.depth_sort": 56 * n,
        "fwd.pair_scan": n * (4 + 8 + 4),
        "fwd.duplicate": nvis * (4 + 4 + 8) + 8 * P,
        "fwd.tile_sort": 16 * P * tile_passes,
        "fwd.ranges": 4 * P + 8 * tiles,
        "fwd.blend": None,
        "bwd.blend": None,
        "bwd.preprocess": nvis * 36 + 2 * n * (4 * fpg),
    }.get(name)


def timed_loop(fn, steps, torch):
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def cpu_baseline(scene, cam, opts, n_tiles_sample=24):
    """The FP64 oracle on a bounded sample of the same frame: full
    preprocess, key emission and stable sort, and the blend of a random
    sample of tiles, scaled to the frame's tile count."""
    import oracle
    from oracle import forward as F
    t = time.perf_counter()
    pre = F.preprocess(scene, cam, opts)
    t_pre = time.perf_counter() - t
    t = time.perf_counter()
    keys, vals, nt = F.emit_pairs(pre)
    keys, vals = F.sort_pairs(keys, vals)
    rng = F.tile_ranges(keys, nt)
    t_sort = time.perf_counter() - t
    pick = np.random.default_rng(0).choice(nt, size=min(n_tiles_sample, nt), replace=False)
    t = time.perf_counter()
    F.blend_image(pre, cam, opts, vals, rng, tiles=pick)
    t_blend = (time.perf_counter() - t) * nt / len(pick)
    frame_s = t_pre + t_sort + t_blend
    return {"value": 1.0 / frame_s, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": (f"full preprocess + key sort of the frame ({t_pre + t_sort:.1f} s), "
                       f"blend of {len(pick)} random tiles of {nt} scaled to the frame "
                       f"({t_blend:.1f} s est.); numpy float64, one process"),
            "frame_s_est": frame_s, "preprocess_s": t_pre, "sort_s": t_sort,
            "blend_s_est": t_blend, "host_cpu": platform.processor() or platform.machine(),
            "host_cpu_count": os.cpu_count()}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested); "
              "the rasteriser is a single-GPU build", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2501_00342_amd import _lib as L
    from paper_2501_00342_amd import raster, scenes

    assert torch.cuda.is_available()
    sc, cams, opts = scenes.workload(args.workload)
    cam = cams[0]
    W, H = cam.width, cam.height
    rast = raster.Rasterizer(cams, opts, sc.n, sc.sh_degree, sc.n_lobes)
    params = raster.params_to_device(sc)
    target = torch.from_numpy(scenes.target_image(W, H, 1).reshape(-1)).cuda()
    out = rast.forward(params, check=True)          # sizes the pair capacity
    grad_img = torch.empty_like(out.image)

    def fwd():
        rast.forward(params, out=out, check=False)

    def fwd_bwd():
        rast.forward(params, out=out, check=False)
        rast.l1(out.image, target, grad_out=grad_img)
        rast.backward(params, out, grad_img)

    if args.profile_steps:
        for _ in range(args.profile_steps):
            fwd_bwd()
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps}), flush=True)
        return

    for _ in range(args.warmup):
        fwd_bwd()
    torch.cuda.synchronize()
    bits, P = rast.status()
    assert bits == 0, f"status bits {bits}"

    L.LIB.render_set_timing(1)
    L.stage_times()
    fwd_ms = timed_loop(fwd, args.steps, torch)
    st_fwd, nf, _ = L.stage_times()
    fb_ms = timed_loop(fwd_bwd, args.steps, torch)
    st_fb, nf2, nb2 = L.stage_times()
    L.LIB.render_set_timing(0)
    names = L.stage_names()

    visited, evaluated = rast.blend_work(params)
    n_vis = int(np.count_nonzero(rast.depth_keys().cpu().numpy().view(np.uint32) != 0xFFFFFFFF))
    tiles = int(rast.layout.n_tiles)
    tile_passes = math.ceil(max(1, math.ceil(math.log2(max(tiles, 2)))) / 8)
    fpg = sc.floats_per_gaussian()

    stages = {}
    for i, nm in enumerate(names):
        calls = nf if nm.startswith("fwd") else nb2
        src = st_fwd if nm.startswith("fwd") else st_fb
        if calls <= 0:
            continue
        ms = src[i] / calls
        b = stage_bytes(nm, sc.n, n_vis, P, tiles, fpg, tile_passes, W * H)
        ent = {"ms": round(ms, 5)}
        if b is not None and ms > 0:
            ent["alg_bytes"] = int(b)
            ent["GBps"] = round(b / (ms * 1e-3) / 1e9, 1)
            ent["hbm_frac"] = round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        stages[nm] = ent

    # dominant forward kernel group and its roofline
    fwd_names = [n for n in stages if n.startswith("fwd.") and n != "fwd.setup"]
    dom = max(fwd_names, key=lambda n: stages[n]["ms"])
    if dom == "fwd.blend":
        ops = evaluated * 24 + visited * 4          # lane-ops (blend costs)
        ach = ops / (stages[dom]["ms"] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": round(ach, 3),
                "peak": round(VALU_PEAK_TOPS, 2), "unit": "Tlane-op/s",
                "frac": round(ach / VALU_PEAK_TOPS, 4), "traffic": None}
    else:
        b = stages[dom]["alg_bytes"]
        ach = b / (stages[dom]["ms"] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None}

    result = {
        "metric": "frames/s & fwd+bwd ms at 3M Gaussians 1600x1060, SG vs SH-3 form, same GPU",
        "value": round(1000.0 / fwd_ms, 2), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(fwd_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "gaussians": sc.n, "width": W, "height": H,
                   "colour": f"SH{sc.sh_degree}+{sc.n_lobes}SG", "tile": f"{opts.tile_w}x{opts.tile_h}"},
        "fwd_bwd_ms": round(fb_ms, 4),
        "pairs": int(P), "visible": n_vis, "tiles": tiles,
        "blend_visited": visited, "blend_evaluated": evaluated,
        "stages": stages, "roofline": roof,
    }

    if not args.no_sh3:
        sh3 = scenes.sh3_scene(sc.n, 1) if args.workload == "sg-3m-1600" else None
        if sh3 is not None:
            r3 = raster.Rasterizer(cams, opts, sh3.n, sh3.sh_degree, sh3.n_lobes)
            p3 = raster.params_to_device(sh3)
            o3 = r3.forward(p3, check=True)
            g3 = torch.empty_like(o3.image)

            def fwd3():
                r3.forward(p3, out=o3, check=False)

            def fb3():
                r3.forward(p3, out=o3, check=False)
                r3.l1(o3.image, target, grad_out=g3)
                r3.backward(p3, o3, g3)

            for _ in range(args.warmup):
                fb3()
            L.LIB.render_set_timing(1)
            L.stage_times()
            sh3_fwd = timed_loop(fwd3, args.steps, torch)
            st3, n3, _ = L.stage_times()
            sh3_fb = timed_loop(fb3, args.steps, torch)
            L.stage_times()
            L.LIB.render_set_timing(0)
            result["sh3"] = {"frames_per_s": round(1000.0 / sh3_fwd, 2), "fwd_ms": round(sh3_fwd, 4),
                             "fwd_bwd_ms": round(sh3_fb, 4),
                             "preprocess_ms": round(st3[names.index("fwd.preprocess")] / max(n3, 1), 5)}
            result["sg_over_sh3_fps"] = round(sh3_fwd / fwd_ms, 4)
            del r3, p3, o3, g3

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(sc, cam, opts)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
