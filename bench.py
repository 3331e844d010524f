"""Benchmark of the SG-Splatting rasteriser on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sg-3m-1600]

Workload: 3M clustered Gaussians, 1600x1060, SG form (SH degree 1 + 4
lobes) beside the degree-3 SH form on the same geometry.  Prints one JSON
line: forward frames/s of the SG form (value; the forward captured once in
a HIP graph and replayed), forward+backward ms (L1 loss against a seeded
target), the same passes launched eagerly, the SH-3 form's figures,
per-stage times from HIP events inside the eager timed loops, the roofline
of the dominant kernel, and the FP64 oracle's throughput on a bounded
sample of the same frame on the host CPU.
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
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--tile", default=None, help="fixed launch shape tw,th,ppt,ppt_bwd,batch")
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


def capture(fn, torch):
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


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
    from paper_2501_00342_amd import autotune
    sc, cams, opts = scenes.workload(args.workload)
    cam = cams[0]
    W, H = cam.width, cam.height
    params = raster.params_to_device(sc)
    target = torch.from_numpy(np.concatenate(
        [scenes.target_image(c.width, c.height, 1 + i).reshape(-1) for i, c in enumerate(cams)])).cuda()
    tune_report = None
    if args.tile:
        tw, th, ppt, pptb, batch = (int(x) for x in args.tile.split(","))
        opts = scenes.Options(tile_w=tw, tile_h=th, ppt=ppt, ppt_bwd=pptb, batch=batch)
    elif not args.no_tune and not args.profile_steps:
        opts, tune_report = autotune.tune(params, cams, opts, sc.n, sc.sh_degree, sc.n_lobes,
                                          backward=False, reps=3, tiles=[(16, 16), (32, 8), (16, 8)],
                                          batches=(128, 256), target=target)
    rast = raster.Rasterizer(cams, opts, sc.n, sc.sh_degree, sc.n_lobes)
    out = rast.forward(params, check=True)          # sizes the pair capacity
    grad_img = torch.empty_like(out.image)
    grads = {k: torch.empty_like(v) for k, v in params.items()}

    def fwd():
        rast.forward(params, out=out, check=False)

    def fwd_bwd():
        rast.forward(params, out=out, check=False)
        rast.l1(out.image, target, grad_out=grad_img)
        rast.backward_into(params, out, grad_img, grads)

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

    # the same passes captured once in a HIP graph and replayed
    g_fwd = capture(fwd, torch)
    g_fb = capture(fwd_bwd, torch)
    fwd_graph_ms = timed_loop(g_fwd.replay, args.steps, torch)
    fb_graph_ms = timed_loop(g_fb.replay, args.steps, torch)

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
        "metric": ("frames/s & fwd+bwd ms at 3M Gaussians 1600x1060, SG vs SH-3 form, same GPU"
                   if args.workload == "sg-3m-1600" else f"frames/s & fwd+bwd ms, {args.workload}"),
        "value": round(1000.0 / fwd_graph_ms, 2), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(fwd_graph_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "gaussians": sc.n, "cameras": len(cams),
                   "width": W, "height": H, "colour": f"SH{sc.sh_degree}+{sc.n_lobes}SG",
                   "tile": f"{opts.tile_w}x{opts.tile_h}", "ppt": rast.copts.pixels_per_thread,
                   "ppt_bwd": rast.copts.pixels_per_thread_bwd, "batch": opts.batch},
        "fwd_bwd_ms": round(fb_graph_ms, 4),
        "eager": {"frames_per_s": round(1000.0 / fwd_ms, 2), "fwd_ms": round(fwd_ms, 4),
                  "fwd_bwd_ms": round(fb_ms, 4)},
        "pairs": int(P), "visible": n_vis, "tiles": tiles,
        "blend_visited": visited, "blend_evaluated": evaluated,
        "stages": stages, "roofline": roof,
    }
    if tune_report is not None:
        result["autotune"] = sorted(tune_report, key=lambda r: r["ms"])[:5]
    if len(cams) > 1:
        result["views_per_s"] = round(len(cams) * 1000.0 / fwd_graph_ms, 2)
    # per-tile load (list lengths), e.g. for the stress workload
    rng = rast.ranges().cpu().numpy().view(np.uint32).astype(np.int64)
    cnt = rng[:, 1] - rng[:, 0]
    bins = np.bincount(np.ceil(np.log2(np.maximum(cnt, 1))).astype(np.int64))
    result["tile_load"] = {"p50": float(np.percentile(cnt, 50)), "p90": float(np.percentile(cnt, 90)),
                           "p99": float(np.percentile(cnt, 99)), "max": int(cnt.max()),
                           "empty": int((cnt == 0).sum()),
                           "log2_bins": {f"<=2^{i}": int(b) for i, b in enumerate(bins) if b}}

    if not args.no_sh3:
        sh3 = scenes.sh3_scene(sc.n, 1) if args.workload == "sg-3m-1600" else None
        if sh3 is not None:
            r3 = raster.Rasterizer(cams, opts, sh3.n, sh3.sh_degree, sh3.n_lobes)
            p3 = raster.params_to_device(sh3)
            o3 = r3.forward(p3, check=True)
            g3 = torch.empty_like(o3.image)

            def fwd3():
                r3.forward(p3, out=o3, check=False)

            gr3 = {k: torch.empty_like(v) for k, v in p3.items()}

            def fb3():
                r3.forward(p3, out=o3, check=False)
                r3.l1(o3.image, target, grad_out=g3)
                r3.backward_into(p3, o3, g3, gr3)

            for _ in range(args.warmup):
                fb3()
            L.LIB.render_set_timing(1)
            L.stage_times()
            sh3_fwd = timed_loop(fwd3, args.steps, torch)
            st3, n3, _ = L.stage_times()
            sh3_fb = timed_loop(fb3, args.steps, torch)
            L.stage_times()
            L.LIB.render_set_timing(0)
            gf3 = capture(fwd3, torch)
            gb3 = capture(fb3, torch)
            sh3_fwd_g = timed_loop(gf3.replay, args.steps, torch)
            sh3_fb_g = timed_loop(gb3.replay, args.steps, torch)
            result["sh3"] = {"frames_per_s": round(1000.0 / sh3_fwd_g, 2),
                             "fwd_ms": round(sh3_fwd_g, 4), "fwd_bwd_ms": round(sh3_fb_g, 4),
                             "eager_fwd_ms": round(sh3_fwd, 4), "eager_fwd_bwd_ms": round(sh3_fb, 4),
                             "preprocess_ms": round(st3[names.index("fwd.preprocess")] / max(n3, 1), 5)}
            result["sg_over_sh3_fps"] = round(sh3_fwd_g / fwd_graph_ms, 4)
            result["sg_over_sh3_fwd_bwd"] = round(sh3_fb_g / fb_graph_ms, 4)
            del r3, p3, o3, g3, gf3, gb3

    if not args.no_cpu_baseline and len(cams) == 1:
        result["cpu_baseline"] = cpu_baseline(sc, cam, opts)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
