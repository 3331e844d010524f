"""Benchmark of the SG-Splatting rasteriser on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sg-3m-1600]

Workload: 3M clustered Gaussians, 1600x1060, SG form (SH degree 1 + 4
lobes) beside the degree-3 SH form on the same geometry.  Prints one JSON
line: forward frames/s of the SG form (value; the forward captured once in
a HIP graph and replayed), forward+backward ms (L1 loss against a seeded
target), the same passes launched eagerly, the SH-3 form's figures (and a
paired comparison: both forms' graphs replayed in alternation),
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
COPY_BYTES = 1 << 28      # calibration kernel: bytes read (and written) per launch
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
    ap.add_argument("--profile-pass", choices=("both", "fwd", "fwdbwd"), default="both",
                    help="with --profile-steps: run only the forward's launch shape (fwd), "
                         "only forward + L1 + backward at its own shape (fwdbwd), or both")
    ap.add_argument("--no-tune", action="store_true", help="library defaults, no autotuner")
    ap.add_argument("--retune", action="store_true",
                    help="time every launch shape again instead of using the cached choice")
    ap.add_argument("--tile", default=None,
                    help="fixed launch shape tw,th,ppt,ppt_bwd,batch[,schedule]")
    return ap.parse_args()


GEOM_FLOATS = 3 + 3 + 4 + 1   # mean, log-scale, quaternion, opacity logit


def stage_bytes(name, n, items, nvis, nvis_g, P, tiles, fpg, strips, E, npix):
    """Algorithmic HBM bytes of each stage for one frame, as this design moves
    them: n Gaussians, items (camera, Gaussian) items, nvis of them visible,
    nvis_g Gaussians visible in some camera (the only ones whose colour is
    read), P pairs, E first-level (strip, item) entries over `strips` strips."""
    kb = 2 if strips <= 65536 else 4  # bytes per strip key
    strip_passes = max(1, math.ceil(math.ceil(math.log2(max(strips, 2))) / 8))
    fc = fpg - GEOM_FLOATS             # colour floats per Gaussian
    return {
        "fwd.preprocess": n * 4 * GEOM_FLOATS + nvis_g * 4 * fc + items * (4 + 8) + nvis * 64,
        # pass 0 reads every depth key twice (count, then rank) and writes the
        # visible (key, item); the two middle passes read keys (count), read
        # and write (key, item); the last reads keys, then (key, item) and each
        # item's rectangle, and writes item, entry count and rectangle
        "fwd.depth_sort": 8 * items + 8 * nvis + 2 * 20 * nvis + 36 * nvis,
        # entry counts read twice (block sums with the rectangles, then the
        # scan), offsets written
        "fwd.pair_scan": 20 * nvis,
        # the duplicate only counts: it reads each chunk's items (offset,
        # item, rectangle)
        "fwd.duplicate": nvis * (4 + 4 + 8),
        # first level: the first strip pass generates the entries from the
        # items again and writes (strip, position); a later pass reads the
        # strip ids (upsweep), then reads and writes (strip, position).
        # Second level: the count reads each entry and its rectangle; the
        # scatter reads entry, rectangle and item and writes every pair once
        "fwd.tile_sort": nvis * (4 + 4 + 8) + (kb + 4) * E
        + (strip_passes - 1) * (kb + 2 * (kb + 4)) * E + (4 + 8) * E + (4 + 8 + 4) * E + 4 * P,
        "fwd.tile_order": None,  # heavy-first order of the queue schedule
        "fwd.blend": None,
        "bwd.blend": None,
        # geometry read and its gradient written for every Gaussian, colour
        # read for the visible ones, colour gradient written for all
        "bwd.preprocess": nvis * 36 + 2 * n * 4 * GEOM_FLOATS + nvis_g * 4 * fc + n * 4 * fc,
    }.get(name)


def stage_bytes_all_params(name, n, items, nvis, fpg):
    """The same stages counted with every Gaussian's full parameter record
    read (and, backward, its gradient written), visible or not: what a
    layout that cannot skip the colour of culled Gaussians moves."""
    return {
        "fwd.preprocess": n * 4 * fpg + 4 * items + 64 * nvis,
        "bwd.preprocess": 36 * nvis + 2 * n * 4 * fpg,
    }.get(name)


def standard_binning_bytes(items, nvis, P, tiles):
    """Bytes of the usual binning: an exclusive scan of the per-item pair
    counts, the duplicate writing 64-bit (tile << 32 | depth) keys with
    32-bit values, an LSD radix sort of 8-bit digits over the low 32 +
    ceil(log2 tiles) key bits, and the range search over the sorted keys."""
    passes = math.ceil((32 + math.ceil(math.log2(max(tiles, 2)))) / 8)
    return (8 * items + (16 * nvis + 12 * P) + (8 + 24 * passes) * P + (8 * P + 8 * tiles)), passes


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


def alternating_steps(fns, steps, torch):
    """Per-step times (ms) of several step functions run in strict
    alternation (f0, f1, ..., f0, f1, ...): each step between its own pair
    of events on the current stream, so that neighbouring samples of the
    forms see the same clock and temperature."""
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)] for _ in fns]
    torch.cuda.synchronize()
    for i in range(steps):
        for f, e in zip(fns, ev):
            e[i][0].record()
            f()
            e[i][1].record()
    torch.cuda.synchronize()
    return [np.array([a.elapsed_time(b) for a, b in e]) for e in ev]


def summary(t):
    return {"median_ms": round(float(np.median(t)), 5), "p10_ms": round(float(np.percentile(t, 10)), 5),
            "p90_ms": round(float(np.percentile(t, 90)), 5), "samples": int(len(t))}


def ratio_ci(num, den, reps=2000, seed=0):
    """median(num) / median(den) and its bootstrap 95% interval, resampling
    the alternation index (each resample keeps neighbouring pairs)."""
    rng = np.random.default_rng(seed)
    n = len(num)
    idx = rng.integers(0, n, size=(reps, n))
    r = np.median(num[idx], axis=1) / np.median(den[idx], axis=1)
    return (round(float(np.median(num) / np.median(den)), 4),
            [round(float(np.percentile(r, 2.5)), 4), round(float(np.percentile(r, 97.5)), 4)])


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


def cpu_baseline(scene, cam, opts, target, workers=16):
    """The FP64 oracle over the whole frame on the host's cores: preprocess,
    key emission, stable sort and ranges (one process, NumPy), the blend of
    every tile (a pool of worker processes over tiles), then the backward of
    the L1 loss: the blend backward over every tile on the pool and the chain
    rule to the raw parameters (one process).  Runs before the GPU is
    initialised, so the forked workers hold no device state."""
    from oracle import backward as OB
    from oracle import forward as F
    from oracle import parallel as OP
    nw = OP.workers(workers)
    st = {}
    t = time.perf_counter()
    pre = F.preprocess(scene, cam, opts)
    st["preprocess_s"] = time.perf_counter() - t
    t = time.perf_counter()
    keys, vals, nt = F.emit_pairs(pre)
    keys, vals = F.sort_pairs(keys, vals)
    rng = F.tile_ranges(keys, nt)
    st["sort_s"] = time.perf_counter() - t
    t = time.perf_counter()
    img = OP.blend_image(pre, cam, opts, vals, rng, n_workers=nw)[0]
    st["blend_s"] = time.perf_counter() - t
    frame_s = st["preprocess_s"] + st["sort_s"] + st["blend_s"]
    _, gimg = OB.l1_loss(img, target)
    t = time.perf_counter()
    g2 = OP.blend_backward(pre, cam, opts, vals, rng, gimg, n_workers=nw)
    st["blend_backward_s"] = time.perf_counter() - t
    t = time.perf_counter()
    OB.preprocess_backward(scene, cam, opts, pre, g2)
    st["preprocess_backward_s"] = time.perf_counter() - t
    fb_s = frame_s + st["blend_backward_s"] + st["preprocess_backward_s"]
    return {"value": round(1.0 / frame_s, 5), "unit": "frames/s", "cores": nw, "kind": "oracle",
            "sample": (f"the whole frame, forward ({frame_s:.1f} s) and L1 backward "
                       f"({fb_s - frame_s:.1f} s): numpy float64, blend and blend backward on "
                       f"{nw} worker processes over tiles, the rest in one process"),
            "frame_s": round(frame_s, 3), "fwd_bwd_s": round(fb_s, 3),
            "stages_s": {k: round(v, 3) for k, v in st.items()},
            "host_cpu": platform.processor() or platform.machine(),
            "host_cpu_count": os.cpu_count()}


SINGLE_KERNEL_STAGES = ("fwd.preprocess", "fwd.duplicate", "fwd.blend")


def source_digest(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


_CSRC = "paper_2501_00342_amd/csrc/"
# the source files of each single-kernel stage whose counters may be quoted:
# a counter summary holds their digest, and goes stale when any of them changes
TRAFFIC_SOURCES = {
    "fwd.blend": [_CSRC + "blend.hip", _CSRC + "common.hpp"],
    "bwd.blend": [_CSRC + "blend.hip", _CSRC + "common.hpp"],
    "fwd.preprocess": [_CSRC + "preprocess.hip", _CSRC + "colour.hpp", _CSRC + "sh_basis.hpp",
                       _CSRC + "common.hpp"],
    "fwd.duplicate": [_CSRC + "sort.hip", _CSRC + "common.hpp"],
}


def counter_traffic(stage, workload, shape):
    """HBM bytes per launch of `stage` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by the calibration kernel), or
    None when there is none for this workload and launch shape, or the
    kernel's source has changed since the counters were taken."""
    import glob
    src = TRAFFIC_SOURCES.get(stage)
    if src is None:
        return None
    digest = source_digest(src)
    for fn in sorted(glob.glob(os.path.join(ROOT, "profiles", "*counters*.md"))):
        with open(fn) as f:
            for line in f:
                if not line.startswith("traffic_json: "):
                    continue
                try:
                    rec = json.loads(line[len("traffic_json: "):])
                except ValueError:
                    continue
                if (rec.get("stage") == stage and rec.get("workload") == workload
                        and rec.get("shape") == shape and rec.get("source_sha256") == digest):
                    return {"bytes": int(rec["bytes_per_launch"]),
                            "file": os.path.relpath(fn, ROOT)}
    return None


def choose_options(args, torch, scenes, autotune, params, cams, base, scene, target):
    """(forward options, forward+backward options, tuning reports)."""
    if args.tile:
        v = [int(x) for x in args.tile.split(",")]
        o = scenes.Options(tile_w=v[0], tile_h=v[1], ppt=v[2], ppt_bwd=v[3], batch=v[4],
                           schedule=v[5] if len(v) > 5 else 0)
        return o, o, None
    if args.no_tune:
        return base, base, None
    # launch shapes picked by the autotuner (cached per GPU and workload): one
    # for the forward alone, one for forward + L1 + backward
    kw = dict(reps=6 if args.retune else 3, tiles=[(16, 16), (32, 8), (16, 8)], batches=(64, 128, 256), target=target,
              use_cache=not args.retune)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    picked, reports = [], {}
    for bwd in (False, True):
        o, rep = autotune.tune(params, cams, base, scene.n, scene.sh_degree, scene.n_lobes,
                               backward=bwd, **kw)
        picked.append(o)
        timed = [r for r in rep if r.get("ms") is not None]
        reports["fwd_bwd" if bwd else "fwd"] = sorted(timed, key=lambda r: r["ms"])[:3]
        if args.retune:
            key = autotune.cache_key(arch, cams, scene.n, scene.sh_degree, scene.n_lobes, bwd)
            best = min(timed, key=lambda r: r["ms"])
            print(json.dumps({"autotune_entry": {key: {
                "choice": {k: best[k] for k in best if k not in ("ms", "error")},
                "report": rep}}}), file=sys.stderr, flush=True)
    return picked[0], picked[1], reports


def shape_of(rast, o):
    c = rast.copts
    return (f"{o.tile_w}x{o.tile_h},ppt{c.pixels_per_thread},pptb{c.pixels_per_thread_bwd},"
            f"b{c.batch or 128},s{c.schedule or 0}")


def measure_form(args, torch, L, raster, scenes, autotune, scene, cams, base, target,
                 profile=False, colour_dtype=None):
    """Tune, then time one colour form: eager passes with per-stage HIP
    events, then the same passes captured in HIP graphs and replayed.
    colour_dtype: storage type of the colour parameters (float32 default)."""
    params = raster.params_to_device(scene, colour_dtype=colour_dtype or torch.float32)
    opts_f, opts_b, reports = choose_options(args, torch, scenes, autotune, params, cams, base,
                                             scene, target)
    if profile:
        # counter runs: one launch shape per pass, so every dispatch of a
        # kernel name belongs to one shape.  The checked forward that sizes
        # the pair capacity comes first; a 64-element negation marks where
        # the profiled steps begin (the counter summaries read only the
        # dispatches after it)
        passes = ("fwd", "fwdbwd") if args.profile_pass == "both" else (args.profile_pass,)
        for ps in passes:
            o = opts_f if ps == "fwd" else opts_b
            r = raster.Rasterizer(cams, o, scene.n, scene.sh_degree, scene.n_lobes)
            ob = r.forward(params, check=True)
            gi = torch.empty_like(ob.image)
            gr = raster.new_grads(params)
            mark = torch.ones(64, device="cuda")
            torch.cuda.synchronize()
            torch.neg(mark, out=mark)
            for _ in range(args.profile_steps):
                r.forward(params, out=ob, check=False)
                if ps == "fwdbwd":
                    r.l1(ob.image, target, grad_out=gi)
                    r.backward_into(params, ob, gi, gr)
            torch.cuda.synchronize()
            print(json.dumps({"profile_pass": ps, "shape": shape_of(r, o)}), flush=True)
            del r, ob, gi, gr
        return None
    rast = raster.Rasterizer(cams, opts_f, scene.n, scene.sh_degree, scene.n_lobes)
    out = rast.forward(params, check=True)          # sizes the pair capacity
    if opts_b == opts_f:
        rast_b, out_b = rast, out
    else:
        rast_b = raster.Rasterizer(cams, opts_b, scene.n, scene.sh_degree, scene.n_lobes)
        out_b = rast_b.forward(params, check=True)
    grad_img = torch.empty_like(out_b.image)
    grads = raster.new_grads(params)

    def fwd():
        rast.forward(params, out=out, check=False)

    def fwd_bwd():
        rast_b.forward(params, out=out_b, check=False)
        rast_b.l1(out_b.image, target, grad_out=grad_img)
        rast_b.backward_into(params, out_b, grad_img, grads)

    for _ in range(args.warmup):
        fwd()
        fwd_bwd()
    torch.cuda.synchronize()
    for r in (rast, rast_b):
        bits, _ = r.status()
        assert bits == 0, f"status bits {bits}"

    L.LIB.render_set_timing(1)
    L.stage_times()
    fwd_ms = timed_loop(fwd, args.steps, torch)
    st_fwd, nf, _ = L.stage_times()
    fb_ms = timed_loop(fwd_bwd, args.steps, torch)
    st_fb, _, nb = L.stage_times()
    L.LIB.render_set_timing(0)
    g_fwd = capture(fwd, torch)
    g_fb = capture(fwd_bwd, torch)
    fwd_graph_ms = timed_loop(g_fwd.replay, args.steps, torch)
    fb_graph_ms = timed_loop(g_fb.replay, args.steps, torch)
    # the graphs replay into out, out_b, grad_img and grads: they are kept
    # with the graphs, so no replay ever writes memory the allocator reused
    return dict(rast=rast, rast_b=rast_b, params=params, opts_f=opts_f, opts_b=opts_b,
                reports=reports, fwd_ms=fwd_ms, fb_ms=fb_ms, fwd_graph_ms=fwd_graph_ms,
                fb_graph_ms=fb_graph_ms, st_fwd=st_fwd, nf=nf, st_fb=st_fb, nb=nb,
                g_fwd=g_fwd, g_fb=g_fb, buffers=(out, out_b, grad_img, grads, target))


def paired_comparison(m, m3, steps, torch):
    """SG and SH-3 graphs replayed in strict alternation, every step timed on
    its own: medians, p10/p90, and the bootstrap 95% interval of each
    SH-3 / SG time ratio (the SG speed-up)."""
    fw = alternating_steps([m["g_fwd"].replay, m3["g_fwd"].replay], steps, torch)
    fb = alternating_steps([m["g_fb"].replay, m3["g_fb"].replay], steps, torch)
    r_fwd, ci_fwd = ratio_ci(fw[1], fw[0])
    r_fb, ci_fb = ratio_ci(fb[1], fb[0])
    return {"steps_per_form": steps, "sg_fwd": summary(fw[0]), "sh3_fwd": summary(fw[1]),
            "sg_fwd_bwd": summary(fb[0]), "sh3_fwd_bwd": summary(fb[1]),
            "sg_over_sh3_fps": r_fwd, "sg_over_sh3_fps_ci95": ci_fwd,
            "sg_over_sh3_fwd_bwd": r_fb, "sg_over_sh3_fwd_bwd_ci95": ci_fb}, fw[0], fb[0]


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested); "
              "the rasteriser is a single-GPU build", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2501_00342_amd import _lib as L
    from paper_2501_00342_amd import autotune, raster, scenes

    sc, cams, base = scenes.workload(args.workload)
    cam = cams[0]
    W, H = cam.width, cam.height
    targets = [scenes.target_image(c.width, c.height, 1 + i) for i, c in enumerate(cams)]
    # the oracle's leg first: its worker processes fork before the GPU is used
    cpu = None
    if not args.no_cpu_baseline and not args.profile_steps and len(cams) == 1:
        cpu = cpu_baseline(sc, cam, base, targets[0])
    assert torch.cuda.is_available()
    target = torch.from_numpy(np.concatenate([t.reshape(-1) for t in targets])).cuda()
    mods = (torch, L, raster, scenes, autotune)

    if args.profile_steps:
        measure_form(args, *mods, sc, cams, base, target, profile=True)
        # counter calibration: an elementwise kernel that reads and writes
        # COPY_BYTES each (torch's neg), profiled in the same run
        src = torch.ones(COPY_BYTES // 4, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps, "copy_bytes": COPY_BYTES}),
              flush=True)
        return

    m = measure_form(args, *mods, sc, cams, base, target)
    rast, opts = m["rast"], m["opts_f"]
    names = L.stage_names()
    bits, P = rast.status()
    visited, evaluated, blended = rast.blend_work(m["params"])
    bwd_work = m["rast_b"].blend_bwd_work(m["params"], m["buffers"][1])
    vis_items = (rast.depth_keys().cpu().numpy().view(np.uint32) != 0xFFFFFFFF).reshape(len(cams), sc.n)
    n_vis = int(np.count_nonzero(vis_items))
    n_vis_g = int(np.count_nonzero(vis_items.any(axis=0)))
    tiles = int(rast.layout.n_tiles)
    strips = rast.n_strips()
    E = int(rast.header()[5].item())
    fpg = sc.floats_per_gaussian()

    stages = {}
    for i, nm in enumerate(names):
        calls = m["nf"] if nm.startswith("fwd") else m["nb"]
        src = m["st_fwd"] if nm.startswith("fwd") else m["st_fb"]
        if calls <= 0:
            continue
        ms = src[i] / calls
        items = len(cams) * sc.n
        b = stage_bytes(nm, sc.n, items, n_vis, n_vis_g, P, tiles, fpg, strips, E, W * H)
        ent = {"ms": round(ms, 5)}
        if b is not None and ms > 0:
            ent["alg_bytes"] = int(b)
            ent["GBps"] = round(b / (ms * 1e-3) / 1e9, 1)
            ent["hbm_frac"] = round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        ba = stage_bytes_all_params(nm, sc.n, items, n_vis, fpg)
        if ba is not None and ms > 0:
            ent["alg_bytes_all_params"] = int(ba)
            ent["hbm_frac_all_params"] = round(ba / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        stages[nm] = ent

    # binning as a whole (depth sort to the last tile pass, which also writes
    # the ranges) beside the bytes the usual 64-bit key sort would move
    bin_names = ("fwd.depth_sort", "fwd.pair_scan", "fwd.duplicate", "fwd.tile_sort")
    bin_ms = sum(stages[nm]["ms"] for nm in bin_names if nm in stages)
    std_b, std_passes = standard_binning_bytes(len(cams) * sc.n, n_vis, P, tiles)
    binning = {"ms": round(bin_ms, 5),
               "alg_bytes": int(sum(stages[nm].get("alg_bytes", 0) for nm in bin_names if nm in stages)),
               "bytes_64bit_key_sort": int(std_b), "key_sort_passes": std_passes}
    if bin_ms > 0:
        binning["ms_64bit_key_sort_at_hbm_peak"] = round(std_b / (HBM_PEAK_GBS * 1e9) * 1e3, 5)

    # roofline of the forward's dominant kernel (stages that are one launch)
    dom = max((n for n in SINGLE_KERNEL_STAGES if n in stages), key=lambda n: stages[n]["ms"])
    shape = shape_of(rast, opts)
    tr = counter_traffic(dom, args.workload, shape)
    if dom == "fwd.blend":
        # lane-ops per launch: 4 per thread visit (dx, the two x-terms, the
        # column test), 9 per evaluated pair (dy, the two whitened
        # coordinates, q, exp2, opacity product, alpha_max clamp, alpha_min
        # test), 8 more per pair that blends (1 - alpha, T (1 - alpha), the
        # T_min test, w, three colour and one depth FMA)
        ops = visited * 4 + evaluated * 9 + blended * 8
        ach = ops / (stages[dom]["ms"] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": round(ach, 3),
                "peak": round(VALU_PEAK_TOPS, 2), "unit": "Tlane-op/s",
                "frac": round(ach / VALU_PEAK_TOPS, 4), "ms_per_launch": stages[dom]["ms"],
                "lane_ops_per_launch": int(ops)}
    else:
        b = stages[dom]["alg_bytes"]
        ach = b / (stages[dom]["ms"] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "ms_per_launch": stages[dom]["ms"], "alg_bytes_per_launch": int(b)}
    roof["traffic"] = tr["bytes"] if tr else None
    if tr:
        roof["traffic_source"] = tr["file"]
    roof["shape"] = shape

    # the backward blend (the largest kernel of forward + backward): 4
    # lane-ops per thread visit (column test, dx, the two x-terms), 9 per
    # evaluated pair (as the forward), 32 per pair that carries a gradient
    # (1 / (1 - alpha), T, w, three colour gradients, the colour dot product,
    # dL/dalpha, the running sum behind, the clamp test, dL/dopacity and the
    # five mean and conic gradients), and per wave reduction the 9 x 63
    # additions that sum nine values over 64 lanes
    roof_bwd = None
    if "bwd.blend" in stages:
        bv, be, bb, br = bwd_work
        ops_b = 4 * bv + 9 * be + 32 * bb + 9 * 63 * br
        ms_b = stages["bwd.blend"]["ms"]
        ach_b = ops_b / (ms_b * 1e-3) / 1e12
        shape_b = shape_of(m["rast_b"], m["opts_b"])
        tr_b = counter_traffic("bwd.blend", args.workload, shape_b)
        roof_bwd = {"kernel": "bwd.blend", "bound": "alu", "achieved": round(ach_b, 3),
                    "peak": round(VALU_PEAK_TOPS, 2), "unit": "Tlane-op/s",
                    "frac": round(ach_b / VALU_PEAK_TOPS, 4), "ms_per_launch": ms_b,
                    "lane_ops_per_launch": int(ops_b),
                    "work": {"visited": bv, "evaluated": be, "blended": bb, "reductions": br},
                    "atomic_instructions": br, "traffic": tr_b["bytes"] if tr_b else None,
                    "shape": shape_b}
        if tr_b:
            roof_bwd["traffic_source"] = tr_b["file"]

    result = {
        "metric": ("frames/s & fwd+bwd ms at 3M Gaussians 1600x1060, SG vs SH-3 form, same GPU"
                   if args.workload == "sg-3m-1600" else f"frames/s & fwd+bwd ms, {args.workload}"),
        "value": round(1000.0 / m["fwd_graph_ms"], 2), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(m["fwd_graph_ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "gaussians": sc.n, "cameras": len(cams),
                   "width": W, "height": H, "colour": f"SH{sc.sh_degree}+{sc.n_lobes}SG",
                   "fwd_shape": shape, "fwd_bwd_shape": shape_of(m["rast_b"], m["opts_b"])},
        "fwd_bwd_ms": round(m["fb_graph_ms"], 4),
        "eager": {"frames_per_s": round(1000.0 / m["fwd_ms"], 2), "fwd_ms": round(m["fwd_ms"], 4),
                  "fwd_bwd_ms": round(m["fb_ms"], 4)},
        "pairs": int(P), "visible": n_vis, "tiles": tiles, "strips": strips, "strip_entries": E,
        "blend_visited": visited, "blend_evaluated": evaluated, "blend_blended": blended,
        "stages": stages, "binning": binning, "roofline": roof, "roofline_bwd": roof_bwd,
        # the paper's own rendering speed (Table 1: trained Mip-NeRF360
        # scenes, one RTX 3090, Gaussian counts not given): context only
        "paper_context": {"hardware": "RTX 3090", "scenes": "Mip-NeRF360, trained",
                          "fps_3dgs_sh3": 247, "fps_sg_splatting": 334},
    }
    if m["reports"]:
        result["autotune"] = m["reports"]
    # per-tile load (list lengths), e.g. for the stress workload
    rng = rast.ranges().cpu().numpy().view(np.uint32).astype(np.int64)
    cnt = rng[:, 1] - rng[:, 0]
    bins = np.bincount(np.ceil(np.log2(np.maximum(cnt, 1))).astype(np.int64))
    result["tile_load"] = {"p50": float(np.percentile(cnt, 50)), "p90": float(np.percentile(cnt, 90)),
                           "p99": float(np.percentile(cnt, 99)), "max": int(cnt.max()),
                           "empty": int((cnt == 0).sum()),
                           "log2_bins": {f"<=2^{i}": int(b) for i, b in enumerate(bins) if b}}

    # the same SG form with its colour stored as bfloat16 (the bandwidth side
    # of the compact model): block timings and the colour-dependent stages
    if args.workload == "sg-3m-1600" and not args.no_sh3:
        mh = measure_form(args, *mods, sc, cams, base, target, colour_dtype=torch.bfloat16)
        st_h = {nm: round((mh["st_fwd"] if nm.startswith("fwd") else mh["st_fb"])[i] /
                          max(mh["nf"] if nm.startswith("fwd") else mh["nb"], 1), 5)
                for i, nm in enumerate(names)}
        result["colour_bf16"] = {"fwd_ms": round(mh["fwd_graph_ms"], 4),
                                 "fwd_bwd_ms": round(mh["fb_graph_ms"], 4),
                                 "fwd_ms_f32_same_run": round(m["fwd_graph_ms"], 4),
                                 "fwd_bwd_ms_f32_same_run": round(m["fb_graph_ms"], 4),
                                 "preprocess_ms": st_h["fwd.preprocess"],
                                 "bwd_preprocess_ms": st_h["bwd.preprocess"],
                                 "colour_bytes_per_visible_gaussian": 2 * 40}
        del mh

    stat_steps = max(100, args.steps)
    if not args.no_sh3 and args.workload == "sg-3m-1600":
        sh3 = scenes.sh3_scene(sc.n, 1)
        m3 = measure_form(args, *mods, sh3, cams, base, target)
        i_pre = names.index("fwd.preprocess")
        result["sh3"] = {"frames_per_s": round(1000.0 / m3["fwd_graph_ms"], 2),
                         "fwd_ms": round(m3["fwd_graph_ms"], 4),
                         "fwd_bwd_ms": round(m3["fb_graph_ms"], 4),
                         "eager_fwd_ms": round(m3["fwd_ms"], 4),
                         "eager_fwd_bwd_ms": round(m3["fb_ms"], 4),
                         "preprocess_ms": round(m3["st_fwd"][i_pre] / max(m3["nf"], 1), 5),
                         "stages_ms": {nm: round((m3["st_fwd"] if nm.startswith("fwd") else
                                                  m3["st_fb"])[i] /
                                                 max(m3["nf"] if nm.startswith("fwd") else m3["nb"], 1), 5)
                                       for i, nm in enumerate(names)},
                         "fwd_shape": shape_of(m3["rast"], m3["opts_f"]),
                         "fwd_bwd_shape": shape_of(m3["rast_b"], m3["opts_b"])}
        # the two forms' own loops move with the GPU clock between them; the
        # headline ratios come from the paired replays in alternation
        result["sg_over_sh3_fps_unpaired"] = round(m3["fwd_graph_ms"] / (1000.0 / result["value"]), 4)
        result["sg_over_sh3_fwd_bwd_unpaired"] = round(m3["fb_graph_ms"] / result["fwd_bwd_ms"], 4)
        paired, sg_fwd, sg_fb = paired_comparison(m, m3, stat_steps, torch)
        result["sg_vs_sh3_paired"] = paired
        result["sg_over_sh3_fps"] = paired["sg_over_sh3_fps"]
        result["sg_over_sh3_fps_ci95"] = paired["sg_over_sh3_fps_ci95"]
        result["sg_over_sh3_fwd_bwd"] = paired["sg_over_sh3_fwd_bwd"]
        result["sg_over_sh3_fwd_bwd_ci95"] = paired["sg_over_sh3_fwd_bwd_ci95"]
        del m3
    else:
        sg_fwd, sg_fb = alternating_steps([m["g_fwd"].replay, m["g_fb"].replay], stat_steps, torch)
    # the headline: medians of the per-step samples (the paired run's SG
    # samples when the SH-3 form is measured too)
    med_f, med_fb = float(np.median(sg_fwd)), float(np.median(sg_fb))
    result["value"] = round(1000.0 / med_f, 2)
    result["ms_per_step"] = round(med_f, 4)
    result["fwd_bwd_ms"] = round(med_fb, 4)
    result["timing"] = {"fwd": summary(sg_fwd), "fwd_bwd": summary(sg_fb),
                        "block_fwd_ms": round(m["fwd_graph_ms"], 4),
                        "block_fwd_bwd_ms": round(m["fb_graph_ms"], 4),
                        "note": ("value and ms_per_step: median of per-step HIP-event times of "
                                 "the forward's graph replay; block_*: mean of one K-step block")}
    if len(cams) > 1:
        result["views_per_s"] = round(len(cams) * 1000.0 / med_f, 2)
    del m, rast
    torch.cuda.empty_cache()

    if cpu is not None:
        cpu["gpu_speedup_fwd"] = round(cpu["frame_s"] * 1e3 / result["ms_per_step"], 1)
        cpu["gpu_speedup_fwd_bwd"] = round(cpu["fwd_bwd_s"] * 1e3 / result["fwd_bwd_ms"], 1)
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
