"""Autotuner for the rasteriser's launch shape.

Picks the tile shape, the pixels per thread of the forward and backward
blends, the LDS batch depth and the tile schedule (one workgroup per tile or
the persistent heavy-first queue) by timing the candidates on the caller's own
scene and cameras, and caches the winner in a JSON file keyed by (GPU
architecture, camera sizes, Gaussian-count bucket, colour form, pass).
The rendered image does not depend on the choice (the splat footprint is an
integer pixel rectangle, independent of the tile shape); n_contrib counts
positions in the chosen tile's list.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import asdict, replace

from .scenes import Options

# (tile_w, tile_h) -> allowed pixels per thread (block = whole waves)
TILE_PPT = {
    (16, 16): (1, 2, 4),
    (32, 8): (1, 2, 4),
    (16, 8): (1, 2),
    (8, 16): (1, 2),
    (8, 8): (1,),
}
BATCHES = (128, 256, 512)
SCHEDULES = (1, 2, 3)   # grid, heavy-first queue, heavy-first one-wave slices


def default_cache_path() -> str:
    base = os.environ.get("SGSPLAT_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "sgsplat"))
    return os.path.join(base, "autotune.json")


def cache_key(arch: str, cams, n: int, sh_degree: int, n_lobes: int, backward: bool) -> str:
    sizes = sorted({(int(c.width), int(c.height)) for c in cams})
    bucket = 0 if n <= 0 else int(math.ceil(math.log2(n)))
    size_s = ",".join(f"{w}x{h}" for w, h in sizes)
    return (f"v2|{arch}|{size_s}|cams{len(cams)}|n2^{bucket}|sh{sh_degree}k{n_lobes}|"
            f"{'fwdbwd' if backward else 'fwd'}")


def candidates(tiles=None, batches=BATCHES, backward=True, schedules=SCHEDULES):
    """Every valid (tile, ppt, ppt_bwd, batch, schedule) combination."""
    out = []
    for (tw, th), ppts in TILE_PPT.items():
        if tiles is not None and (tw, th) not in tiles:
            continue
        for b in batches:
            for p in ppts:
                for pb in (ppts if backward else (ppts[0],)):
                    for sc in schedules:
                        out.append({"tile_w": tw, "tile_h": th, "ppt": p, "ppt_bwd": pb,
                                    "batch": b, "schedule": sc})
    return out


# choices measured on MI355X for the standard workloads, shipped with the
# package; a user cache entry of the same key takes precedence
PACKAGED_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_gfx950.json")


def load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(key: str, cache_path: str | None = None):
    """Cached entry for `key`: the user cache first, then the packaged table."""
    for p in (cache_path or default_cache_path(), PACKAGED_TABLE):
        ent = load_cache(p).get(key)
        if ent is not None:
            return ent
    return None


def save_cache(path: str, cache: dict) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(params: dict, cams, base: Options, n: int, sh_degree: int, n_lobes: int,
         backward: bool = True, reps: int = 5, tiles=None, batches=BATCHES,
         cache_path: str | None = None, use_cache: bool = True, target=None,
         schedules=SCHEDULES):
    """Time every candidate and return (best Options, report list).

    params: device tensors of the scene (raster.params_to_device).  With
    `backward`, a candidate is timed on forward + L1 + backward, else on the
    forward alone.
    """
    import torch

    from . import raster

    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    key = cache_key(arch, cams, n, sh_degree, n_lobes, backward)
    cache_path = cache_path or default_cache_path()
    if use_cache:
        ent = lookup(key, cache_path)
        if ent is not None:
            return replace(base, **ent["choice"]), ent["report"]

    if target is None and backward:
        target = torch.rand(3 * sum(int(c.width) * int(c.height) for c in cams),
                            device=next(iter(params.values())).device)
    report = []
    best, best_ms = None, float("inf")
    from ._lib import SgsError
    for cand in candidates(tiles, batches, backward, schedules):
        opts = replace(base, **cand)
        rast = raster.Rasterizer(cams, opts, n, sh_degree, n_lobes)
        try:
            out = rast.forward(params, check=True)
        except SgsError as e:     # e.g. more pairs than one call may hold
            report.append(dict(cand, ms=None, error=str(e)))
            del rast
            continue
        gimg = torch.empty_like(out.image)
        grads = raster.new_grads(params)

        def step():
            rast.forward(params, out=out, check=False)
            if backward:
                rast.l1(out.image, target, grad_out=gimg)
                rast.backward_into(params, out, gimg, grads)

        step()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            step()
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / reps
        report.append(dict(cand, ms=round(ms, 4)))
        if ms < best_ms:
            best, best_ms = cand, ms
        del rast, out, gimg, grads
    torch.cuda.empty_cache()
    if use_cache:
        cache = load_cache(cache_path)
        cache[key] = {"choice": best, "report": report}
        save_cache(cache_path, cache)
    return replace(base, **best), report


__all__ = ["tune", "candidates", "cache_key", "load_cache", "save_cache", "default_cache_path",
           "lookup", "PACKAGED_TABLE",
           "TILE_PPT", "BATCHES", "SCHEDULES", "asdict"]
