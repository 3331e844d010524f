"""Tile-parallel runs of the oracle's blend on the host's cores — TEST
INFRASTRUCTURE ONLY (the tests and the benchmark's CPU-baseline leg).

The per-tile work is `forward.blend_image` and `backward.blend_backward`,
unchanged: this module only deals the tiles of a frame out to worker
processes and merges what they return.  Every pixel belongs to exactly one
tile, so forward results are placed, not combined; the backward's
per-Gaussian sums are added in float64 in the parent (a different order of
float64 additions than one sequential pass, which changes results only at
the level of float64 rounding).

Workers are forked, so they read the parent's preprocess arrays without a
copy; they run NumPy only.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from . import backward as B
from . import forward as F

_JOB = {}


def workers(limit: int = 12) -> int:
    """Worker processes to use: the host's cores, at most `limit`."""
    return max(1, min(int(limit), os.cpu_count() or 1))


def _chunks(tiles, n):
    tiles = list(tiles)
    n = max(1, min(n, len(tiles)))
    # interleaved, so that heavy neighbouring tiles spread over the workers
    return [tiles[i::n] for i in range(n)]


def _fwd_chunk(tiles):
    pre, cam, opts, values, ranges, cam_index, tile_base = _JOB["fwd"]
    img, dep, T, n, fl, alts = F.blend_image(pre, cam, opts, values, ranges,
                                             cam_index=cam_index, tile_base=tile_base,
                                             tiles=tiles)
    GX = pre.grid[0]
    pys, pxs = [], []
    for t in tiles:
        px, py = F.tile_pixels(t % GX, t // GX, opts, int(cam.width), int(cam.height))
        pys.append(py)
        pxs.append(px)
    py = np.concatenate(pys) if pys else np.zeros(0, np.int64)
    px = np.concatenate(pxs) if pxs else np.zeros(0, np.int64)
    return py, px, img[:, py, px], dep[py, px], T[py, px], n[py, px], fl[py, px], alts


def blend_image(pre, cam, opts, values, ranges, cam_index=0, tile_base=0, tiles=None,
                n_workers=None):
    """`forward.blend_image` over the frame's tiles on `n_workers` processes;
    same return value."""
    GX, GY = pre.grid
    todo = list(range(GX * GY)) if tiles is None else list(tiles)
    W, H = int(cam.width), int(cam.height)
    image = np.zeros((3, H, W))
    depth = np.zeros((H, W))
    final_T = np.ones((H, W))
    ncon = np.zeros((H, W), np.int64)
    flagged = np.zeros((H, W), bool)
    alts = {}
    nw = workers() if n_workers is None else max(1, int(n_workers))
    _JOB["fwd"] = (pre, cam, opts, values, ranges, cam_index, tile_base)
    try:
        if nw == 1:
            parts = [_fwd_chunk(todo)]
        else:
            with mp.get_context("fork").Pool(nw) as pool:
                parts = pool.map(_fwd_chunk, _chunks(todo, 4 * nw))
    finally:
        _JOB.pop("fwd", None)
    for py, px, c, d, t, n, fl, a in parts:
        image[:, py, px] = c
        depth[py, px] = d
        final_T[py, px] = t
        ncon[py, px] = n
        flagged[py, px] = fl
        alts.update(a)
    return image, depth, final_T, ncon, flagged, alts


def _bwd_chunk(tiles):
    pre, cam, opts, values, ranges, gimg, cam_index, tile_base, gdep, galp = _JOB["bwd"]
    out = B.blend_backward(pre, cam, opts, values, ranges, gimg, cam_index=cam_index,
                           tile_base=tile_base, tiles=tiles, grad_depth=gdep,
                           grad_alpha=galp)
    names = B.GRAD2D + ("z",)
    stack = np.stack([out[k] for k in names])
    idx = np.nonzero(np.any(stack != 0.0, axis=0))[0]
    return idx, stack[:, idx]


def blend_backward(pre, cam, opts, values, ranges, grad_image, cam_index=0, tile_base=0,
                   tiles=None, grad_depth=None, grad_alpha=None, n_workers=None):
    """`backward.blend_backward` over the frame's tiles on `n_workers`
    processes; same return value (per-Gaussian sums added in the parent)."""
    GX, GY = pre.grid
    todo = list(range(GX * GY)) if tiles is None else list(tiles)
    n = pre.z.shape[0]
    names = B.GRAD2D + ("z",)
    total = np.zeros((len(names), n))
    nw = workers() if n_workers is None else max(1, int(n_workers))
    _JOB["bwd"] = (pre, cam, opts, values, ranges, grad_image, cam_index, tile_base,
                   grad_depth, grad_alpha)
    try:
        if nw == 1:
            parts = [_bwd_chunk(todo)]
        else:
            with mp.get_context("fork").Pool(nw) as pool:
                parts = pool.map(_bwd_chunk, _chunks(todo, 4 * nw))
    finally:
        _JOB.pop("bwd", None)
    for idx, vals in parts:
        total[:, idx] += vals
    return {k: total[i] for i, k in enumerate(names)}
