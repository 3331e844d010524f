"""Shared set-up for the GPU tests: run the HIP path on a scene and pull
its results to NumPy."""
from __future__ import annotations

import numpy as np
import torch

from paper_2501_00342_amd import raster
from paper_2501_00342_amd.scenes import Scene


def run_forward(scene: Scene, cams, opts, capacity=None, check=True):
    rast = raster.Rasterizer.for_scene(scene, cams, opts,
                             device="cuda", capacity=capacity)
    params = raster.params_to_device(scene)
    out = rast.forward(params, check=check)
    torch.cuda.synchronize()
    return rast, params, out


def camera_numpy(out, cams, k=0):
    img, dep, T, n = out.camera(k, cams)
    return (img.cpu().numpy().astype(np.float64), dep.cpu().numpy().astype(np.float64),
            T.cpu().numpy().astype(np.float64), n.cpu().numpy().astype(np.int64))


def pairs_count(rast):
    bits, pairs = rast.status()
    return bits, pairs


def records_numpy(rast):
    rec = rast.records().cpu().numpy()
    ints = rec.view(np.uint32)
    return rec, ints
