"""Rounding of float32 colour parameters to the half-precision storage
types the rasteriser accepts (round to nearest, ties to even), for giving
the oracle exactly the values the device reads."""
from __future__ import annotations

import dataclasses

import numpy as np

COLOUR_FIELDS = ("sh", "sg_axes", "sg_log_sharpness", "sg_amplitudes")


def round_bf16(a) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).reshape(np.shape(a))


def round_f16(a) -> np.ndarray:
    """float32 -> nearest float16 (ties to even), returned as float32."""
    return np.asarray(a, np.float32).astype(np.float16).astype(np.float32)


def rounded_scene(scene, kind: str):
    """A copy of `scene` whose colour arrays hold the rounded values."""
    f = round_bf16 if kind == "bf16" else round_f16
    return dataclasses.replace(scene, **{k: f(getattr(scene, k)) for k in COLOUR_FIELDS})
