"""ctypes binding of libsgsplat.so (argument marshalling only).

The names mirror the C ABI declared in include/sgsplat.h.  Every call runs
in the HIP library; nothing here computes.  Importing this module without
the built library raises ImportError: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, c_char_p, c_double, c_float, c_int32, c_int64,
                    c_size_t, c_uint32, c_uint64, c_void_p)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsgsplat.so")

SGS_OK, SGS_E_INVALID, SGS_E_CAPACITY, SGS_E_HIP = 0, 1, 2, 3
SGS_STATUS_CAPACITY, SGS_STATUS_CAMERAS = 1, 2
SCHEDULE_GRID, SCHEDULE_QUEUE = 1, 2
SGS_FLAG_CHECK_CAPACITY = 1
COLOUR_F32, COLOUR_BF16, COLOUR_F16 = 0, 1, 2
NOALLOC_WORKSPACE_BYTES = 64 << 20
LOBES_FREE, LOBES_WORLD, LOBES_FRAME = 0, 1, 2
MAX_SH_DEGREE, MAX_LOBES, MAX_CAMERAS, MAX_IMAGE_SIDE = 3, 8, 1024, 32767


class Gaussians(Structure):
    _fields_ = [("n", c_int64), ("sh_degree", c_int32), ("n_lobes", c_int32),
                ("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p),
                ("opacity_logits", c_void_p), ("sh", c_void_p), ("sg_axes", c_void_p),
                ("sg_log_sharpness", c_void_p), ("sg_amplitudes", c_void_p),
                ("colour_stride", c_int64), ("lobe_axes", c_int32),
                ("sh_adaptive", c_int32 * 2), ("colour_dtype", c_int32)]


class Grads(Structure):
    _fields_ = [("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p),
                ("opacity_logits", c_void_p), ("sh", c_void_p), ("sg_axes", c_void_p),
                ("sg_log_sharpness", c_void_p), ("sg_amplitudes", c_void_p)]


class Camera(Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("R", c_float * 9), ("t", c_float * 3),
                ("fx", c_float), ("fy", c_float), ("cx", c_float), ("cy", c_float),
                ("znear", c_float), ("bg", c_float * 3)]


class Options(Structure):
    _fields_ = [("tile_w", c_int32), ("tile_h", c_int32), ("batch", c_int32),
                ("dilation", c_float), ("guard", c_float), ("alpha_min", c_float),
                ("alpha_max", c_float), ("t_min", c_float), ("pixels_per_thread", c_int32),
                ("pixels_per_thread_bwd", c_int32), ("schedule", c_int32)]


class Adam(Structure):
    _fields_ = [("lr", c_float * 8), ("beta1", c_double), ("beta2", c_double), ("eps", c_double),
                ("step", c_int32), ("sg_start", c_int32)]


class Outputs(Structure):
    _fields_ = [("image", c_void_p), ("depth", c_void_p), ("final_T", c_void_p),
                ("n_contrib", c_void_p), ("alpha", c_void_p)]


class Layout(Structure):
    _fields_ = [("total_bytes", c_size_t), ("header", c_size_t), ("cam_table", c_size_t),
                ("records", c_size_t), ("depth_keys", c_size_t), ("tile_rects", c_size_t),
                ("sorted_items", c_size_t), ("pair_offsets", c_size_t), ("pair_tiles", c_size_t),
                ("pair_values", c_size_t), ("ranges", c_size_t), ("grad2d", c_size_t),
                ("n_items", c_int64), ("n_tiles", c_int64), ("n_pixels", c_int64),
                ("pair_capacity", c_int64), ("n_strips", c_int64)]


EXPORTS = ("render_workspace_bytes", "render_layout", "render_forward", "render_forward_noalloc",
           "render_backward",
           "render_l1", "render_status", "render_read_keys", "render_set_timing",
           "render_stage_times", "render_stage_name", "render_blend_work",
           "render_blend_bwd_work", "render_adam_step", "render_last_error")
N_STAGES = 11


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run `python -m paper_2501_00342_amd.build` "
            "(the rasteriser has no non-HIP path)")
    lib = ctypes.CDLL(LIB_PATH)
    P = POINTER
    lib.render_workspace_bytes.restype = c_size_t
    lib.render_workspace_bytes.argtypes = [P(Gaussians), P(Camera), c_int32, P(Options), c_int64]
    lib.render_layout.restype = c_int32
    lib.render_layout.argtypes = [P(Gaussians), P(Camera), c_int32, P(Options), c_int64, P(Layout)]
    lib.render_forward.restype = c_int32
    lib.render_forward.argtypes = [P(Gaussians), P(Camera), c_void_p, c_int32, P(Options),
                                   c_void_p, c_size_t, c_int64, P(Outputs), c_int32,
                                   P(c_int64), c_void_p]
    lib.render_forward_noalloc.restype = c_int32
    lib.render_forward_noalloc.argtypes = [P(Gaussians), P(Camera), c_void_p, c_int32, P(Options),
                                           c_int64, P(Outputs), c_int32, P(c_int64), c_void_p]
    lib.render_backward.restype = c_int32
    lib.render_backward.argtypes = [P(Gaussians), P(Camera), c_void_p, c_int32, P(Options),
                                    c_void_p, c_size_t, c_int64, P(Outputs), c_void_p,
                                    c_void_p, c_void_p, P(Grads), c_void_p]
    lib.render_l1.restype = c_int32
    lib.render_l1.argtypes = [P(Camera), c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                              c_void_p, c_void_p]
    lib.render_status.restype = c_int32
    lib.render_status.argtypes = [c_void_p, P(c_uint32), P(c_int64), c_void_p]
    lib.render_read_keys.restype = c_int32
    lib.render_read_keys.argtypes = [c_void_p, P(Layout), c_int64, c_void_p, c_void_p]
    lib.render_set_timing.restype = c_int32
    lib.render_set_timing.argtypes = [c_int32]
    lib.render_stage_times.restype = c_int32
    lib.render_stage_times.argtypes = [P(c_float), c_int32, P(c_int32), P(c_int32)]
    lib.render_stage_name.restype = c_char_p
    lib.render_stage_name.argtypes = [c_int32]
    lib.render_blend_work.restype = c_int32
    lib.render_blend_work.argtypes = [P(Gaussians), P(Camera), c_void_p, c_int32, P(Options),
                                      c_void_p, c_size_t, c_int64, c_void_p, c_void_p]
    lib.render_blend_bwd_work.restype = c_int32
    lib.render_blend_bwd_work.argtypes = [P(Gaussians), P(Camera), c_void_p, c_int32, P(Options),
                                          c_void_p, c_size_t, c_int64, P(Outputs), c_void_p,
                                          c_void_p]
    lib.render_adam_step.restype = c_int32
    lib.render_adam_step.argtypes = [P(Gaussians), P(Adam), P(Grads), P(Grads), P(Grads), c_void_p]
    lib.render_last_error.restype = c_char_p
    lib.render_last_error.argtypes = []
    return lib


LIB = _load()


class SgsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sgsplat error {code}: {msg}")
        self.code = code


def check(code: int):
    if code != SGS_OK:
        raise SgsError(code, LIB.render_last_error().decode())


def stage_names():
    return [LIB.render_stage_name(i).decode() for i in range(N_STAGES)]


def stage_times():
    """(per-stage summed ms, forward calls, backward calls) since last query."""
    ms = (c_float * N_STAGES)()
    nf, nb = c_int32(0), c_int32(0)
    check(LIB.render_stage_times(ms, N_STAGES, ctypes.byref(nf), ctypes.byref(nb)))
    return list(ms), nf.value, nb.value


def last_error() -> str:
    return LIB.render_last_error().decode()


def camera_struct(cam) -> Camera:
    c = Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    for i, v in enumerate(cam.R.reshape(-1)):
        c.R[i] = float(v)
    for i in range(3):
        c.t[i] = float(cam.t[i])
        c.bg[i] = float(cam.bg[i])
    c.fx, c.fy, c.cx, c.cy, c.znear = cam.fx, cam.fy, cam.cx, cam.cy, cam.znear
    return c


def camera_array(cams):
    arr = (Camera * len(cams))()
    for i, cam in enumerate(cams):
        arr[i] = camera_struct(cam)
    return arr


def options_struct(opts) -> Options:
    o = Options()
    o.tile_w, o.tile_h, o.batch = int(opts.tile_w), int(opts.tile_h), int(opts.batch)
    o.dilation, o.guard = opts.dilation, opts.guard
    o.alpha_min, o.alpha_max, o.t_min = opts.alpha_min, opts.alpha_max, opts.t_min
    o.pixels_per_thread = int(getattr(opts, "ppt", 0))
    o.pixels_per_thread_bwd = int(getattr(opts, "ppt_bwd", 0))
    o.schedule = int(getattr(opts, "schedule", 0))
    return o


def gaussians_struct(n, sh_degree, n_lobes, ptrs: dict, colour_stride: int = 0,
                     lobe_axes: int = LOBES_FREE, sh_adaptive=(0, 0),
                     colour_dtype: int = 0) -> Gaussians:
    g = Gaussians()
    g.n, g.sh_degree, g.n_lobes = int(n), int(sh_degree), int(n_lobes)
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "sg_axes",
              "sg_log_sharpness", "sg_amplitudes"):
        setattr(g, k, ptrs.get(k) or None)
    g.colour_stride = int(colour_stride)
    g.lobe_axes = int(lobe_axes)
    g.sh_adaptive[0], g.sh_adaptive[1] = int(sh_adaptive[0]), int(sh_adaptive[1])
    g.colour_dtype = int(colour_dtype)
    return g


def grads_struct(ptrs: dict) -> Grads:
    g = Grads()
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "sg_axes",
              "sg_log_sharpness", "sg_amplitudes"):
        setattr(g, k, ptrs.get(k) or None)
    return g


__all__ = ["LIB", "LIB_PATH", "EXPORTS", "Gaussians", "Grads", "Camera", "Options", "Outputs", "Adam",
           "Layout", "check", "last_error", "SgsError", "camera_struct", "camera_array",
           "options_struct", "gaussians_struct", "grads_struct", "c_int64", "c_uint32",
           "c_double", "c_uint64"]
