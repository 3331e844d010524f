"""PyTorch front end of the HIP rasteriser.

PyTorch supplies device memory and the stream; every step of the render
runs in libsgsplat.so.  `Rasterizer` owns one workspace (records, pairs,
ranges) that a backward reuses from its forward; `render` wraps it in a
torch.autograd.Function.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L
from .scenes import FIELDS, Options, Scene

REC_FIELDS = ("u_hi", "v_hi", "u_lo", "v_lo", "w1x", "w1y", "w2x", "w2y", "opacity",
              "r", "g", "b", "z", "rect_x", "rect_y", "radius")


# The C-ABI keeps the geometry component-major ((C, N) rows, read for every
# Gaussian) and the colour Gaussian-major ((N, ...), read only for Gaussians
# that survive culling); a Scene holds every array component-major.
COLOUR_FIELDS = ("sh", "sg_axes", "sg_log_sharpness", "sg_amplitudes")


def to_device_layout(name: str, a: np.ndarray) -> np.ndarray:
    """One Scene array in the C-ABI layout: colour (..., N) -> (N, ...)."""
    if name in COLOUR_FIELDS:
        return np.ascontiguousarray(np.moveaxis(a, -1, 0))
    return np.ascontiguousarray(a)


def to_scene_layout(arrays: dict) -> dict:
    """Arrays in the C-ABI layout (parameters or gradients, numpy) in the
    Scene's component-major layout: colour (N, ...) -> (..., N)."""
    return {k: (np.ascontiguousarray(np.moveaxis(v, 0, -1)) if k in COLOUR_FIELDS else v)
            for k, v in arrays.items()}


def colour_record_floats(sh_degree: int, n_lobes: int, lobe_mode: int = L.LOBES_FREE) -> int:
    """Floats of one Gaussian's colour: SH, axis rows, sharpness, amplitudes."""
    from .scenes import axis_vectors
    return 3 * (sh_degree + 1) ** 2 + 3 * axis_vectors(lobe_mode, n_lobes) + 4 * n_lobes


COLOUR_DTYPES = {torch.float32: L.COLOUR_F32, torch.bfloat16: L.COLOUR_BF16,
                 torch.float16: L.COLOUR_F16}


def params_to_device(scene: Scene, device="cuda", packed: bool = True,
                     colour_dtype=torch.float32) -> dict:
    """Scene arrays -> device tensors in the C-ABI layout: the geometry in
    float32, the colour in `colour_dtype` (float32, or bfloat16 / float16
    storage: the float32 values rounded to nearest even).

    packed: the four colour tensors are views into one (N, S) buffer, each
    Gaussian's colour one contiguous record of 3 (L+1)^2 + 3 A + 4 K
    elements and S that rounded up to whole 16-byte pieces (the layout the
    rasteriser fetches fastest); otherwise each colour tensor is contiguous
    on its own."""
    def dev(k):
        t = torch.from_numpy(to_device_layout(k, getattr(scene, k))).to(device)
        return t.to(colour_dtype) if k in COLOUR_FIELDS else t
    out = {k: dev(k) for k in FIELDS if k not in COLOUR_FIELDS or not packed}
    if packed:
        n, nc3, K = scene.n, 3 * (scene.sh_degree + 1) ** 2, scene.n_lobes
        A = scene.n_axis_vectors
        rs = nc3 + 3 * A + 4 * K
        w = 16 // torch.tensor([], dtype=colour_dtype).element_size()
        rec = torch.zeros((n, (rs + w - 1) // w * w), dtype=colour_dtype, device=device)
        at = 0
        for k, width in (("sh", nc3), ("sg_axes", 3 * A), ("sg_log_sharpness", K),
                         ("sg_amplitudes", 3 * K)):
            a = dev(k)
            view = rec[:, at:at + width].view(a.shape)
            view.copy_(a)
            out[k] = view
            at += width
    return out


def colour_dtype_code(params: dict) -> int:
    """The colour_dtype of the C-ABI for these tensors (one type for all four)."""
    types = {params[k].dtype for k in COLOUR_FIELDS}
    assert len(types) == 1, "colour tensors of different types"
    return COLOUR_DTYPES[types.pop()]


def colour_stride(params: dict) -> int:
    """The colour_stride of the C-ABI for these tensors: 0 when every colour
    tensor is contiguous, else their common first-dimension stride."""
    cols = [params[k] for k in COLOUR_FIELDS if params[k].numel()]
    if all(t.is_contiguous() for t in cols):
        return 0
    st = {t.stride(0) for t in cols}
    assert len(st) == 1, "colour tensors with different strides"
    for t in cols:   # each Gaussian's block is dense
        assert t[0].is_contiguous(), "colour blocks are not contiguous"
    return st.pop()


def new_grads(params: dict) -> dict:
    """Gradient tensors for `params`: the shapes of the parameters, every
    array packed (the layout the backward writes)."""
    return {k: torch.empty(tuple(v.shape), dtype=torch.float32, device=v.device)
            for k, v in params.items()}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if (t is not None and t.numel() > 0) else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class Outputs:
    image: torch.Tensor      # packed (3 * sum W H,) float32
    depth: torch.Tensor      # packed (sum W H,)
    final_T: torch.Tensor
    n_contrib: torch.Tensor  # int32
    alpha: torch.Tensor | None = None   # packed (sum W H,): 1 - final_T, when asked for

    def struct(self) -> "L.Outputs":
        return L.Outputs(_ptr(self.image), _ptr(self.depth), _ptr(self.final_T),
                         _ptr(self.n_contrib), _ptr(self.alpha))

    def camera(self, k: int, cams) -> tuple:
        """(image (3,H,W), depth, final_T, n_contrib) views of camera k."""
        base = sum(int(c.width) * int(c.height) for c in cams[:k])
        W, H = int(cams[k].width), int(cams[k].height)
        img = self.image[3 * base: 3 * (base + W * H)].view(3, H, W)
        sl = slice(base, base + W * H)
        return (img, self.depth[sl].view(H, W), self.final_T[sl].view(H, W),
                self.n_contrib[sl].view(H, W))


class Rasterizer:
    """Plans and runs forward/backward passes for fixed cameras and options.

    capacity: initial (tile, Gaussian) pair capacity; grown automatically
    when `auto_grow` and a forward reports more pairs (one host sync).
    """

    def __init__(self, cams, opts: Options, n: int, sh_degree: int, n_lobes: int,
                 device="cuda", capacity: int | None = None, auto_grow: bool = True,
                 lobe_mode: int = L.LOBES_FREE, sh_adaptive=(0, 0)):
        self.cams = list(cams)
        self.opts = opts
        self.n, self.sh_degree, self.n_lobes = int(n), int(sh_degree), int(n_lobes)
        self.lobe_mode, self.sh_adaptive = int(lobe_mode), tuple(int(t) for t in sh_adaptive)
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.host_cams = L.camera_array(self.cams)
        raw = bytes(self.host_cams)
        self.dev_cams = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(self.device)
        self.copts = L.options_struct(opts)
        self.n_pixels = sum(int(c.width) * int(c.height) for c in self.cams)
        self.auto_grow = auto_grow
        self.capacity = int(capacity if capacity is not None else max(1 << 16, 8 * self.n))
        self.capacity = min(self.capacity, (1 << 30) - 1)
        self.ws = None
        self.layout = None
        # bumped by every forward and every reallocation: the workspace then
        # holds another render's records, pairs and ranges
        self.generation = 0
        self._alloc()

    @classmethod
    def for_scene(cls, scene: Scene, cams, opts: Options, **kw) -> "Rasterizer":
        """A Rasterizer for the colour form of `scene` (degree, lobes, lobe
        mode, adaptive SH thresholds)."""
        return cls(cams, opts, scene.n, scene.sh_degree, scene.n_lobes,
                   lobe_mode=scene.lobe_mode, sh_adaptive=scene.sh_adaptive, **kw)

    # -- planning ----------------------------------------------------------
    def _gstruct(self, params: dict | None):
        ptrs = {k: (params[k].data_ptr() if params[k].numel() else None) for k in FIELDS} \
            if params else {}
        cs = colour_stride(params) if params else 0
        ct = colour_dtype_code(params) if params else L.COLOUR_F32
        return L.gaussians_struct(self.n, self.sh_degree, self.n_lobes, ptrs, cs,
                                  self.lobe_mode, self.sh_adaptive, ct)

    def _alloc(self):
        g = self._gstruct(None)
        lay = L.Layout()
        L.check(L.LIB.render_layout(ctypes.byref(g), self.host_cams, len(self.cams),
                                    ctypes.byref(self.copts), self.capacity, ctypes.byref(lay)))
        self.layout = lay
        self.ws = torch.empty(int(lay.total_bytes), dtype=torch.uint8, device=self.device)
        self.generation += 1

    def new_outputs(self, alpha: bool = False) -> Outputs:
        P = self.n_pixels
        d = self.device
        return Outputs(torch.empty(3 * P, dtype=torch.float32, device=d),
                       torch.empty(P, dtype=torch.float32, device=d),
                       torch.empty(P, dtype=torch.float32, device=d),
                       torch.empty(P, dtype=torch.int32, device=d),
                       torch.empty(P, dtype=torch.float32, device=d) if alpha else None)

    def _check_params(self, params):
        for k in FIELDS:
            t = params[k]
            assert t.device == self.device, k
            assert t.dtype == torch.float32 or (k in COLOUR_FIELDS and t.dtype in COLOUR_DTYPES), k
            if k in COLOUR_FIELDS:
                assert t.shape[0] == self.n or t.numel() == 0, k
            else:
                assert t.is_contiguous() and (t.shape[-1] == self.n or t.numel() == 0), k
        colour_stride(params)   # the colour tensors share one layout
        colour_dtype_code(params)   # and one element type

    # -- passes --------------------------------------------------------------
    def forward(self, params: dict, out: Outputs | None = None, check: bool | None = None) -> Outputs:
        self._check_params(params)
        out = out or self.new_outputs()
        check = self.auto_grow if check is None else check
        g = self._gstruct(params)
        o = out.struct()
        need = L.c_int64(0)
        flags = L.SGS_FLAG_CHECK_CAPACITY if check else 0
        self.generation += 1
        while True:
            rc = L.LIB.render_forward(ctypes.byref(g), self.host_cams, _ptr(self.dev_cams),
                                      len(self.cams), ctypes.byref(self.copts), _ptr(self.ws),
                                      self.ws.numel(), self.capacity, ctypes.byref(o), flags,
                                      ctypes.byref(need), _stream())
            if rc == L.SGS_E_CAPACITY and self.auto_grow:
                if need.value > (1 << 30) - 1:
                    raise L.SgsError(L.SGS_E_CAPACITY, f"{need.value} pairs exceed the 2^30 - 1 "
                                     "pair limit of one call; render fewer cameras per call")
                self.capacity = min((1 << 30) - 1, int(need.value * 1.15) + 4096)
                self.ws = None
                torch.cuda.current_stream().synchronize()
                self._alloc()
                continue
            L.check(rc)
            return out

    def backward(self, params: dict, out: Outputs, grad_image: torch.Tensor,
                 grad_depth: torch.Tensor | None = None,
                 grad_alpha: torch.Tensor | None = None) -> dict:
        grads = new_grads(params)
        self.backward_into(params, out, grad_image, grads, grad_depth, grad_alpha)
        return grads

    def backward_into(self, params: dict, out: Outputs, grad_image: torch.Tensor,
                      grads: dict, grad_depth: torch.Tensor | None = None,
                      grad_alpha: torch.Tensor | None = None) -> dict:
        """Backward writing into preallocated gradient tensors (no allocation:
        usable under stream capture).  grad_depth / grad_alpha: optional
        upstream gradients of the depth and accumulated-alpha images."""
        self._check_params(params)
        assert grad_image.dtype == torch.float32 and grad_image.is_contiguous()
        assert grad_image.numel() == 3 * self.n_pixels
        for t in (grad_depth, grad_alpha):
            assert t is None or (t.dtype == torch.float32 and t.is_contiguous()
                                 and t.numel() == self.n_pixels)
        for k in FIELDS:   # the backward writes every gradient array packed
            assert grads[k].is_contiguous() and grads[k].shape == params[k].shape, k
        g = self._gstruct(params)
        gr = L.grads_struct({k: (grads[k].data_ptr() if grads[k].numel() else None)
                             for k in FIELDS})
        o = out.struct()
        L.check(L.LIB.render_backward(ctypes.byref(g), self.host_cams, _ptr(self.dev_cams),
                                      len(self.cams), ctypes.byref(self.copts), _ptr(self.ws),
                                      self.ws.numel(), self.capacity, ctypes.byref(o),
                                      _ptr(grad_image), _ptr(grad_depth), _ptr(grad_alpha),
                                      ctypes.byref(gr), _stream()))
        return grads

    def l1(self, image: torch.Tensor, target: torch.Tensor, grad_out: torch.Tensor | None = None):
        """(loss as a device float64 scalar, dL/dimage)."""
        grad = grad_out if grad_out is not None else torch.empty_like(image)
        loss = torch.empty((), dtype=torch.float64, device=self.device)
        L.check(L.LIB.render_l1(self.host_cams, len(self.cams), _ptr(self.ws), _ptr(image),
                                _ptr(target), _ptr(grad), _ptr(loss), _stream()))
        return loss, grad

    def blend_work(self, params: dict) -> tuple:
        """(visited, evaluated, blended) pixel-entry pairs of the last forward."""
        counts = torch.zeros(3, dtype=torch.int64, device=self.device)
        g = self._gstruct(params)
        L.check(L.LIB.render_blend_work(ctypes.byref(g), self.host_cams, _ptr(self.dev_cams),
                                        len(self.cams), ctypes.byref(self.copts), _ptr(self.ws),
                                        self.ws.numel(), self.capacity, _ptr(counts), _stream()))
        c = counts.cpu()
        return int(c[0]), int(c[1]), int(c[2])

    def blend_bwd_work(self, params: dict, out: "Outputs") -> tuple:
        """(visited, evaluated, blended, reductions) of the backward blend's
        walk over the forward that produced `out`."""
        counts = torch.zeros(4, dtype=torch.int64, device=self.device)
        g = self._gstruct(params)
        o = out.struct()
        L.check(L.LIB.render_blend_bwd_work(ctypes.byref(g), self.host_cams, _ptr(self.dev_cams),
                                            len(self.cams), ctypes.byref(self.copts),
                                            _ptr(self.ws), self.ws.numel(), self.capacity,
                                            ctypes.byref(o), _ptr(counts), _stream()))
        c = counts.cpu()
        return int(c[0]), int(c[1]), int(c[2]), int(c[3])

    def status(self) -> tuple:
        bits, pairs = L.c_uint32(0), L.c_int64(0)
        L.check(L.LIB.render_status(_ptr(self.ws), ctypes.byref(bits), ctypes.byref(pairs),
                                    _stream()))
        return int(bits.value), int(pairs.value)

    # -- inspection (tests) --------------------------------------------------
    def _view(self, off, count, dtype):
        nbytes = count * torch.tensor([], dtype=dtype).element_size()
        return self.ws[off: off + nbytes].view(dtype)

    def records(self) -> torch.Tensor:
        return self._view(self.layout.records, 16 * self.layout.n_items, torch.float32).view(-1, 16)

    def n_strips(self) -> int:
        return int(self.layout.n_strips)

    def header(self):
        """The 16 header words: status bits, pairs, visible items, the two
        tile-queue counters, first-level entries, second-level chunks."""
        return self._view(self.layout.header, 16, torch.int32)

    def depth_keys(self):
        return self._view(self.layout.depth_keys, self.layout.n_items, torch.int32)

    def tile_rects(self):
        return self._view(self.layout.tile_rects, self.layout.n_items, torch.int64)

    def ranges(self):
        return self._view(self.layout.ranges, 2 * self.layout.n_tiles, torch.int32).view(-1, 2)

    def pair_values(self, count):
        return self._view(self.layout.pair_values, count, torch.int32)

    def grad2d(self):
        """(10, items): d/d(u, v, Qa, Qb, Qc, opacity, r, g, b, z) of the last
        backward (row 9 only after one with a depth or alpha gradient)."""
        rec = self._view(self.layout.grad2d, 16 * self.layout.n_items, torch.float32).view(-1, 16)
        # records exist for the visible items only (depth key not all ones)
        vis = (self.depth_keys() != -1).unsqueeze(1)
        return torch.where(vis, rec[:, :10], torch.zeros_like(rec[:, :10])).t()

    def sorted_keys(self, count) -> torch.Tensor:
        keys = torch.empty(count, dtype=torch.int64, device=self.device)
        L.check(L.LIB.render_read_keys(_ptr(self.ws), ctypes.byref(self.layout), count,
                                       _ptr(keys), _stream()))
        return keys


class StaleWorkspaceError(RuntimeError):
    """A backward whose forward's workspace was overwritten by a later
    forward (or reallocated) on the same Rasterizer."""


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rast: Rasterizer, *params):
        p = dict(zip(FIELDS, params))
        out = rast.forward(p, out=rast.new_outputs(alpha=True))
        ctx.rast = rast
        ctx.generation = rast.generation
        ctx.out = out
        ctx.save_for_backward(*params)
        ctx.mark_non_differentiable(out.final_T, out.n_contrib)
        # unused outputs give None, not zeros: no depth or alpha pass then
        ctx.set_materialize_grads(False)
        return out.image, out.depth, out.alpha, out.final_T, out.n_contrib

    @staticmethod
    def backward(ctx, g_image, g_depth, g_alpha, *_):
        # the backward walks the tile lists of the workspace: they must still
        # be those of this forward
        if ctx.rast.generation != ctx.generation:
            raise StaleWorkspaceError(
                "the Rasterizer ran another forward (or regrew its workspace) after this "
                "render; its backward would read that render's tile lists.  Call backward "
                "before the next forward, or use one Rasterizer per pending render.")
        params = dict(zip(FIELDS, ctx.saved_tensors))
        if g_image is None:
            g_image = torch.zeros_like(ctx.out.image)
        grads = ctx.rast.backward(params, ctx.out, g_image.contiguous(),
                                  None if g_depth is None else g_depth.contiguous(),
                                  None if g_alpha is None else g_alpha.contiguous())
        return (None, *[grads[k] for k in FIELDS])


def render(rast: Rasterizer, params: dict):
    """Differentiable render: returns packed (image, depth, final_T,
    n_contrib); image and depth carry gradients to every parameter."""
    image, depth, alpha, final_T, n_contrib = _RenderFn.apply(rast, *[params[k] for k in FIELDS])
    return image, depth, final_T, n_contrib


def render_with_alpha(rast: Rasterizer, params: dict):
    """Differentiable render with the accumulated alpha (1 - final_T):
    returns packed (image, depth, alpha, final_T, n_contrib); image, depth
    and alpha carry gradients."""
    return _RenderFn.apply(rast, *[params[k] for k in FIELDS])
