"""Adam over the Gaussian parameters through the library's fused update
(render_adam_step): one launch per step, moments kept on the device.

The learning rates default to the 3D-GS ones, which the paper keeps
(Experiments, Implementation), and the SG lobe arrays join at iteration
`sg_start` (2,000 in the paper) with learning rate 0.0025.  The position
rate is scaled by the scene extent and decayed by the caller, as in 3D-GS.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from .scenes import FIELDS

# 3D-GS learning rates (position: initial value, times the scene extent);
# the SG lobes: the paper's 0.0025
DEFAULT_LR = {"means": 1.6e-4, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2,
              "sh": 2.5e-3, "sg_axes": 2.5e-3, "sg_log_sharpness": 2.5e-3,
              "sg_amplitudes": 2.5e-3}
SG_START = 2000


class Adam:
    """Fused Adam for the parameter tensors of one Rasterizer's colour form.

    params: the dict the rasteriser renders (updated in place).  Gradients
    are the packed tensors `Rasterizer.backward` returns."""

    def __init__(self, rast, params: dict, lr: dict | None = None, sg_start: int = SG_START,
                 betas=(0.9, 0.999), eps: float = 1e-15):
        self.rast = rast
        self.params = params
        self.lr = dict(DEFAULT_LR if lr is None else lr)
        self.sg_start = int(sg_start)
        self.betas, self.eps = betas, eps
        self.exp_avg = {k: torch.zeros(tuple(v.shape), dtype=torch.float32, device=v.device)
                        for k, v in params.items()}
        self.exp_avg_sq = {k: torch.zeros_like(t) for k, t in self.exp_avg.items()}
        self.step_count = 0

    @staticmethod
    def _grads_struct(d: dict) -> L.Grads:
        return L.grads_struct({k: (d[k].data_ptr() if d[k].numel() else None) for k in FIELDS})

    def step(self, grads: dict):
        self.step_count += 1
        cfg = L.Adam()
        for i, k in enumerate(FIELDS):
            cfg.lr[i] = float(self.lr.get(k, 0.0))
        cfg.beta1, cfg.beta2, cfg.eps = self.betas[0], self.betas[1], self.eps
        cfg.step, cfg.sg_start = self.step_count, self.sg_start
        for k in FIELDS:
            assert grads[k].is_contiguous() and grads[k].shape == self.params[k].shape, k
        g = self.rast._gstruct(self.params)
        L.check(L.LIB.render_adam_step(ctypes.byref(g), ctypes.byref(cfg),
                                       ctypes.byref(self._grads_struct(grads)),
                                       ctypes.byref(self._grads_struct(self.exp_avg)),
                                       ctypes.byref(self._grads_struct(self.exp_avg_sq)),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
