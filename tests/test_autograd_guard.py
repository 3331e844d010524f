"""The autograd Function refuses a backward whose forward's workspace was
overwritten by a later forward on the same Rasterizer (CPU: the rasteriser
is replaced by a stand-in that only counts calls)."""
import pytest
import torch

from paper_2501_00342_amd import raster
from paper_2501_00342_amd.scenes import FIELDS


class _StandIn:
    """Duck-typed Rasterizer: forward bumps the generation like the real
    one; backward returns zeros."""

    def __init__(self):
        self.generation = 1
        self.backwards = 0

    def forward(self, p, out=None):
        self.generation += 1
        n = 4
        return raster.Outputs(p["opacity_logits"].detach().repeat(3) * 1.0,
                              torch.zeros(n), torch.ones(n), torch.zeros(n, dtype=torch.int32),
                              torch.zeros(n))

    def new_outputs(self, alpha=False):
        return None

    def backward(self, params, out, g, g_depth=None, g_alpha=None):
        self.backwards += 1
        return {k: torch.zeros_like(v) for k, v in params.items()}


def _params():
    p = {k: torch.zeros(4, requires_grad=True) for k in FIELDS}
    return p


def test_backward_after_second_forward_raises():
    r = _StandIn()
    p = _params()
    img1, *_ = raster.render(r, p)
    img2, *_ = raster.render(r, p)          # overwrites the workspace img1 needs
    with pytest.raises(raster.StaleWorkspaceError):
        img1.sum().backward()
    img2.sum().backward()                   # the latest render is fine
    assert r.backwards == 1


def test_alternating_forward_backward_is_accepted():
    r = _StandIn()
    p = _params()
    for _ in range(3):
        img, *_ = raster.render(r, p)
        img.sum().backward()
    assert r.backwards == 3
