"""Pins of the oracle's Adam with the staged SG start — no GPU.

Against torch.optim.Adam on the CPU (a library implementation of the same
algorithm), the closed form of Adam's first step, and the staged start:
untouched lobe arrays before sg_start, then a fresh Adam's first step.
"""
import numpy as np
import pytest
import torch

from oracle import optim as O

LR = {"means": 1.6e-4, "log_scales": 5e-3, "quats": 1e-3, "opacity_logits": 5e-2,
      "sh": 2.5e-3, "sg_axes": 2.5e-3, "sg_log_sharpness": 2.5e-3, "sg_amplitudes": 2.5e-3}
SHAPES = {"means": (3, 50), "log_scales": (3, 50), "quats": (4, 50), "opacity_logits": (50,),
          "sh": (4, 3, 50), "sg_axes": (4, 3, 50), "sg_log_sharpness": (4, 50),
          "sg_amplitudes": (4, 3, 50)}


def _arrays(seed):
    rng = np.random.default_rng(seed)
    return {k: rng.normal(size=s) for k, s in SHAPES.items()}


def test_matches_torch_adam_over_several_steps():
    p0 = _arrays(0)
    P = dict(p0)
    M = {k: np.zeros_like(a) for k, a in p0.items()}
    V = {k: np.zeros_like(a) for k, a in p0.items()}
    tp = {k: torch.tensor(a, dtype=torch.float64, requires_grad=True) for k, a in p0.items()}
    opt = torch.optim.Adam([{"params": [tp[k]], "lr": LR[k]} for k in O.FIELDS],
                           betas=(0.9, 0.999), eps=1e-15)
    for step in range(1, 6):
        G = _arrays(100 + step)
        P, M, V = O.adam_step(P, G, M, V, LR, step)
        for k in O.FIELDS:
            tp[k].grad = torch.tensor(G[k], dtype=torch.float64)
        opt.step()
        for k in O.FIELDS:
            assert np.allclose(P[k], tp[k].detach().numpy(), rtol=1e-13, atol=1e-15), (step, k)


def test_first_step_closed_form():
    """t = 1: m_hat = g and v_hat = g^2, so p moves by lr g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    p, g = rng.normal(size=100), rng.normal(size=100)
    z = np.zeros(100)
    new, m, v = O.adam_update(p, g, z, z, 0.01, 1, eps=1e-8)
    assert np.allclose(new, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=1e-16)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


@pytest.mark.parametrize("sg_start", [3, 2000])
def test_staged_start_of_the_lobes(sg_start):
    P = _arrays(2)
    M = {k: np.zeros_like(a) for k, a in P.items()}
    V = {k: np.zeros_like(a) for k, a in P.items()}
    steps = [1, 2, sg_start - 1, sg_start, sg_start + 1]
    for step in steps:
        G = _arrays(200 + step)
        P1, M1, V1 = O.adam_step(P, G, M, V, LR, step, sg_start=sg_start)
        for k in O.LOBE_FIELDS:
            if step < sg_start:
                assert np.array_equal(P1[k], P[k]) and np.array_equal(M1[k], M[k])
            elif step == sg_start:
                # a fresh Adam's first step
                want = P[k] - LR[k] * G[k] / (np.abs(G[k]) + 1e-15)
                assert np.allclose(P1[k], want, rtol=1e-12)
        for k in ("means", "sh"):
            assert not np.array_equal(P1[k], P[k])
        P, M, V = P1, M1, V1
