"""FP64 Adam with the staged SG introduction — TEST INFRASTRUCTURE ONLY.

The optimiser of the training the rasteriser serves (paper: Experiments,
Implementation): every parameter array is trained with Adam (Kingma and
Ba) at the 3D-GS learning rates, except that the SG lobe arrays join only
after the first iterations (2,000 in the paper) with learning rate 0.0025.

Per array with step count t (Adam, Kingma and Ba, Algorithm 1):
    m <- b1 m + (1 - b1) g
    v <- b2 v + (1 - b2) g^2
    m_hat = m / (1 - b1^t),  v_hat = v / (1 - b2^t)
    p <- p - lr m_hat / (sqrt(v_hat) + eps)

Reading (the paper does not say how the lobes' optimiser state starts):
the lobe arrays and their moments are untouched while the iteration is
below sg_start, and their own t counts from 1 at sg_start — as when the
arrays are handed to a fresh Adam at that iteration.
"""
from __future__ import annotations

import numpy as np

FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh",
          "sg_axes", "sg_log_sharpness", "sg_amplitudes")
LOBE_FIELDS = ("sg_axes", "sg_log_sharpness", "sg_amplitudes")


def adam_update(p, g, m, v, lr, t, b1=0.9, b2=0.999, eps=1e-15):
    """One Adam step on one array; returns new (p, m, v) in float64."""
    p, g, m, v = (np.asarray(x, np.float64) for x in (p, g, m, v))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def adam_step(params: dict, grads: dict, m: dict, v: dict, lr: dict, step: int,
              sg_start: int = 0, b1=0.9, b2=0.999, eps=1e-15):
    """Adam over every parameter array (dicts keyed by FIELDS); the lobe
    arrays wait for sg_start.  Returns new (params, m, v) dicts."""
    P, M, V = dict(params), dict(m), dict(v)
    s0 = max(1, int(sg_start))
    for k in FIELDS:
        t = step - s0 + 1 if k in LOBE_FIELDS else step
        if t < 1 or lr.get(k, 0.0) == 0.0 or np.asarray(params[k]).size == 0:
            continue
        P[k], M[k], V[k] = adam_update(params[k], grads[k], m[k], v[k], lr[k], t, b1, b2, eps)
    return P, M, V
