"""FP64 analytic gradient and finite differences — TEST INFRASTRUCTURE ONLY.

The render is the composition of the steps in `forward.py`; its derivative
is taken step by step in reverse:

  blend      C = sum_j alpha_j T_j c_j + T_final bg, T_j = prod_{i<j}(1-alpha_i)
             dC/dc_j = alpha_j T_j
             dC/dalpha_j = T_j c_j - S_j / (1 - alpha_j),
             S_j = sum_{k>j} alpha_k T_k c_k + T_final bg
  alpha      alpha = min(alpha_max, sigma e^p); no derivative when clamped
  power      p = -1/2 d^T Q d, d = (px - u, py - v)
  conic      Q = Sigma'^-1  ->  dSigma' = -Q dQ Q (symmetric bookkeeping)
  EWA        Sigma' = M M^T + dil I, M = J W R S        (eq. 3 and the EWA step)
  colour     rgb = max(0, 0.5 + SH(d) + sum_k a_k e^{lambda_k (d.mu_k - 1)})
             (eqs. 4, 5, 9); the view direction d depends on the mean.
  activations  exp, sigmoid, and the normalisations of q and mu.

Discrete decisions (cull, rectangle, alpha_min skip, T_min stop) have zero
derivative; clamps (alpha_max, colour >= 0, the guard band on J, p <= 0) are
differentiated one-sidedly: no derivative where the clamp is active.
Depth carries no gradient.
"""
from __future__ import annotations

import numpy as np

from . import forward as R
from .sh import sh_basis, sh_basis_grad

F64 = np.float64

GRAD2D = ("u", "v", "Qa", "Qb", "Qc", "sigma", "r", "g", "b")


def blend_backward(pre, cam, opts, values, ranges, grad_image, cam_index=0, tile_base=0,
                   tiles=None, grad_depth=None, grad_alpha=None):
    """Per-Gaussian gradients of sum(grad_image * image) (+ sum(grad_depth *
    depth) + sum(grad_alpha * alpha), alpha = 1 - T_final) w.r.t. the 2D
    quantities (u, v, Qa, Qb, Qc, sigma, rgb) and the splat depth z -> dict
    of (N,) arrays.  With `tiles`, only those local tiles' pixels are summed
    (the exact gradient when the upstream gradients are zero elsewhere).

    Depth D = sum_j alpha_j T_j z_j:  dD/dalpha_j = T_j z_j - D_j / (1 -
    alpha_j) with D_j the depth composited behind j, dD/dz_j = alpha_j T_j.
    Alpha A = 1 - prod_j (1 - alpha_j):  dA/dalpha_j = T_final / (1 - alpha_j)."""
    W, H = int(cam.width), int(cam.height)
    amax = R._f(opts.alpha_max)
    bg = cam.bg.astype(F64)
    GX, GY = pre.grid
    n = pre.z.shape[0]
    out = {k: np.zeros(n) for k in GRAD2D + ("z",)}
    gimg = grad_image.astype(F64)
    gdep = np.zeros((H, W)) if grad_depth is None else np.asarray(grad_depth, F64).reshape(H, W)
    galp = np.zeros((H, W)) if grad_alpha is None else np.asarray(grad_alpha, F64).reshape(H, W)
    for t in (range(GX * GY) if tiles is None else tiles):
        tx, ty = t % GX, t // GX
        lo, hi = ranges[tile_base + t]
        if hi <= lo:
            continue
        entries = (values[lo:hi] - cam_index * n).astype(np.int64)
        px, py = R.tile_pixels(tx, ty, opts, W, H)
        C, D, Tf, nn, fl, trace = R._blend_tile(pre, entries, px, py, opts, bg,
                                                want_trace=True)
        gC = gimg[:, py, px]                                  # (3, P)
        gD = gdep[py, px]
        gA = galp[py, px]
        S = Tf[None, :] * bg[:, None]                         # colour behind
        Sd = np.zeros(px.size)                                # depth behind
        for (j, g, blend, a, T) in reversed(trace):
            if not blend.any():
                continue
            w = np.where(blend, a * T, 0.0)
            c = pre.rgb[:, g][:, None]
            # dL/drgb_g
            gr = (gC * w).sum(axis=1)
            out["r"][g] += gr[0]
            out["g"][g] += gr[1]
            out["b"][g] += gr[2]
            out["z"][g] += (gD * w).sum()
            dLda = np.where(blend, (gC * (T * c - S / (1.0 - a))).sum(axis=0)
                            + gD * (T * pre.z[g] - Sd / (1.0 - a))
                            + gA * Tf / (1.0 - a), 0.0)
            S = S + w * c
            Sd = Sd + w * pre.z[g]
            dx = px - pre.u[g]
            dy = py - pre.v[g]
            Qa, Qb, Qc = pre.conic[:, g]
            power = -0.5 * (Qa * dx * dx + 2.0 * Qb * dx * dy + Qc * dy * dy)
            E = np.exp(np.minimum(power, 0.0))
            unclamped = blend & (pre.opacity[g] * E <= amax)
            dLdsig = np.where(unclamped, dLda * E, 0.0)
            dLdp = np.where(unclamped & (power <= 0.0), dLda * a, 0.0)
            out["sigma"][g] += dLdsig.sum()
            out["Qa"][g] += (dLdp * (-0.5 * dx * dx)).sum()
            out["Qb"][g] += (dLdp * (-dx * dy)).sum()
            out["Qc"][g] += (dLdp * (-0.5 * dy * dy)).sum()
            out["u"][g] += (dLdp * (Qa * dx + Qb * dy)).sum()
            out["v"][g] += (dLdp * (Qb * dx + Qc * dy)).sum()
    return out


def _pixel_contributions(pre, opts, px, py, gC, blended, T_final, bg, gD=0.0, gA=0.0):
    """Back-to-front walk of one pixel's blended splats [(g, alpha, T before
    it)] ending at T_final: dict g -> 10-vector ordered as GRAD2D + (z,)."""
    amax = R._f(opts.alpha_max)
    gC = np.asarray(gC, F64)
    S = T_final * bg
    Sd = 0.0
    out = {}
    for (g, a, T) in reversed(blended):
        w = a * T
        c = pre.rgb[:, g]
        grgb = gC * w
        dLda = float((gC * (T * c - S / (1.0 - a))).sum()
                     + gD * (T * pre.z[g] - Sd / (1.0 - a)) + gA * T_final / (1.0 - a))
        S = S + w * c
        Sd = Sd + w * pre.z[g]
        dx = px - pre.u[g]
        dy = py - pre.v[g]
        Qa, Qb, Qc = pre.conic[:, g]
        power = -0.5 * (Qa * dx * dx + 2.0 * Qb * dx * dy + Qc * dy * dy)
        E = np.exp(min(power, 0.0))
        v = np.zeros(10)
        v[9] = gD * w
        if pre.opacity[g] * E <= amax:
            dLdp = dLda * a if power <= 0.0 else 0.0
            v[5] = dLda * E
            v[2] = dLdp * (-0.5 * dx * dx)
            v[3] = dLdp * (-dx * dy)
            v[4] = dLdp * (-0.5 * dy * dy)
            v[0] = dLdp * (Qa * dx + Qb * dy)
            v[1] = dLdp * (Qb * dx + Qc * dy)
        v[6:9] = grgb
        out[int(g)] = out.get(int(g), 0.0) + v
    return out


def pixel_backward(pre, cam, opts, px, py, gC, gD=0.0, gA=0.0):
    """2D-gradient contributions of one pixel (brute-force list, as in
    `forward.render_pixel`) for upstream gradients gC (3,) of its colour and
    gD, gA of its depth and alpha: (dict g -> 10-vector ordered as GRAD2D +
    (z,), tie flag) on the FP64 decision path."""
    bg = cam.bg.astype(F64)
    entries = R.pixel_list(pre, px, py)
    pxa, pya = np.array([px]), np.array([py])
    C, D, Tf, nn, fl, trace = R._blend_tile(pre, entries, pxa, pya, opts, bg, want_trace=True)
    blended = [(g, float(a[0]), float(T[0])) for (j, g, blend, a, T) in trace if blend[0]]
    return (_pixel_contributions(pre, opts, px, py, gC, blended, float(Tf[0]), bg, gD, gA),
            bool(fl[0]))


def _quat_rotation_grad(w, x, y, z, gR):
    """Gradient of the rotation matrix entries w.r.t. (w, x, y, z)."""
    gw = 2.0 * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2]
                - y * gR[2][0] + x * gR[2][1])
    gx = 2.0 * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - 2.0 * x * gR[1][1]
                - w * gR[1][2] + z * gR[2][0] + w * gR[2][1] - 2.0 * x * gR[2][2])
    gy = 2.0 * (-2.0 * y * gR[0][0] + x * gR[0][1] + w * gR[0][2] + x * gR[1][0]
                + z * gR[1][2] - w * gR[2][0] + z * gR[2][1] - 2.0 * y * gR[2][2])
    gz = 2.0 * (-2.0 * z * gR[0][0] - w * gR[0][1] + x * gR[0][2] + w * gR[1][0]
                - 2.0 * z * gR[1][1] + y * gR[1][2] + x * gR[2][0] + y * gR[2][1])
    return gw, gx, gy, gz


def preprocess_backward(scene, cam, opts, pre, g2):
    """Chain rule from the 2D gradients to the raw parameters -> dict in the
    scene's SoA layout (zeros for culled Gaussians)."""
    n = scene.n
    vis = pre.visible
    fx, fy = R._f(cam.fx), R._f(cam.fy)
    Rc = cam.R.astype(F64)
    X = scene.means.astype(F64)
    out = {k: np.zeros(a.shape) for k, a in scene.arrays().items()}

    # opacity
    sig = pre.opacity
    out["opacity_logits"] = g2["sigma"] * sig * (1.0 - sig)

    # colour
    grgb = np.stack([g2["r"], g2["g"], g2["b"]]) * (pre.rgb_raw >= 0.0)
    d = pre.dirs
    nc = (scene.sh_degree + 1) ** 2
    # adaptive SH: coefficients above a Gaussian's degree take no part
    mask = R.sh_mask(scene, R.sh_degrees(scene, pre.radius))
    Y = sh_basis(scene.sh_degree, d) * mask
    dY = sh_basis_grad(scene.sh_degree, d) * mask[:, None, :]
    sh = scene.sh.astype(F64)
    out["sh"][:nc] = grgb[None, :, :] * Y[:, None, :]
    g_dir = np.einsum("cn,lcn,lkn->kn", grgb, sh[:nc], dY)
    mode = getattr(scene, "lobe_mode", R.LOBES_FREE)
    mu_all = R.lobe_axes(scene)
    g_mus = []
    for k in range(scene.n_lobes):
        mu = mu_all[k]
        lam = np.exp(scene.sg_log_sharpness[k].astype(F64))
        cosv = (d * mu).sum(axis=0)
        e = np.where(cosv - 1.0 == 0.0, 1.0, np.exp(lam * (cosv - 1.0)))
        amp = scene.sg_amplitudes[k].astype(F64)
        out["sg_amplitudes"][k] = grgb * e
        s = (grgb * amp).sum(axis=0) * e
        out["sg_log_sharpness"][k] = s * (cosv - 1.0) * lam
        g_mu = s * lam * d                       # w.r.t. the unit axis mu_k
        if mode == R.LOBES_FREE:
            mu_raw = scene.sg_axes[k].astype(F64)
            mlen = np.sqrt((mu_raw * mu_raw).sum(axis=0))
            out["sg_axes"][k] = (g_mu - mu * (mu * g_mu).sum(axis=0)) / mlen
        g_mus.append(g_mu)
        g_dir = g_dir + s * lam * mu
    if mode == R.LOBES_FRAME and scene.n_lobes:
        # mu_k is column k of R(q_hat), q = (1, omega): dL/dR[i][k] = dL/dmu_k[i],
        # then the rotation's quaternion gradient, the normalisation of q,
        # and the three free components of q
        q, qn = R.frame_quaternion(scene.sg_axes[0])
        qh = q / qn
        gRf = [[g_mus[k][i] if k < len(g_mus) else 0.0 * qn for k in range(3)]
               for i in range(3)]
        gqh = np.array(_quat_rotation_grad(*qh, gRf))
        gq = (gqh - qh * (qh * gqh).sum(axis=0)) / qn
        out["sg_axes"][0] = gq[1:4]
    gX = (g_dir - d * (d * g_dir).sum(axis=0)) / pre.dist

    # conic -> Sigma' = [[A, B], [B, C]]
    A, B, C, det = pre.A, pre.B, pre.C, pre.A * pre.C - pre.B * pre.B
    gQa, gQb, gQc = g2["Qa"], g2["Qb"], g2["Qc"]
    d2 = det * det
    gA = (-C * C * gQa + B * C * gQb - B * B * gQc) / d2
    gC = (-B * B * gQa + A * B * gQb - A * A * gQc) / d2
    gB = (2.0 * B * C * gQa - (A * C + B * B) * gQb + 2.0 * A * B * gQc) / d2

    # recompute the forward intermediates
    s_ = np.exp(scene.log_scales.astype(F64))
    q = scene.quats.astype(F64)
    qn = np.sqrt((q * q).sum(axis=0))
    qh = q / qn
    Rq = R.quat_to_rotation(*qh)
    M3 = [[Rq[i][a] * s_[a] for a in range(3)] for i in range(3)]
    xc = pre.xc
    z = xc[2]
    xn, yn = xc[0] * (1.0 / z), xc[1] * (1.0 / z)
    W, H = int(cam.width), int(cam.height)
    guard = R._f(opts.guard)
    limx = guard * ((0.5 * W) / fx)
    limy = guard * ((0.5 * H) / fy)
    xn_c = np.minimum(np.maximum(xn, -limx), limx)
    yn_c = np.minimum(np.maximum(yn, -limy), limy)
    J = [[fx / z, 0.0 * z, -(fx * xn_c) / z], [0.0 * z, fy / z, -(fy * yn_c) / z]]
    T2 = [[sum(J[i][m] * Rc[m, k] for m in range(3)) for k in range(3)] for i in range(2)]
    M = [[sum(T2[i][m] * M3[m][a] for m in range(3)) for a in range(3)] for i in range(2)]

    # Sigma' = M M^T + dil I
    gM = [[2.0 * gA * M[0][a] + gB * M[1][a] for a in range(3)],
          [gB * M[0][a] + 2.0 * gC * M[1][a] for a in range(3)]]
    # M = T2 M3
    gT2 = [[sum(gM[i][a] * M3[k][a] for a in range(3)) for k in range(3)] for i in range(2)]
    gM3 = [[sum(T2[i][k] * gM[i][a] for i in range(2)) for a in range(3)] for k in range(3)]
    # M3 = Rq diag(s)
    gRq = [[gM3[i][a] * s_[a] for a in range(3)] for i in range(3)]
    gs = np.array([sum(gM3[i][a] * Rq[i][a] for i in range(3)) for a in range(3)])
    out["log_scales"] = gs * s_
    gqh = np.array(_quat_rotation_grad(*qh, gRq))
    out["quats"] = (gqh - qh * (qh * gqh).sum(axis=0)) / qn

    # T2 = J Rc
    gJ = [[sum(gT2[i][k] * Rc[m, k] for k in range(3)) for m in range(3)] for i in range(2)]
    # J entries and (u, v) as functions of the camera-space mean
    gxc = np.zeros((3, n))
    z2 = z * z
    gxc[2] += gJ[0][0] * (-fx / z2) + gJ[1][1] * (-fy / z2)
    fxc = pre.xclamp
    fyc = pre.yclamp
    gxc[0] += np.where(fxc, 0.0, gJ[0][2] * (-fx / z2))
    gxc[2] += np.where(fxc, gJ[0][2] * (fx * xn_c / z2), gJ[0][2] * (2.0 * fx * xc[0] / (z2 * z)))
    gxc[1] += np.where(fyc, 0.0, gJ[1][2] * (-fy / z2))
    gxc[2] += np.where(fyc, gJ[1][2] * (fy * yn_c / z2), gJ[1][2] * (2.0 * fy * xc[1] / (z2 * z)))
    gu, gv = g2["u"], g2["v"]
    if "z" in g2:                       # the splat depth is the camera-space z
        gxc[2] += g2["z"]
    gxc[0] += gu * fx / z
    gxc[1] += gv * fy / z
    gxc[2] += -gu * fx * xc[0] / z2 - gv * fy * xc[1] / z2
    gX = gX + Rc.T @ gxc
    out["means"] = gX

    for k in out:
        out[k] = np.where(vis, out[k], 0.0)
    return out


def l1_loss(image, target):
    """L = mean over 3HW of |image - target|; dL/dimage = sign(.)/(3HW),
    sign(0) = 0."""
    diff = image.astype(F64) - target.astype(F64)
    m = diff.size
    return np.abs(diff).sum() / m, np.sign(diff) / m


def render_and_grad(scene, cam, opts, target=None, grad_image=None, grad_depth=None,
                    grad_alpha=None):
    """Forward render, L1 loss against `target` (or the given grad image,
    and optional depth / alpha upstream gradients), and the analytic
    gradient of the raw parameters."""
    img = R.render(scene, cam, opts)
    pre = R.preprocess(scene, cam, opts)
    if grad_image is None:
        loss, grad_image = l1_loss(img.image, target)
    else:
        loss = None
    g2 = blend_backward(pre, cam, opts, img.values, img.ranges, grad_image,
                        grad_depth=grad_depth, grad_alpha=grad_alpha)
    grads = preprocess_backward(scene, cam, opts, pre, g2)
    return img, loss, g2, grads


# ----------------------------------------------------------------------------
# Finite differences
# ----------------------------------------------------------------------------

def signature(scene, cam, opts, target):
    """Every discrete decision of the render: culled set, rectangles, the
    per-pixel blended lists with their stops, clamp masks and L1 signs."""
    pre = R.preprocess(scene, cam, opts)
    img = R.render(scene, cam, opts)
    W, H = int(cam.width), int(cam.height)
    amax = R._f(opts.alpha_max)
    parts = [pre.visible.tobytes(), pre.rect.tobytes(), pre.radius.tobytes(),
             pre.xclamp.tobytes(),
             pre.yclamp.tobytes(), (pre.rgb_raw >= 0).tobytes(),
             img.n_contrib.tobytes(), img.values.tobytes(), img.ranges.tobytes(),
             np.sign(img.image - target).tobytes()]
    GX, GY = pre.grid
    for t in range(GX * GY):
        lo, hi = img.ranges[t]
        if hi <= lo:
            continue
        entries = img.values[lo:hi].astype(np.int64)
        px, py = R.tile_pixels(t % GX, t // GX, opts, W, H)
        *_, trace = R._blend_tile(pre, entries, px, py, opts, cam.bg.astype(F64), True)
        for (j, g, blend, a, T) in trace:
            parts.append(blend.tobytes())
            parts.append((a >= amax).tobytes())
    return b"".join(parts)


def loss_fn(scene, cam, opts, target):
    img = R.render(scene, cam, opts)
    return l1_loss(img.image, target)[0]


def fd_grad(scene, cam, opts, target, field, index, rel_step=1e-6):
    """Central difference of the L1 loss w.r.t. one raw parameter
    scene.<field>[index].  Returns (value, valid): valid is False when a
    discrete decision changes between the two evaluations."""
    arr = getattr(scene, field)
    base = float(arr[index])
    h = rel_step * max(1.0, abs(base))
    sig0 = signature(scene, cam, opts, target)
    vals = []
    valid = True
    for sgn in (+1.0, -1.0):
        sc = scene.copy()
        a = getattr(sc, field).astype(np.float64)
        a[index] = base + sgn * h
        # the parameters stay float64 here: the oracle reads them with astype
        setattr(sc, field, a)
        vals.append(loss_fn(sc, cam, opts, target))
        if signature(sc, cam, opts, target) != sig0:
            valid = False
    return (vals[0] - vals[1]) / (2.0 * h), valid


def linear_loss(scene, cam, opts, grad_image, grad_depth=None, grad_alpha=None):
    """sum(grad_image * image) + sum(grad_depth * depth) + sum(grad_alpha *
    (1 - T_final)): the loss whose gradient blend_backward takes for these
    upstream gradients."""
    img = R.render(scene, cam, opts)
    L = float((np.asarray(grad_image, F64) * img.image).sum())
    if grad_depth is not None:
        L += float((np.asarray(grad_depth, F64) * img.depth).sum())
    if grad_alpha is not None:
        L += float((np.asarray(grad_alpha, F64) * (1.0 - img.final_T)).sum())
    return L


def fd_grad_linear(scene, cam, opts, grad_image, grad_depth, grad_alpha, field, index,
                   rel_step=1e-6):
    """Central difference of linear_loss w.r.t. scene.<field>[index];
    (value, valid) with valid False when a discrete decision changes."""
    arr = getattr(scene, field)
    base = float(arr[index])
    h = rel_step * max(1.0, abs(base))
    zero = np.zeros((3, int(cam.height), int(cam.width)))
    sig0 = signature(scene, cam, opts, zero)
    vals = []
    valid = True
    for sgn in (+1.0, -1.0):
        sc = scene.copy()
        a = getattr(sc, field).astype(np.float64)
        a[index] = base + sgn * h
        setattr(sc, field, a)
        vals.append(linear_loss(sc, cam, opts, grad_image, grad_depth, grad_alpha))
        if signature(sc, cam, opts, zero) != sig0:
            valid = False
    return (vals[0] - vals[1]) / (2.0 * h), valid
