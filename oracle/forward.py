"""FP64 CPU oracle of the SG-Splatting rasteriser — TEST INFRASTRUCTURE ONLY.

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
use this module; the product path never imports it.  It shares no code with
the HIP path: plain NumPy in float64, slow and direct.

What it computes (paper, Methods):
  * Gaussian density exp(-1/2 (x-X)^T Sigma^-1 (x-X))            (eq. 2)
  * Sigma = R S S^T R^T from a quaternion and a scale vector      (eq. 3)
  * EWA projection to a 2D splat (Preliminaries, citing Zwicker et al.)
  * colour = low-degree SH (eq. 4) + K spherical-Gaussian lobes
    a_k exp(lambda_k (d . mu_k - 1))                          (eqs. 5-7, 9)
  * front-to-back alpha blending of the depth-sorted splats (Overview,
    Preliminaries).

Readings where the paper is silent (all are self-consistency only — "parity
unpinned" against the paper itself, since it prints no worked example):
  R1 quaternion (w,x,y,z);  R2 raw parameters with exp/sigmoid activations,
  q and mu normalised;  R3 view direction = camera centre -> Gaussian mean,
  one per Gaussian;  R4 rgb = max(0, 0.5 + SH + sum SG);  R5 diffuse = SH
  degree 0;  R6 real SH with Condon-Shortley phase;  R7 free lobe axes;
  R9 guard 1.3 on J, dilation 0.3 on both diagonal entries;  R10 cull
  z <= znear;  R11 radius ceil(3 sqrt(lambda_1));  R12 footprint = integer
  pixel rectangle;  R13 pixel centres at integer coordinates;  R14 key =
  (tile << 32) | bits(float32 z), ties by Gaussian index;  R15 power
  clamped to <= 0;  R16 alpha_max 0.99, alpha_min 1/255 (skip), T_min 1e-4
  (exclusive stop);  R17 depth = sum alpha T z, n_contrib = 1 + position of
  the last blended entry in the tile list;  R18 background T*bg;  R19 empty
  tile -> range (0,0);  R21 a non-finite raw parameter or a lobe axis of
  zero length -> culled.

Key path.  Every value that decides an integer (cull flag, radius, pixel and
tile rectangle, depth key) is computed with one prescribed sequence of IEEE
float64 operations — no fused multiply-add, sums left to right as written —
so that any implementation following the same sequence obtains the same
integers.  The only non-correctly-rounded step on it is exp() of the
log-scales.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .sh import sh_basis

F64 = np.float64


# ----------------------------------------------------------------------------
# Preprocess
# ----------------------------------------------------------------------------

@dataclass
class Pre:
    """Per-Gaussian preprocess results (index = Gaussian)."""
    visible: np.ndarray        # bool
    xc: np.ndarray             # (3,N) camera-space mean
    z: np.ndarray              # camera depth (float64)
    depth_bits: np.ndarray     # uint32 bits of float32(z)
    A: np.ndarray              # 2D covariance [[A, B], [B, C]]
    B: np.ndarray
    C: np.ndarray
    det: np.ndarray
    lam1: np.ndarray
    radius: np.ndarray         # int64
    u: np.ndarray              # projected mean, pixels
    v: np.ndarray
    rect: np.ndarray           # (4,N) int64 px0, px1, py0, py1 (inclusive)
    tile_rect: np.ndarray      # (4,N) int64 tx0, tx1, ty0, ty1 (inclusive)
    tiles_touched: np.ndarray  # int64, 0 for culled
    conic: np.ndarray          # (3,N) Qa, Qb, Qc with Q = Sigma'^-1
    opacity: np.ndarray        # sigma = sigmoid(logit)
    rgb: np.ndarray            # (3,N) clamped colour
    rgb_raw: np.ndarray        # (3,N) before the clamp
    dirs: np.ndarray           # (3,N) unit view direction
    dist: np.ndarray           # |X - camera centre|
    xclamp: np.ndarray         # bool: guard clamp active on x
    yclamp: np.ndarray
    grid: tuple                # (GX, GY) tiles


def _f(x) -> float:
    """Every scalar crossing the C-ABI is float32; take its exact value."""
    return float(np.float32(x))


def _finite_params(scene) -> np.ndarray:
    ok = np.ones(scene.n, bool)
    for a in scene.arrays().values():
        if a.size:
            ok &= np.isfinite(a.reshape(-1, scene.n)).all(axis=0)
    return ok


def quat_to_rotation(w, x, y, z):
    """Rotation matrix of a unit quaternion (w, x, y, z) (eq. 3's R)."""
    return [[1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)],
            [2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)],
            [2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)]]


def camera_centre(cam) -> np.ndarray:
    R = cam.R.astype(F64)
    t = cam.t.astype(F64)
    return np.array([-((R[0, j] * t[0] + R[1, j] * t[1]) + R[2, j] * t[2]) for j in range(3)])


LOBES_FREE, LOBES_WORLD, LOBES_FRAME = 0, 1, 2


def frame_quaternion(omega):
    """Unit quaternion of the orthonormal lobe frame from its 3 parameters
    omega (3,N): q = (1, omega) / |(1, omega)|, i.e. the rotation whose
    Gibbs (Cayley) vector is omega.  Every rotation but the half-turns is
    reached, and the map is smooth everywhere (|q| >= 1)."""
    w = np.asarray(omega, F64)
    q = np.stack([np.ones(w.shape[1]), w[0], w[1], w[2]])
    return q, np.sqrt((q * q).sum(axis=0))


def lobe_axes(scene):
    """Unit lobe axes mu_k, (K, 3, N), by the scene's lobe mode.

    free : each lobe's own axis, normalised (eq. 5's mu).
    world: the paper's fixed orthogonal axes (1,0,0), (0,1,0), (0,0,1)
           (Experiments, Implementation; eqs. 7-8).
    frame: the columns of a rotation R(q) with q from 3 parameters per
           Gaussian (Methods, Multi-Axis Orthogonal Gaussians: three
           orthogonal lobes need 3 extra parameters for their directions;
           eq. 8 holds by construction)."""
    n, K = scene.n, scene.n_lobes
    mode = getattr(scene, "lobe_mode", LOBES_FREE)
    if mode == LOBES_FREE:
        mu = scene.sg_axes.astype(F64)
        return mu / np.sqrt((mu * mu).sum(axis=1, keepdims=True))
    if mode == LOBES_WORLD:
        return np.broadcast_to(np.eye(3)[:K, :, None], (K, 3, n)).astype(F64)
    q, qn = frame_quaternion(scene.sg_axes[0])
    Rq = quat_to_rotation(*(q / qn))
    return np.array([[Rq[i][k] for i in range(3)] for k in range(K)])


def sh_degrees(scene, radius):
    """SH degree used by each Gaussian (N,): sh_degree, or with adaptive
    thresholds (t0, t1) on the projected radius r: 0 where r <= t0, at most
    1 where r <= t1, sh_degree above (Methods, Mixing Spherical Harmonics
    and Spherical Gaussians: degree 0-2 chosen by the size of the 2D
    projection, large Gaussians degree 2)."""
    L = scene.sh_degree
    t0, t1 = tuple(getattr(scene, "sh_adaptive", (0, 0)))
    deg = np.full(scene.n, L, np.int64)
    if t0 > 0 and radius is not None:
        r = np.asarray(radius)
        deg = np.where(r <= t1, np.minimum(1, L), deg)
        deg = np.where(r <= t0, 0, deg)
    return deg


def sh_mask(scene, deg):
    """(NC, N) 1 where coefficient l is used (l < (deg + 1)^2), else 0."""
    nc = (scene.sh_degree + 1) ** 2
    return (np.arange(nc)[:, None] < (deg[None, :] + 1) ** 2).astype(F64)


def colour(scene, dirs, radius=None):
    """rgb_raw = 0.5 + SH(d) + sum_k a_k exp(lambda_k (d.mu_k - 1))  (eq. 9, R4);
    with adaptive SH, coefficients above a Gaussian's degree are unused."""
    Y = sh_basis(scene.sh_degree, dirs) * sh_mask(scene, sh_degrees(scene, radius))
    nc = Y.shape[0]
    sh = scene.sh.astype(F64)
    raw = 0.5 + np.einsum("lcn,ln->cn", sh[:nc], Y)
    mu_all = lobe_axes(scene)
    for k in range(scene.n_lobes):
        mu = mu_all[k]
        lam = np.exp(scene.sg_log_sharpness[k].astype(F64))
        t = (dirs * mu).sum(axis=0) - 1.0
        # eq. 5; along the axis (t = 0) the lobe is 1 for any sharpness
        e = np.where(t == 0.0, 1.0, np.exp(lam * t))
        raw = raw + scene.sg_amplitudes[k].astype(F64) * e
    return raw


def zero_axis(scene) -> np.ndarray:
    """Gaussians with a free lobe axis of zero length (no direction to
    normalise; the orthogonal modes have none)."""
    bad = np.zeros(scene.n, bool)
    if getattr(scene, "lobe_mode", LOBES_FREE) != LOBES_FREE:
        return bad
    for k in range(scene.n_lobes):
        a = scene.sg_axes[k].astype(F64)
        bad |= (a * a).sum(axis=0) == 0.0
    return bad


def preprocess(scene, cam, opts) -> Pre:
    n = scene.n
    W, H = int(cam.width), int(cam.height)
    fx, fy, cx, cy = _f(cam.fx), _f(cam.fy), _f(cam.cx), _f(cam.cy)
    znear = _f(cam.znear)
    dil, guard = _f(opts.dilation), _f(opts.guard)
    Rc = cam.R.astype(F64)
    tc = cam.t.astype(F64)
    X = scene.means.astype(F64)

    # camera-space mean: ((R_i0 X0 + R_i1 X1) + R_i2 X2) + t_i
    xc = np.array([((Rc[i, 0] * X[0] + Rc[i, 1] * X[1]) + Rc[i, 2] * X[2]) + tc[i]
                   for i in range(3)])
    z = xc[2]

    with np.errstate(all="ignore"):
        # activations (R2)
        s = np.exp(scene.log_scales.astype(F64))
        q = scene.quats.astype(F64)
        qn = np.sqrt(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3])
        iq = 1.0 / qn
        qw, qx, qy, qz = q[0] * iq, q[1] * iq, q[2] * iq, q[3] * iq
        Rq = quat_to_rotation(qw, qx, qy, qz)
        M3 = [[Rq[i][a] * s[a] for a in range(3)] for i in range(3)]   # R S (eq. 3)

        # EWA local affine approximation with the guard band (R9)
        iz = 1.0 / z
        xn = xc[0] * iz
        yn = xc[1] * iz
        limx = guard * ((0.5 * W) / fx)
        limy = guard * ((0.5 * H) / fy)
        xn_c = np.minimum(np.maximum(xn, -limx), limx)
        yn_c = np.minimum(np.maximum(yn, -limy), limy)
        J00 = fx * iz
        J02 = -(fx * xn_c) * iz
        J11 = fy * iz
        J12 = -(fy * yn_c) * iz
        T2 = [[J00 * Rc[0, k] + J02 * Rc[2, k] for k in range(3)],
              [J11 * Rc[1, k] + J12 * Rc[2, k] for k in range(3)]]
        M = [[(T2[i][0] * M3[0][a] + T2[i][1] * M3[1][a]) + T2[i][2] * M3[2][a]
              for a in range(3)] for i in range(2)]
        # Sigma' = M M^T + dil I  (M M^T = J W R S S^T R^T W^T J^T)
        pp = (M[0][0] * M[0][0] + M[0][1] * M[0][1]) + M[0][2] * M[0][2]
        qq = (M[1][0] * M[1][0] + M[1][1] * M[1][1]) + M[1][2] * M[1][2]
        bb = (M[0][0] * M[1][0] + M[0][1] * M[1][1]) + M[0][2] * M[1][2]
        A = pp + dil
        C = qq + dil
        B = bb
        # det = AC - B^2 without cancellation (Lagrange identity on M's rows)
        crx = M[0][1] * M[1][2] - M[0][2] * M[1][1]
        cry = M[0][2] * M[1][0] - M[0][0] * M[1][2]
        crz = M[0][0] * M[1][1] - M[0][1] * M[1][0]
        det = (((crx * crx + cry * cry) + crz * crz) + dil * (pp + qq)) + dil * dil
        h = (A - C) * 0.5
        lam1 = (A + C) * 0.5 + np.sqrt(h * h + B * B)
        radius = np.ceil(3.0 * np.sqrt(lam1))                    # R11
        u = fx * xn + cx
        v = fy * yn + cy
        lox = np.ceil(u - radius)
        hix = np.floor(u + radius)
        loy = np.ceil(v - radius)
        hiy = np.floor(v + radius)

        # colour (image path)
        cc = camera_centre(cam)
        dvec = X - cc[:, None]
        dist = np.sqrt((dvec * dvec).sum(axis=0))
        dirs = dvec / dist
        rgb_raw = colour(scene, dirs, radius)
        opacity = 1.0 / (1.0 + np.exp(-scene.opacity_logits.astype(F64)))

    finite = (_finite_params(scene) & ~zero_axis(scene) & np.isfinite(A) & np.isfinite(B)
              & np.isfinite(C) & np.isfinite(det) & np.isfinite(lam1) & np.isfinite(u)
              & np.isfinite(v))
    visible = (finite & (z > znear) & (lox <= W - 1) & (hix >= 0)
               & (loy <= H - 1) & (hiy >= 0))

    rect = np.zeros((4, n), np.int64)
    vi = visible
    rect[0, vi] = np.maximum(lox[vi], 0).astype(np.int64)
    rect[1, vi] = np.minimum(hix[vi], W - 1).astype(np.int64)
    rect[2, vi] = np.maximum(loy[vi], 0).astype(np.int64)
    rect[3, vi] = np.minimum(hiy[vi], H - 1).astype(np.int64)
    tw, th = int(opts.tile_w), int(opts.tile_h)
    GX = (W + tw - 1) // tw
    GY = (H + th - 1) // th
    trect = np.zeros((4, n), np.int64)
    trect[0] = rect[0] // tw
    trect[1] = rect[1] // tw
    trect[2] = rect[2] // th
    trect[3] = rect[3] // th
    touched = np.where(visible, (trect[1] - trect[0] + 1) * (trect[3] - trect[2] + 1), 0)

    with np.errstate(all="ignore"):
        conic = np.array([C / det, -B / det, A / det])
        depth_bits = z.astype(np.float32).view(np.uint32)
    rgb = np.maximum(rgb_raw, 0.0)
    return Pre(visible, xc, z, depth_bits, A, B, C, det, lam1,
               np.where(visible, radius, 0).astype(np.int64), u, v, rect, trect,
               touched.astype(np.int64), conic, opacity, rgb, rgb_raw, dirs, dist,
               (xn < -limx) | (xn > limx), (yn < -limy) | (yn > limy), (GX, GY))


# ----------------------------------------------------------------------------
# Keys, sort, ranges
# ----------------------------------------------------------------------------

def emit_pairs(pres, tile_bases=None, n_per_cam=None):
    """Duplicate each visible Gaussian once per touched tile.

    Pairs are emitted camera by camera, Gaussian index ascending, tiles of a
    rectangle row-major.  key = (global tile << 32) | depth bits (R14);
    value = camera * N + g.
    """
    if not isinstance(pres, (list, tuple)):
        pres = [pres]
    keys, vals = [], []
    base = 0
    for c, pre in enumerate(pres):
        n = pre.z.shape[0]
        GX, GY = pre.grid
        cnt = pre.tiles_touched
        g = np.repeat(np.arange(n, dtype=np.int64), cnt)
        start = np.repeat(np.cumsum(cnt) - cnt, cnt)
        j = np.arange(g.size, dtype=np.int64) - start
        wdt = pre.tile_rect[1, g] - pre.tile_rect[0, g] + 1
        tx = pre.tile_rect[0, g] + j % wdt
        ty = pre.tile_rect[2, g] + j // wdt
        tile = base + ty * GX + tx
        keys.append((tile.astype(np.uint64) << np.uint64(32))
                    | pre.depth_bits[g].astype(np.uint64))
        vals.append((c * n + g).astype(np.uint64))
        base += GX * GY
    return np.concatenate(keys), np.concatenate(vals), base


def sort_pairs(keys, vals):
    """Stable ascending sort by key; ties keep emission (Gaussian) order."""
    order = np.argsort(keys, kind="stable")
    return keys[order], vals[order]


def tile_ranges(sorted_keys, n_tiles):
    """[start, end) of each tile's entries; empty tiles get (0, 0) (R19)."""
    tiles = (sorted_keys >> np.uint64(32)).astype(np.int64)
    t = np.arange(n_tiles)
    lo = np.searchsorted(tiles, t, side="left")
    hi = np.searchsorted(tiles, t, side="right")
    empty = lo == hi
    lo[empty] = 0
    hi[empty] = 0
    return np.stack([lo, hi], axis=1).astype(np.int64)


# ----------------------------------------------------------------------------
# Blend
# ----------------------------------------------------------------------------

@dataclass
class Image:
    image: np.ndarray        # (3,H,W)
    depth: np.ndarray        # (H,W)
    final_T: np.ndarray      # (H,W)
    n_contrib: np.ndarray    # (H,W) int64
    flagged: np.ndarray      # (H,W) bool: a decision fell inside a tie band
    alternatives: dict       # (py,px) -> list of (rgb(3), depth, T, n) outcomes
    keys: np.ndarray
    values: np.ndarray
    ranges: np.ndarray


ALPHA_BAND = 1e-4   # relative half-width of the alpha >= alpha_min tie band
T_BAND = 1e-3       # relative half-width of the T' < T_min tie band
MAX_OUTCOMES = 64


def _alpha(pre, g, dx, dy, amax):
    Qa, Qb, Qc = pre.conic[0, g], pre.conic[1, g], pre.conic[2, g]
    power = -0.5 * (Qa * dx * dx + 2.0 * Qb * dx * dy + Qc * dy * dy)
    p = np.minimum(power, 0.0)                                   # R15
    return np.minimum(amax, pre.opacity[g] * np.exp(p))


def _blend_tile(pre, entries, px, py, opts, bg, want_trace=False):
    """Blend the pixels (px, py) over the list `entries` (Gaussian ids).

    Returns C (3,P), D, T, n, flagged and, if asked, per-entry traces.
    """
    amin, amax, tmin = _f(opts.alpha_min), _f(opts.alpha_max), _f(opts.t_min)
    npx = px.size
    C = np.zeros((3, npx))
    D = np.zeros(npx)
    T = np.ones(npx)
    n = np.zeros(npx, np.int64)
    done = np.zeros(npx, bool)
    flagged = np.zeros(npx, bool)
    trace = []
    for j, g in enumerate(entries):
        if done.all():
            break
        inr = ((px >= pre.rect[0, g]) & (px <= pre.rect[1, g])
               & (py >= pre.rect[2, g]) & (py <= pre.rect[3, g]))
        evald = ~done & inr
        if not evald.any():
            continue
        dx = px - pre.u[g]
        dy = py - pre.v[g]
        a = _alpha(pre, g, dx, dy, amax)
        flagged |= evald & (np.abs(a - amin) <= ALPHA_BAND * amin)
        take = evald & (a >= amin)
        Tn = T * (1.0 - a)
        flagged |= take & (np.abs(Tn - tmin) <= T_BAND * tmin)
        stop = take & (Tn < tmin)
        done |= stop
        blend = take & ~stop
        w = np.where(blend, a * T, 0.0)
        C += w * pre.rgb[:, g][:, None]
        D += w * pre.z[g]
        if want_trace:
            trace.append((j, g, blend, a, T.copy()))
        T = np.where(blend, Tn, T)
        n = np.where(blend, j + 1, n)
    return C, D, T, n, flagged, trace


def pixel_outcomes(pre, entries, px, py, opts, bg):
    """Every result a correct FP32 renderer may give at one pixel.

    Walks the list like the blend.  At each decision whose FP64 value falls
    inside its tie band (alpha within ALPHA_BAND of alpha_min, or T' within
    T_BAND of T_min) both branches are followed.  Returns a list of
    (rgb(3), depth, T, n) — the FP64 decision path last — or None when the
    branches exceed MAX_OUTCOMES.
    """
    amin, amax, tmin = _f(opts.alpha_min), _f(opts.alpha_max), _f(opts.t_min)
    out = []

    class _TooMany(Exception):
        pass

    def actions(a, T):
        near_a = abs(a - amin) <= ALPHA_BAND * amin
        acts = []
        if a >= amin or near_a:
            Tn = T * (1.0 - a)
            near_t = abs(Tn - tmin) <= T_BAND * tmin
            first = "stop" if Tn < tmin else "blend"
            acts.append(first)
            if near_t:
                acts.append("blend" if first == "stop" else "stop")
        if a < amin:
            acts.insert(0, "skip")
        elif near_a:
            acts.append("skip")
        return acts

    def walk(j0, T, C, D, n):
        for j in range(j0, len(entries)):
            g = entries[j]
            if not (pre.rect[0, g] <= px <= pre.rect[1, g]
                    and pre.rect[2, g] <= py <= pre.rect[3, g]):
                continue
            a = float(_alpha(pre, g, px - pre.u[g], py - pre.v[g], amax))
            acts = actions(a, T)
            for alt in acts[1:]:
                if alt == "stop":
                    out.append((C + T * bg, D, T, n))
                elif alt == "blend":
                    walk(j + 1, T * (1.0 - a), C + a * T * pre.rgb[:, g],
                         D + a * T * pre.z[g], j + 1)
                else:
                    walk(j + 1, T, C, D, n)
                if len(out) > MAX_OUTCOMES:
                    raise _TooMany
            if acts[0] == "stop":
                out.append((C + T * bg, D, T, n))
                return
            if acts[0] == "blend":
                C = C + a * T * pre.rgb[:, g]
                D = D + a * T * pre.z[g]
                T = T * (1.0 - a)
                n = j + 1
        out.append((C + T * bg, D, T, n))

    try:
        walk(0, 1.0, np.zeros(3), 0.0, 0)
    except _TooMany:
        return None
    return out


def tile_pixels(tx, ty, opts, W, H):
    tw, th = int(opts.tile_w), int(opts.tile_h)
    xs = np.arange(tx * tw, min((tx + 1) * tw, W))
    ys = np.arange(ty * th, min((ty + 1) * th, H))
    py, px = np.meshgrid(ys, xs, indexing="ij")
    return px.ravel(), py.ravel()


def blend_image(pre, cam, opts, values, ranges, n_per_cam=None, cam_index=0,
                tile_base=0, tiles=None):
    """Front-to-back compositing of every pixel of one camera (or of the
    tiles listed in `tiles`)."""
    W, H = int(cam.width), int(cam.height)
    bg = cam.bg.astype(F64)
    GX, GY = pre.grid
    n = pre.z.shape[0]
    image = np.zeros((3, H, W))
    depth = np.zeros((H, W))
    final_T = np.ones((H, W))
    ncon = np.zeros((H, W), np.int64)
    flagged = np.zeros((H, W), bool)
    alts = {}
    todo = range(GX * GY) if tiles is None else tiles
    for t in todo:
        tx, ty = t % GX, t // GX
        lo, hi = ranges[tile_base + t]
        entries = (values[lo:hi] - cam_index * n).astype(np.int64)
        px, py = tile_pixels(tx, ty, opts, W, H)
        C, D, T, nn, fl, _ = _blend_tile(pre, entries, px, py, opts, bg)
        image[:, py, px] = C + T * bg[:, None]
        depth[py, px] = D
        final_T[py, px] = T
        ncon[py, px] = nn
        flagged[py, px] = fl
        for k in np.nonzero(fl)[0]:
            alts[(int(py[k]), int(px[k]))] = pixel_outcomes(
                pre, entries, int(px[k]), int(py[k]), opts, bg)
    return image, depth, final_T, ncon, flagged, alts


def render(scene, cam, opts) -> Image:
    """Full forward render of one camera (steps: preprocess, keys, stable
    sort, ranges, blend)."""
    pre = preprocess(scene, cam, opts)
    keys, vals, ntiles = emit_pairs(pre)
    keys, vals = sort_pairs(keys, vals)
    ranges = tile_ranges(keys, ntiles)
    img, dep, T, n, fl, alts = blend_image(pre, cam, opts, vals, ranges)
    return Image(img, dep, T, n, fl, alts, keys, vals, ranges)


def render_batch(scene, cams, opts):
    """Several cameras in one key space: global tile = camera tile base +
    local tile, value = camera * N + g."""
    pres = [preprocess(scene, c, opts) for c in cams]
    keys, vals, ntiles = emit_pairs(pres)
    keys, vals = sort_pairs(keys, vals)
    ranges = tile_ranges(keys, ntiles)
    out = []
    base = 0
    for ci, (pre, cam) in enumerate(zip(pres, cams)):
        GX, GY = pre.grid
        img, dep, T, n, fl, alts = blend_image(pre, cam, opts, vals, ranges,
                                               cam_index=ci, tile_base=base)
        out.append(Image(img, dep, T, n, fl, alts, None, None, None))
        base += GX * GY
    return pres, out, keys, vals, ranges


# ----------------------------------------------------------------------------
# Brute-force per-pixel render (no tiles): for sampled pixels of large scenes
# ----------------------------------------------------------------------------

def pixel_list(pre, px, py):
    """Gaussians whose pixel rectangle holds (px, py), ordered by
    (depth key, index) — the order any tile list gives them."""
    m = (pre.visible & (pre.rect[0] <= px) & (pre.rect[1] >= px)
         & (pre.rect[2] <= py) & (pre.rect[3] >= py))
    g = np.nonzero(m)[0]
    order = np.lexsort((g, pre.depth_bits[g]))
    return g[order]


def tile_position(pre, tile_x, tile_y, g):
    """Position of Gaussian g in the sorted list of tile (tile_x, tile_y)."""
    tr = pre.tile_rect
    m = (pre.visible & (tr[0] <= tile_x) & (tr[1] >= tile_x)
         & (tr[2] <= tile_y) & (tr[3] >= tile_y))
    b = pre.depth_bits
    before = m & ((b < b[g]) | ((b == b[g]) & (np.arange(b.size) < g)))
    return int(before.sum())


def render_pixel(pre, cam, opts, px, py):
    """(rgb(3), depth, T, n_contrib, flagged, outcomes) of one pixel by brute
    force; n_contrib is expressed as a position in the pixel's tile list."""
    bg = cam.bg.astype(F64)
    entries = pixel_list(pre, px, py)
    C, D, T, nn, fl, _ = _blend_tile(pre, entries, np.array([px]), np.array([py]), opts, bg)
    n_loc = int(nn[0])
    if n_loc > 0:
        g_last = entries[n_loc - 1]
        n_tile = tile_position(pre, px // int(opts.tile_w), py // int(opts.tile_h), g_last) + 1
    else:
        n_tile = 0
    outs = None
    if fl[0]:
        raw = pixel_outcomes(pre, entries, px, py, opts, bg)
        if raw is not None:
            outs = []
            for (c, d, t, k) in raw:
                kt = 0 if k == 0 else tile_position(
                    pre, px // int(opts.tile_w), py // int(opts.tile_h), entries[k - 1]) + 1
                outs.append((c, d, t, kt))
    return (C[:, 0] + T[0] * bg, float(D[0]), float(T[0]), n_tile, bool(fl[0]), outs)
