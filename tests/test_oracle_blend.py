"""Pins of the oracle's keys, sort, ranges and alpha blending against
textbook routines, brute force and closed forms — no GPU."""
import math

import numpy as np
import pytest

import oracle
from oracle import forward as F
from paper_2501_00342_amd import scenes

OPTS = scenes.Options()


def test_sort_and_ranges_three_independent_agreements():
    sc = scenes.config0_scene(0)
    cam = scenes.config0_camera()
    pre = F.preprocess(sc, cam, OPTS)
    keys, vals, ntiles = F.emit_pairs(pre)
    sk, sv = F.sort_pairs(keys, vals)
    # (1) Python's sorted() over (tile, depth bits, g) tuples
    tup = sorted(zip((keys >> np.uint64(32)).tolist(),
                     (keys & np.uint64(0xFFFFFFFF)).tolist(), vals.tolist()))
    assert [((t << 32) | d) for t, d, _ in tup] == sk.tolist()
    assert [g for *_, g in tup] == sv.tolist()
    # (2) a plain loop for ranges
    rng = F.tile_ranges(sk, ntiles)
    tiles = (sk >> np.uint64(32)).tolist()
    for t in range(ntiles):
        idx = [i for i, x in enumerate(tiles) if x == t]
        assert tuple(rng[t]) == ((idx[0], idx[-1] + 1) if idx else (0, 0))
    # (3) emission: every visible Gaussian once per tile of its rectangle
    cnt = np.bincount(vals.astype(np.int64), minlength=sc.n)
    assert np.array_equal(cnt, pre.tiles_touched)


def test_equal_depth_ties_keep_gaussian_order():
    sc = scenes.config0_scene(0, 10)
    sc.means[:, :] = np.array([[0.0], [0.0], [0.0]], np.float32)
    pre = F.preprocess(sc, scenes.config0_camera(), OPTS)
    keys, vals, _ = F.emit_pairs(pre)
    sk, sv = F.sort_pairs(keys, vals)
    for t in np.unique(sk >> np.uint64(32)):
        m = (sk >> np.uint64(32)) == t
        assert np.all(np.diff(sv[m].astype(np.int64)) > 0)


def test_tiled_blend_equals_brute_force_per_pixel():
    sc = scenes.config0_scene(1, 400)
    cam = scenes.config0_camera(48, 40)
    img = F.render(sc, cam, OPTS)
    pre = F.preprocess(sc, cam, OPTS)
    for py in range(0, 40, 3):
        for px in range(0, 48, 5):
            rgb, d, T, n, fl, _ = F.render_pixel(pre, cam, OPTS, px, py)
            assert np.array_equal(rgb, img.image[:, py, px])
            assert d == img.depth[py, px] and T == img.final_T[py, px]
            assert n == img.n_contrib[py, px]


def _iso_scene(centres, ls, logits, dc):
    n = len(centres)
    z = np.zeros
    sh = z((1, 3, n), np.float32)
    sh[0] = np.asarray(dc, np.float32).T
    return scenes.Scene(0, 0, np.asarray(centres, np.float32).T, np.full((3, n), ls, np.float32),
                        np.tile(np.array([[1], [0], [0], [0]], np.float32), (1, n)),
                        np.asarray(logits, np.float32), sh, z((0, 3, n), np.float32),
                        z((0, n), np.float32), z((0, 3, n), np.float32))


C0 = 0.5 / math.sqrt(math.pi)


def test_single_gaussian_closed_form():
    """image = alpha rgb + (1 - alpha) bg, alpha = min(0.99, sigma e^{-|d|^2/(2 v)})
    with v = (f s / z)^2 + 0.3 for an isotropic Gaussian on the axis."""
    bg = np.array([0.1, 0.2, 0.3], np.float32)
    cam = scenes.pinhole(33, 33, np.eye(3), (0.0, 0.0, 0.0), bg=bg)
    sc = _iso_scene([[0, 0, 3.0]], -4.0, [0.5], [[0.2, -0.1, 0.4]])
    img = F.render(sc, cam, OPTS)
    s = math.exp(float(np.float32(-4.0)))
    var = (cam.fx * s / 3.0) ** 2 + float(np.float32(0.3))
    sig = 1 / (1 + math.exp(-0.5))
    rgb = 0.5 + C0 * np.float32([0.2, -0.1, 0.4]).astype(np.float64)
    r = math.ceil(3 * math.sqrt(var))
    for py in range(33):
        for px in range(33):
            d2 = (px - 16) ** 2 + (py - 16) ** 2
            a = min(float(np.float32(0.99)), sig * math.exp(-0.5 * d2 / var))
            inside = abs(px - 16) <= r and abs(py - 16) <= r
            if not inside or a < float(np.float32(1 / 255)):
                exp_img = bg.astype(np.float64)
            else:
                exp_img = a * rgb + (1 - a) * bg
            assert np.allclose(img.image[:, py, px], exp_img, atol=1e-12)


def test_two_gaussian_compositing_closed_form():
    cam = scenes.pinhole(9, 9, np.eye(3), (0.0, 0.0, 0.0))
    sc = _iso_scene([[0, 0, 3.0], [0, 0, 2.0]], -3.0, [0.3, -0.2],
                    [[0.3, 0.0, -0.3], [-0.2, 0.5, 0.1]])
    img = F.render(sc, cam, OPTS)
    pre = F.preprocess(sc, cam, OPTS)
    # nearer Gaussian (index 1) first
    a2 = pre.opacity[1]
    a1 = pre.opacity[0]
    c = a2 * pre.rgb[:, 1] + (1 - a2) * a1 * pre.rgb[:, 0]
    assert np.allclose(img.image[:, 4, 4], c, atol=1e-14)
    assert img.final_T[4, 4] == pytest.approx((1 - a2) * (1 - a1), rel=1e-14)
    assert img.n_contrib[4, 4] == 2


def test_zero_opacity_gives_background():
    bg = np.array([0.3, 0.6, 0.9], np.float32)
    sc = scenes.config0_scene(0, 200)
    sc.opacity_logits[:] = -1e4
    cam = scenes.config0_camera(40, 40)
    cam.bg = bg
    img = F.render(sc, cam, OPTS)
    assert np.all(img.image == bg.astype(np.float64)[:, None, None])
    assert np.all(img.final_T == 1.0) and np.all(img.n_contrib == 0) and np.all(img.depth == 0)


def test_full_opacity_saturates_at_alpha_max_and_stops():
    cam = scenes.pinhole(9, 9, np.eye(3), (0.0, 0.0, 0.0))
    sc = _iso_scene([[0, 0, 2.0], [0, 0, 3.0], [0, 0, 4.0]], -1.0, [30.0, 30.0, 30.0],
                    [[0.1, 0.1, 0.1]] * 3)
    img = F.render(sc, cam, OPTS)
    amax = float(np.float32(0.99))
    # first blends with alpha_max; second would bring T below T_min: stop
    assert img.final_T[4, 4] == 1 - amax
    assert img.n_contrib[4, 4] == 1


def test_input_order_invariance():
    sc = scenes.config0_scene(2, 500)
    cam = scenes.config0_camera(64, 64)
    a = F.render(sc, cam, OPTS)
    perm = np.random.default_rng(0).permutation(500)
    b = F.render(sc.subset(perm), cam, OPTS)
    assert np.array_equal(a.image, b.image) and np.array_equal(a.final_T, b.final_T)
    assert np.array_equal(a.depth, b.depth) and np.array_equal(a.n_contrib, b.n_contrib)


@pytest.mark.parametrize("tw,th", [(8, 8), (32, 8), (16, 32)])
def test_image_independent_of_tile_size(tw, th):
    sc = scenes.config0_scene(3, 500)
    cam = scenes.config0_camera(70, 50)
    a = F.render(sc, cam, OPTS)
    b = F.render(sc, cam, scenes.Options(tile_w=tw, tile_h=th))
    assert np.array_equal(a.image, b.image) and np.array_equal(a.final_T, b.final_T)
    assert np.array_equal(a.depth, b.depth)


def test_tie_band_outcomes_contain_the_fp64_result():
    sc = scenes.config0_scene(0)
    cam = scenes.config0_camera()
    img = F.render(sc, cam, OPTS)
    for (py, px), outs in img.alternatives.items():
        assert outs is not None and len(outs) >= 2
        c, d, T, n = outs[-1]                        # the FP64 decision path
        assert np.array_equal(c, img.image[:, py, px]) and n == img.n_contrib[py, px]
        assert any(not np.array_equal(o[0], c) for o in outs[:-1])


def test_batched_keys_are_per_camera_keys_with_tile_bases():
    sc = scenes.config0_scene(0, 300)
    cams = [scenes.config0_camera(40, 30), scenes.pinhole(24, 20, np.eye(3), (0.1, 0, 3.5))]
    pres, outs, keys, vals, ranges = F.render_batch(sc, cams, OPTS)
    base = 0
    for ci, cam in enumerate(cams):
        single = F.render(sc, cam, OPTS)
        assert np.array_equal(outs[ci].image, single.image)
        m = (vals // 300) == ci
        k = keys[m] - (np.uint64(base) << np.uint64(32))
        assert np.array_equal(k, single.keys)
        assert np.array_equal(vals[m] - ci * 300, single.values)
        base += pres[ci].grid[0] * pres[ci].grid[1]


# ---- tie-band enumeration pinned by closed forms --------------------------
# A pixel at a splat's centre has power 0, so alpha = min(alpha_max, sigma):
# hand-placed splats put alpha or the next transmittance inside a tie band,
# and every alternative outcome is the compositing sum written out.

def _centre_splats(sigmas, rgbs, zs):
    """A Pre-like record of splats all centred on pixel (2, 2)."""
    from types import SimpleNamespace
    n = len(sigmas)
    return SimpleNamespace(
        rect=np.array([[0] * n, [4] * n, [0] * n, [4] * n], np.int64),
        conic=np.array([[1.0] * n, [0.0] * n, [1.0] * n]),
        u=np.full(n, 2.0), v=np.full(n, 2.0),
        opacity=np.asarray(sigmas, np.float64),
        rgb=np.asarray(rgbs, np.float64).T.copy(), z=np.asarray(zs, np.float64))


AMIN = float(np.float32(1.0 / 255.0))
AMAX = float(np.float32(0.99))
TMIN = float(np.float32(1e-4))
BG = np.array([0.25, 0.5, 0.75])


def _same(outs, expected):
    assert outs is not None and len(outs) == len(expected)
    for (c, d, T, n), (ce, de, Te, ne) in zip(outs, expected):
        assert n == ne
        assert np.allclose(c, ce, rtol=1e-13, atol=1e-15)
        assert abs(d - de) <= 1e-13 * abs(de) + 1e-15 and abs(T - Te) <= 1e-13 * Te


@pytest.mark.parametrize("rel", [5e-5, -5e-5])
def test_tie_outcomes_alpha_band_closed_form(rel):
    """One splat with alpha inside the alpha_min band: the skip outcome
    (background, T = 1, n = 0) and the blend outcome (a c + (1 - a) bg,
    D = a z, T = 1 - a, n = 1), the FP64 decision last."""
    a = AMIN * (1.0 + rel)
    rgb, z = np.array([0.9, 0.2, 0.4]), 3.5
    pre = _centre_splats([a], [rgb], [z])
    outs = F.pixel_outcomes(pre, [0], 2, 2, OPTS, BG)
    skip = (BG.copy(), 0.0, 1.0, 0)
    blend = (a * rgb + (1.0 - a) * BG, a * z, 1.0 - a, 1)
    _same(outs, [skip, blend] if rel > 0 else [blend, skip])


def test_tie_outcomes_transmittance_band_closed_form():
    """A saturated splat (alpha = alpha_max) then one whose blend leaves T
    just above t_min: the stop outcome (only the first splat) and the blend
    outcome (both), the FP64 decision (blend) last."""
    a1 = AMAX
    T1 = 1.0 - a1
    a2 = 1.0 - TMIN * (1.0 + 5e-4) / T1
    c1, c2 = np.array([0.3, 0.6, 0.9]), np.array([0.8, 0.1, 0.5])
    z1, z2 = 2.0, 2.5
    pre = _centre_splats([1.0, a2], [c1, c2], [z1, z2])
    outs = F.pixel_outcomes(pre, [0, 1], 2, 2, OPTS, BG)
    T2 = T1 * (1.0 - a2)
    stop = (a1 * c1 + T1 * BG, a1 * z1, T1, 1)
    both = (a1 * c1 + a2 * T1 * c2 + T2 * BG, a1 * z1 + a2 * T1 * z2, T2, 2)
    _same(outs, [stop, both])
    assert TMIN <= T2 <= TMIN * (1.0 + F.T_BAND)


def test_tie_outcomes_nested_bands_closed_form():
    """alpha_min band on the first splat, then a saturated splat, then a
    splat whose T' lies in the t_min band only on the path that blended the
    first: three outcomes, each the compositing sum of its own subset."""
    a0 = AMIN * (1.0 + 5e-5)
    a1 = AMAX
    Tb = (1.0 - a0) * (1.0 - a1)              # T before splat 2, splat 0 blended
    a2 = 1.0 - TMIN * (1.0 + 5e-4) / Tb
    cs = [np.array([0.1, 0.2, 0.3]), np.array([0.7, 0.4, 0.2]), np.array([0.5, 0.9, 0.6])]
    zs = [1.5, 2.0, 2.5]
    pre = _centre_splats([a0, 1.0, a2], cs, zs)
    outs = F.pixel_outcomes(pre, [0, 1, 2], 2, 2, OPTS, BG)

    def composite(used):
        T, C, D = 1.0, np.zeros(3), 0.0
        alphas = [a0, a1, a2]
        for j in used:
            C = C + alphas[j] * T * cs[j]
            D = D + alphas[j] * T * zs[j]
            T = T * (1.0 - alphas[j])
        return (C + T * BG, D, T, used[-1] + 1 if used else 0)

    # on the skip branch T before splat 2 is 1 - a1, so T' sits 0.4% above
    # the FP64 path's: outside the t_min band, splat 2 blends
    assert (1.0 - a1) * (1.0 - a2) > TMIN * (1.0 + F.T_BAND)
    _same(outs, [composite([1, 2]), composite([0, 1]), composite([0, 1, 2])])


def test_tie_outcomes_none_outside_bands():
    """Decisions far from both bands give the single FP64 outcome."""
    pre = _centre_splats([0.5, 0.3], [np.ones(3), np.zeros(3)], [1.0, 2.0])
    outs = F.pixel_outcomes(pre, [0, 1], 2, 2, OPTS, BG)
    # D = 0.5 * 1.0 + (0.3 * 0.5) * 2.0
    _same(outs, [(0.5 * np.ones(3) + 0.35 * BG, 0.8, 0.35, 2)])
