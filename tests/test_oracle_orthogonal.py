"""Pins of the oracle's orthogonal-lobe colour forms and adaptive SH degree
(paper: Methods, Multi-Axis Orthogonal Gaussians, eqs. 7-8; Mixing
Spherical Harmonics and Spherical Gaussians; Experiments, Implementation)
— no GPU.

World axes: three lobes on (1,0,0), (0,1,0), (0,0,1).  Frame: three lobes
on the columns of the rotation with quaternion (1, omega)/|(1, omega)|,
checked against scipy's rotation of the same quaternion.  Adaptive SH: the
colour of a Gaussian whose degree the radius rule lowers equals the colour
of the same Gaussian in a scene of that lower degree.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import backward as G
from oracle import forward as F
from paper_2501_00342_amd import scenes

OPTS = scenes.Options()


def _scene_at(points, lobe_mode, axes, lsh, amp, sh):
    n = points.shape[1]
    return scenes.Scene(
        (int(round(math.sqrt(sh.shape[0]))) - 1), lsh.shape[0],
        np.ascontiguousarray(points.astype(np.float32)),
        np.full((3, n), -3.0, np.float32),
        np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, n)),
        np.zeros(n, np.float32), sh.astype(np.float32), axes.astype(np.float32),
        lsh.astype(np.float32), amp.astype(np.float32), lobe_mode=lobe_mode)


def test_world_axes_closed_form():
    """Seen along +x the first lobe gives its amplitude a_0 (d . e_x = 1);
    the others are perpendicular (d . e_k = 0) and give a_k exp(-lambda_k)."""
    cam = scenes.pinhole(64, 64, np.eye(3), (0.0, 0.0, 0.0))
    rng = np.random.default_rng(0)
    lsh = rng.normal(1.0, 0.5, (3, 3))
    amp = rng.normal(0.0, 0.2, (3, 3, 3))
    sh = np.zeros((1, 3, 3))
    pts = np.array([[3.0, 0.0, 0.0], [0.0, 3.0, 0.0], [0.0, 0.0, 3.0]]).T   # along e_x, e_y, e_z
    sc = _scene_at(pts, scenes.LOBES_WORLD, np.zeros((0, 3, 3)), lsh, amp, sh)
    pre = F.preprocess(sc, cam, OPTS)
    lam = np.exp(lsh.astype(np.float32).astype(np.float64))
    a = amp.astype(np.float32).astype(np.float64)
    for g in range(3):
        want = 0.5 + sum(a[k, :, g] * (1.0 if k == g else math.exp(-lam[k, g])) for k in range(3))
        assert np.allclose(pre.rgb_raw[:, g], want, rtol=0, atol=1e-14), g


def test_frame_axes_are_orthonormal_and_right_handed():
    """eq. 8: mu_i . mu_j = delta_ij for any 3 frame parameters."""
    rng = np.random.default_rng(1)
    n = 500
    sc = scenes.orthogonal_scene(n, 1, scenes.LOBES_FRAME)
    sc.sg_axes[0] = rng.normal(0.0, 3.0, (3, n)).astype(np.float32)
    mu = F.lobe_axes(sc)                                   # (3, 3, N)
    gram = np.einsum("ian,jan->ijn", mu, mu)
    assert np.abs(gram - np.eye(3)[:, :, None]).max() < 1e-14
    det = np.einsum("an,an->n", np.cross(mu[0], mu[1], axis=0), mu[2])
    assert np.abs(det - 1.0).max() < 1e-14


def test_frame_axes_match_scipy_rotation():
    """The frame's columns are scipy's rotation matrix of the quaternion
    (w, x, y, z) = (1, omega) normalised (scipy takes (x, y, z, w))."""
    sc = scenes.orthogonal_scene(200, 2, scenes.LOBES_FRAME)
    mu = F.lobe_axes(sc)
    om = sc.sg_axes[0].astype(np.float64)
    for g in range(0, 200, 7):
        Rm = Rotation.from_quat([om[0, g], om[1, g], om[2, g], 1.0]).as_matrix()
        for k in range(3):
            assert np.allclose(mu[k, :, g], Rm[:, k], rtol=0, atol=1e-14), (g, k)


def test_frame_zero_parameters_give_world_axes():
    sc = scenes.orthogonal_scene(300, 3, scenes.LOBES_FRAME)
    sc.sg_axes[:] = 0.0
    w = sc.copy()
    w.lobe_mode = scenes.LOBES_WORLD
    w.sg_axes = np.zeros((0, 3, sc.n), np.float32)
    cam = scenes.config1_camera(64, 48)
    a, b = F.preprocess(sc, cam, OPTS), F.preprocess(w, cam, OPTS)
    assert np.array_equal(a.rgb_raw, b.rgb_raw)


def test_orthogonal_modes_equal_free_lobes_on_the_same_axes():
    """A frame (or world) scene renders as the free-lobe scene whose axes
    are scipy's rotation columns (or the identity's)."""
    cam = scenes.config1_camera(96, 64)
    for mode in (scenes.LOBES_FRAME, scenes.LOBES_WORLD):
        sc = scenes.orthogonal_scene(3000, 4, mode, sh_degree=1)
        n = sc.n
        axes = np.empty((3, 3, n))
        if mode == scenes.LOBES_FRAME:
            om = sc.sg_axes[0].astype(np.float64)
            Rm = Rotation.from_quat(np.stack([om[0], om[1], om[2], np.ones(n)], axis=1)).as_matrix()
            for k in range(3):
                axes[k] = Rm[:, :, k].T
        else:
            axes[:] = np.eye(3)[:, :, None]
        free = sc.copy()
        free.lobe_mode = scenes.LOBES_FREE
        free.sg_axes = axes           # float64 axes: the oracle reads them as given
        a, b = F.render(sc, cam, OPTS), F.render(free, cam, OPTS)
        assert np.abs(a.image - b.image).max() < 1e-12, mode
        assert np.array_equal(a.n_contrib, b.n_contrib)


def test_three_orthogonal_lobes_use_fifteen_colour_parameters(repo_root):
    """4 per lobe (RGB amplitude, sharpness) and 3 for the frame (Methods,
    Multi-Axis Orthogonal Gaussians), excluding the diffuse term."""
    with open(os.path.join(repo_root, "tests", "golden", "param_counts.json")) as f:
        gold = json.load(f)
    sc = scenes.orthogonal_scene(10, 0, scenes.LOBES_FRAME)
    per = sum(a.reshape(-1, sc.n).shape[0]
              for a in (sc.sg_axes, sc.sg_log_sharpness, sc.sg_amplitudes))
    assert per == gold["colour_params_three_orthogonal_sg_plus_frame"] == 15
    w = scenes.orthogonal_scene(10, 0, scenes.LOBES_WORLD)
    assert sum(a.reshape(-1, w.n).shape[0]
               for a in (w.sg_axes, w.sg_log_sharpness, w.sg_amplitudes)) == 12


def test_adaptive_degree_rule_and_truncated_colour():
    """Each Gaussian's degree follows the radius rule, and its colour equals
    the colour of the same Gaussian in the scene of that fixed degree (the
    first (d+1)^2 coefficients)."""
    sc = scenes.orthogonal_scene(4000, 5, scenes.LOBES_FRAME, sh_degree=2, sh_adaptive=(2, 8))
    cam = scenes.config1_camera(128, 96)
    pre = F.preprocess(sc, cam, OPTS)
    v = pre.visible
    r = pre.radius
    deg = F.sh_degrees(sc, r)
    want = np.where(r <= 2, 0, np.where(r <= 8, 1, 2))
    assert np.array_equal(deg[v], want[v])
    counts = np.bincount(deg[v], minlength=3)
    assert (counts > 0).all(), counts            # the scene exercises every degree
    for d in range(3):
        low = sc.copy()
        low.sh_degree = d
        low.sh = np.ascontiguousarray(sc.sh[:(d + 1) ** 2])
        low.sh_adaptive = (0, 0)
        ref = F.preprocess(low, cam, OPTS)
        m = v & (deg == d)
        assert np.array_equal(pre.rgb_raw[:, m], ref.rgb_raw[:, m]), d


def test_adaptive_off_equals_fixed_degree():
    sc = scenes.orthogonal_scene(2000, 6, scenes.LOBES_WORLD, sh_degree=2)
    cam = scenes.config1_camera(64, 48)
    a = F.preprocess(sc, cam, OPTS)
    sc.sh_adaptive = (0, 0)
    b = F.preprocess(sc, cam, OPTS)
    assert np.array_equal(a.rgb_raw, b.rgb_raw)
    assert np.array_equal(F.sh_degrees(sc, a.radius), np.full(sc.n, 2))


def _fd_case(mode, sh_degree, adaptive):
    sc = scenes.orthogonal_scene(64, 7, mode, sh_degree=sh_degree, sh_adaptive=adaptive,
                                 n_clusters=4)
    return sc, scenes.config1_camera(32, 32), scenes.target_image(32, 32, 2)


@pytest.mark.parametrize("mode,deg,adaptive,field", [
    (scenes.LOBES_FRAME, 2, (2, 8), "sg_axes"),
    (scenes.LOBES_FRAME, 2, (2, 8), "sh"),
    (scenes.LOBES_FRAME, 2, (2, 8), "means"),
    (scenes.LOBES_FRAME, 1, (0, 0), "sg_log_sharpness"),
    (scenes.LOBES_WORLD, 0, (0, 0), "sg_amplitudes"),
    (scenes.LOBES_WORLD, 0, (0, 0), "means"),
])
def test_orthogonal_gradients_match_finite_differences(mode, deg, adaptive, field):
    sc, cam, tgt = _fd_case(mode, deg, adaptive)
    _, _, _, grads = G.render_and_grad(sc, cam, OPTS, target=tgt)
    pre = F.preprocess(sc, cam, OPTS)
    vis = np.nonzero(pre.visible)[0]
    assert vis.size >= 10
    rng = np.random.default_rng(abs(hash((mode, field))) % 2 ** 32)
    arr = getattr(sc, field)
    checked = 0
    for _ in range(12):
        g = int(rng.choice(vis))
        idx = tuple(int(rng.integers(0, s)) for s in arr.shape[:-1]) + (g,)
        fd, ok = G.fd_grad(sc, cam, OPTS, tgt, field, idx)
        if not ok:
            continue
        an = grads[field][idx]
        assert abs(an - fd) <= 1e-4 * max(abs(an), abs(fd)) + 2e-10, (field, idx, an, fd)
        checked += 1
    assert checked >= 6


def test_adaptive_sh_unused_coefficients_get_zero_gradient():
    sc, cam, tgt = _fd_case(scenes.LOBES_FRAME, 2, (2, 8))
    _, _, _, grads = G.render_and_grad(sc, cam, OPTS, target=tgt)
    pre = F.preprocess(sc, cam, OPTS)
    deg = F.sh_degrees(sc, pre.radius)
    for g in np.nonzero(pre.visible)[0]:
        used = (deg[g] + 1) ** 2
        assert np.all(grads["sh"][used:, :, g] == 0.0)
