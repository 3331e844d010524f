"""Pins of the oracle's colour model (paper eqs. 4-9) against closed forms,
quadrature and scipy — no GPU."""
import json
import math
import os

import numpy as np
import pytest
from scipy.special import sph_harm_y

import oracle
from oracle import forward as F
from oracle.sh import sh_basis, sh_basis_grad
from paper_2501_00342_amd import scenes


def _sphere_quadrature(nz=24, nphi=48):
    """Gauss-Legendre in cos(theta) x uniform phi: exact for polynomials of
    degree < min(2 nz, nphi) on the sphere."""
    zs, wz = np.polynomial.legendre.leggauss(nz)
    phis = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    Z, P = np.meshgrid(zs, phis, indexing="ij")
    Wt = np.repeat(wz[:, None], nphi, axis=1) * (2 * math.pi / nphi)
    s = np.sqrt(1 - Z ** 2)
    d = np.stack([s * np.cos(P), s * np.sin(P), Z]).reshape(3, -1)
    return d, Wt.ravel()


def test_sh_orthonormal_by_quadrature():
    d, w = _sphere_quadrature()
    Y = sh_basis(3, d)
    gram = (Y * w) @ Y.T
    assert np.allclose(gram, np.eye(16), atol=1e-12)


def test_sh_matches_scipy_complex_harmonics():
    """Real basis with Condon-Shortley phase = sqrt(2) Re/Im of scipy's
    complex Y_l^m (which carries the phase)."""
    rng = np.random.default_rng(1)
    v = rng.standard_normal((3, 200))
    v /= np.linalg.norm(v, axis=0)
    theta = np.arccos(np.clip(v[2], -1, 1))
    phi = np.arctan2(v[1], v[0])
    Y = sh_basis(3, v)
    i = 0
    for l in range(4):
        for m in range(-l, l + 1):
            c = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                ref = math.sqrt(2) * c.real
            elif m < 0:
                ref = math.sqrt(2) * c.imag
            else:
                ref = c.real
            assert np.allclose(Y[i], ref, atol=1e-12), (l, m)
            i += 1


def test_sh_low_degree_textbook_forms():
    rng = np.random.default_rng(2)
    v = rng.standard_normal((3, 50))
    v /= np.linalg.norm(v, axis=0)
    Y = sh_basis(1, v)
    c0 = 0.5 / math.sqrt(math.pi)
    c1 = math.sqrt(3.0 / (4.0 * math.pi))
    assert np.allclose(Y[0], c0)
    assert np.allclose(Y[1], -c1 * v[1])
    assert np.allclose(Y[2], c1 * v[2])
    assert np.allclose(Y[3], -c1 * v[0])


def test_sh_gradient_matches_numeric_derivative():
    rng = np.random.default_rng(3)
    v = rng.standard_normal((3, 20))
    G = sh_basis_grad(3, v)
    h = 1e-6
    for k in range(3):
        e = np.zeros((3, 1))
        e[k] = h
        num = (sh_basis(3, v + e) - sh_basis(3, v - e)) / (2 * h)
        assert np.allclose(G[:, k, :], num, atol=1e-7)


def _one_lobe_scene(n, mu, log_sharp, amp):
    z = np.zeros
    sh = z((1, 3, n), np.float32)
    return scenes.Scene(
        0, 1, z((3, n), np.float32), np.full((3, n), -3, np.float32),
        np.tile(np.array([[1], [0], [0], [0]], np.float32), (1, n)), z(n, np.float32), sh,
        np.tile(np.asarray(mu, np.float32).reshape(1, 3, 1), (1, 1, n)),
        np.full((1, n), log_sharp, np.float32),
        np.tile(np.asarray(amp, np.float32).reshape(1, 3, 1), (1, 1, n)))


def test_sg_equals_amplitude_along_its_axis_and_decays_to_antipode():
    """eq. 5: C(d) = a exp(lambda (d.mu - 1)) is a at d = mu and
    a exp(-2 lambda) at d = -mu.  Evaluated through the whole preprocess
    by placing the Gaussian on the lobe axis as seen from the camera."""
    cam = scenes.pinhole(128, 128, np.eye(3), (0.0, 0.0, 0.0))
    cc = F.camera_centre(cam)
    assert np.all(cc == 0)
    mu = np.array([0.3, -0.2, 0.93])
    mu /= np.linalg.norm(mu)
    amp = np.array([0.2, -0.1, 0.05])
    for lsh in (0.0, 1.0, 2.0):
        sc = _one_lobe_scene(2, mu, lsh, amp)
        sc.means[:, 0] = (cc + 3.0 * mu).astype(np.float32)
        sc.means[:, 1] = (cc - 3.0 * mu).astype(np.float32)
        sc.sg_axes[0, :, 0] = sc.means[:, 0]          # axis = exact view direction
        sc.sg_axes[0, :, 1] = sc.means[:, 0]
        pre = F.preprocess(sc, cam, scenes.Options())
        lam = math.exp(float(np.float32(lsh)))
        ampf = amp.astype(np.float32).astype(np.float64)
        assert np.allclose(pre.rgb_raw[:, 0], 0.5 + ampf, atol=1e-12)
        assert np.allclose(pre.rgb_raw[:, 1], 0.5 + ampf * math.exp(-2 * lam), atol=1e-6)


def test_sg_small_sharpness_limit_and_monotonic_sharpening():
    d, _ = _sphere_quadrature(8, 16)
    mu = np.array([0.0, 0.0, 1.0])
    sc = _one_lobe_scene(d.shape[1], mu, -30.0, [1.0, 1.0, 1.0])
    c = F.colour(sc, d) - 0.5
    assert np.allclose(c, 1.0, atol=1e-12)           # lambda -> 0: constant a
    prev = None
    off_axis = d[2] < 0.999
    for lsh in (-1.0, 0.0, 1.0, 2.0):
        sc = _one_lobe_scene(d.shape[1], mu, lsh, [1.0, 1.0, 1.0])
        c = (F.colour(sc, d) - 0.5)[0]
        if prev is not None:                         # larger lambda, sharper lobe
            assert np.all(c[off_axis] < prev[off_axis])
        prev = c


@pytest.mark.parametrize("lsh", [-1.0, 0.5, 2.0])
def test_sg_sphere_integral(lsh):
    """int_S2 exp(lambda (d.mu - 1)) = 2 pi (1 - exp(-2 lambda)) / lambda."""
    d, w = _sphere_quadrature(64, 8)
    mu = np.array([0.0, 0.0, 1.0])
    sc = _one_lobe_scene(d.shape[1], mu, lsh, [1.0, 0.0, 0.0])
    c = (F.colour(sc, d) - 0.5)[0]
    lam = math.exp(float(np.float32(lsh)))
    assert abs((c * w).sum() - 2 * math.pi * (1 - math.exp(-2 * lam)) / lam) < 1e-10


def test_colour_clamp_and_offset():
    """R4: rgb = max(0, 0.5 + SH + SG); a very negative DC coefficient
    clamps to 0."""
    sc = scenes.config0_scene(0, 4)
    sc.sg_amplitudes[:] = 0
    sc.sh[0, :, 0] = -10.0
    sc.sh[0, :, 1] = 0.0
    pre = F.preprocess(sc, scenes.config0_camera(), scenes.Options())
    assert np.all(pre.rgb[:, 0] == 0.0) and np.all(pre.rgb_raw[:, 0] < 0)
    assert np.allclose(pre.rgb[:, 1], 0.5)


def test_sh3_form_reduces_to_lower_degree():
    """Degree-3 SH with only degree-0/1 coefficients equals the degree-1
    form with no lobes."""
    sc3 = scenes.sh3_scene(300, 5, n_clusters=5)
    sc3.sh[4:] = 0.0
    sc1 = scenes.Scene(1, 0, sc3.means, sc3.log_scales, sc3.quats, sc3.opacity_logits,
                       np.ascontiguousarray(sc3.sh[:4]), sc3.sg_axes, sc3.sg_log_sharpness,
                       sc3.sg_amplitudes)
    cam = scenes.config1_camera(64, 48)
    a = F.preprocess(sc3, cam, scenes.Options())
    b = F.preprocess(sc1, cam, scenes.Options())
    assert np.allclose(a.rgb_raw, b.rgb_raw, atol=1e-14)


def test_parameter_counts_match_the_paper(repo_root):
    g = json.load(open(os.path.join(repo_root, "tests", "golden", "param_counts.json")))
    sh3 = scenes.sh3_scene(10, 0, n_clusters=2)
    assert sh3.sh.shape[0] == g["sh3_coeffs_per_channel"]
    assert sh3.sh.shape[0] * 3 == g["sh3_coeffs_total"]
    assert sh3.floats_per_gaussian() == g["gaussian_params_sh3"]
    one = _one_lobe_scene(1, [0, 0, 1], 0.0, [1, 1, 1])
    assert one.floats_per_gaussian() - 11 - 3 == g["params_single_sg"]
    assert one.floats_per_gaussian() - 11 == g["colour_params_diffuse_plus_sg"]
    # three orthogonal lobes: colour 3 + sharpness 1 per lobe, plus a frame of 3
    assert 3 * (3 + 1) + 3 == g["colour_params_three_orthogonal_sg_plus_frame"]


def test_half_rounding_helpers_match_torch():
    """The test helpers' bfloat16 / float16 rounding (ties to even) against
    torch's CPU conversions, on random, tie and boundary values."""
    import torch
    from tests.half_colour import round_bf16, round_f16
    rng = np.random.default_rng(5)
    a = np.concatenate([rng.normal(0, 1, 4000), rng.normal(0, 1e-3, 1000),
                        rng.normal(0, 300, 1000)]).astype(np.float32)
    ties = (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32)
    odd = ((np.arange(1, 200, dtype=np.uint32) * 2 + 1) << 16 | 0x8000).view(np.float32)
    x = np.concatenate([a, ties, -ties, odd])
    tb = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    th = torch.from_numpy(x).to(torch.float16).float().numpy()
    assert np.array_equal(round_bf16(x), tb)
    assert np.array_equal(round_f16(x), th)
