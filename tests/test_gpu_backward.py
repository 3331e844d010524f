"""Backward parity of the HIP path against the FP64 oracle (GPU)."""
import numpy as np
import pytest
import torch

from oracle import backward as OB
from oracle import forward as F
from paper_2501_00342_amd import raster, scenes
from tests import parity
from tests.gpu_util import camera_numpy, run_forward

pytestmark = pytest.mark.gpu

FIELDS = scenes.FIELDS


def _tie_exclusion(pre, ref):
    """Gaussians whose rectangle holds a tie-band pixel."""
    ex = np.zeros(pre.z.shape[0], bool)
    for py, px in zip(*np.nonzero(ref.flagged)):
        ex |= (pre.visible & (pre.rect[0] <= px) & (pre.rect[1] >= px)
               & (pre.rect[2] <= py) & (pre.rect[3] >= py))
    return ex


def _backward_case(sc, cam, opts, seed):
    rast, params, out = run_forward(sc, [cam], opts)
    ref = F.render(sc, cam, opts)
    pre = F.preprocess(sc, cam, opts)
    tgt = scenes.target_image(cam.width, cam.height, seed)
    # the same upstream gradient for both sides: L1 of the oracle image
    _, gimg = OB.l1_loss(ref.image, tgt)
    g_dev = torch.from_numpy(gimg.astype(np.float32).reshape(-1)).cuda()
    grads = rast.backward(params, out, g_dev)
    g2_gpu = rast.grad2d().cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    g2_ref = OB.blend_backward(pre, cam, opts, ref.values, ref.ranges, gimg)
    grads_ref = OB.preprocess_backward(sc, cam, opts, pre, g2_ref)
    ex = _tie_exclusion(pre, ref)
    return rast, grads, g2_gpu, g2_ref, grads_ref, ex


def _assert_grads(gpu, ref, ex, what):
    rep = parity.compare_grads(gpu, ref, ex)
    for k, r in rep.items():
        assert r["rel_l2"] <= parity.GRAD_REL and r["elem_viol"] == 0, (what, k, r, rep)


@pytest.mark.parametrize("n,w,h,seed", [(64, 32, 32, 7), (3000, 96, 64, 21), (8000, 160, 112, 22)])
def test_backward_matches_oracle(n, w, h, seed):
    if n == 64:
        sc, cam = scenes.small_clustered(64, 7, 32, 32, n_clusters=4)
    else:
        sc, cam = scenes.small_clustered(n, seed, w, h)
    opts = scenes.Options()
    rast, grads, g2_gpu, g2_ref, grads_ref, ex = _backward_case(sc, cam, opts, seed)
    g2r = {k: g2_ref[k] for k in OB.GRAD2D}
    g2g = {k: g2_gpu[i] for i, k in enumerate(OB.GRAD2D)}
    _assert_grads(g2g, g2r, ex, "2D")
    _assert_grads(raster.to_scene_layout({k: grads[k].cpu().numpy() for k in FIELDS}), grads_ref, ex, "raw")


def test_backward_sh3_form():
    sc = scenes.sh3_scene(3000, 23, n_clusters=20)
    cam = scenes.config1_camera(96, 64)
    rast, grads, g2_gpu, g2_ref, grads_ref, ex = _backward_case(sc, cam, scenes.Options(), 23)
    _assert_grads(raster.to_scene_layout({k: grads[k].cpu().numpy() for k in FIELDS}), grads_ref, ex, "raw")


@pytest.mark.parametrize("tw,th,batch,ppt_bwd", [(32, 8, 512, 4), (16, 16, 256, 1),
                                                 (16, 16, 64, 2), (8, 8, 128, 1)])
def test_backward_other_tile_shape_and_batch(tw, th, batch, ppt_bwd):
    sc, cam = scenes.small_clustered(4000, 24, 120, 80)
    opts = scenes.Options(tile_w=tw, tile_h=th, batch=batch, ppt_bwd=ppt_bwd)
    rast, grads, g2_gpu, g2_ref, grads_ref, ex = _backward_case(sc, cam, opts, 24)
    _assert_grads(raster.to_scene_layout({k: grads[k].cpu().numpy() for k in FIELDS}), grads_ref, ex, "raw")


def test_l1_kernel_matches_definition():
    sc, cam = scenes.small_clustered(2000, 25, 80, 60)
    cams = [cam, scenes.config1_camera(40, 30)]
    rast, params, out = run_forward(sc, cams, scenes.Options())
    tgt = np.concatenate([scenes.target_image(c.width, c.height, 3 + i).reshape(-1)
                          for i, c in enumerate(cams)])
    loss, grad = rast.l1(out.image, torch.from_numpy(tgt).cuda())
    img = out.image.cpu().numpy().astype(np.float64)
    ref_loss, base = 0.0, 0
    ref_grad = np.zeros_like(img)
    for c in cams:
        m = 3 * c.width * c.height
        l, g = OB.l1_loss(img[base:base + m], tgt[base:base + m])
        ref_loss += l
        ref_grad[base:base + m] = g
        base += m
    assert abs(loss.item() - ref_loss) <= 1e-9 * max(1.0, ref_loss)
    assert np.allclose(grad.cpu().numpy(), ref_grad, rtol=1e-6, atol=0)


def test_autograd_function_equals_explicit_backward():
    sc, cam = scenes.small_clustered(2000, 26, 64, 48)
    opts = scenes.Options()
    rast = raster.Rasterizer.for_scene(sc, [cam], opts)
    params = raster.params_to_device(sc)
    leaves = {k: v.clone().requires_grad_(True) for k, v in params.items()}
    image, depth, T, n = raster.render(rast, leaves)
    w = torch.linspace(-1, 1, image.numel(), device=image.device)
    (image * w).sum().backward()
    out = rast.forward(params)
    grads = rast.backward(params, out, w.contiguous())
    for k in FIELDS:
        a, b = leaves[k].grad, grads[k]
        assert torch.allclose(a, b, rtol=1e-5, atol=1e-9 * float(b.abs().max() + 1e-30)), k


def test_batched_backward_sums_camera_gradients():
    """Summed L1 over cameras: the gradient of the batched render equals
    the sum of per-camera gradients."""
    sc, _ = scenes.small_clustered(2500, 27, 64, 48)
    cams = scenes.ring_cameras(3, radius=6.0, seed=5, sizes=((72, 48), (48, 64)))
    opts = scenes.Options()
    rast, params, out = run_forward(sc, cams, opts)
    tgt = torch.from_numpy(np.concatenate(
        [scenes.target_image(c.width, c.height, 9 + i).reshape(-1) for i, c in enumerate(cams)])).cuda()
    _, gimg = rast.l1(out.image, tgt)
    gb = rast.backward(params, out, gimg)
    total = {k: torch.zeros_like(v) for k, v in params.items()}
    base = 0
    for i, c in enumerate(cams):
        m = 3 * c.width * c.height
        r1, p1, o1 = run_forward(sc, [c], opts)
        _, g1 = r1.l1(o1.image, tgt[base:base + m].contiguous())
        gs = r1.backward(p1, o1, g1)
        for k in total:
            total[k] += gs[k]
        base += m
    for k in FIELDS:
        a, b = gb[k].double(), total[k].double()
        scale = float(b.abs().max()) + 1e-30
        assert float((a - b).abs().max()) <= 1e-4 * scale, k


def test_depth_and_alpha_gradients_match_oracle():
    """Upstream gradients on the image, the depth and the accumulated alpha
    (1 - T_final): the ten 2D gradients (with the splat depth) and every raw
    parameter gradient against the oracle."""
    sc, cam = scenes.small_clustered(3000, 28, 96, 64)
    opts = scenes.Options()
    rast = raster.Rasterizer.for_scene(sc, [cam], opts)
    params = raster.params_to_device(sc)
    out = rast.forward(params, out=rast.new_outputs(alpha=True))
    torch.cuda.synchronize()
    T = out.final_T.cpu().numpy()
    assert np.array_equal(out.alpha.cpu().numpy(), (np.float32(1.0) - T).astype(np.float32))
    ref = F.render(sc, cam, opts)
    pre = F.preprocess(sc, cam, opts)
    rng = np.random.default_rng(28)
    gimg = rng.normal(size=(3, 64, 96))
    gdep = rng.normal(size=(64, 96)) * 0.1
    galp = rng.normal(size=(64, 96))
    dev = lambda a: torch.from_numpy(a.astype(np.float32).reshape(-1)).cuda()
    grads = rast.backward(params, out, dev(gimg), dev(gdep), dev(galp))
    g2_gpu = rast.grad2d().cpu().numpy().astype(np.float64)
    g2_ref = OB.blend_backward(pre, cam, opts, ref.values, ref.ranges, gimg,
                               grad_depth=gdep, grad_alpha=galp)
    ex = _tie_exclusion(pre, ref)
    names = OB.GRAD2D + ("z",)
    _assert_grads({k: g2_gpu[i] for i, k in enumerate(names)}, {k: g2_ref[k] for k in names},
                  ex, "2D+z")
    grads_ref = OB.preprocess_backward(sc, cam, opts, pre, g2_ref)
    _assert_grads(raster.to_scene_layout({k: grads[k].cpu().numpy() for k in FIELDS}), grads_ref,
                  ex, "raw")


def test_autograd_depth_and_alpha_equal_explicit_backward():
    sc, cam = scenes.small_clustered(2000, 29, 64, 48)
    rast = raster.Rasterizer.for_scene(sc, [cam], scenes.Options())
    params = raster.params_to_device(sc)
    leaves = {k: v.clone().requires_grad_(True) for k, v in params.items()}
    image, depth, alpha, T, n = raster.render_with_alpha(rast, leaves)
    wi = torch.linspace(-1, 1, image.numel(), device=image.device)
    wd = torch.linspace(1, -1, depth.numel(), device=image.device) * 0.1
    wa = torch.cos(torch.arange(alpha.numel(), device=image.device, dtype=torch.float32))
    ((image * wi).sum() + (depth * wd).sum() + (alpha * wa).sum()).backward()
    out = rast.forward(params, out=rast.new_outputs(alpha=True))
    grads = rast.backward(params, out, wi.contiguous(), wd.contiguous(), wa.contiguous())
    for k in FIELDS:
        a, b = leaves[k].grad, grads[k]
        assert torch.allclose(a, b, rtol=1e-5, atol=1e-9 * float(b.abs().max() + 1e-30)), k


def test_two_renders_then_backward_raises():
    """The autograd Function refuses the first render's backward once a
    second forward has overwritten the shared workspace."""
    sc, cam = scenes.small_clustered(500, 30, 48, 32)
    rast = raster.Rasterizer.for_scene(sc, [cam], scenes.Options())
    leaves = {k: v.clone().requires_grad_(True) for k, v in raster.params_to_device(sc).items()}
    img1, *_ = raster.render(rast, leaves)
    img2, *_ = raster.render(rast, leaves)
    with pytest.raises(raster.StaleWorkspaceError):
        img1.sum().backward()
    img2.sum().backward()
