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
    parity.assert_grads(parity.compare_grads(gpu, ref, ex), what)


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
    _assert_grads(parity.group_2d(g2g), parity.group_2d(g2r), ex, "2D")
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


def _three_cameras(sizes=((72, 48), (48, 64), (88, 40)), radius=6.0):
    """Three cameras of different sizes on a circle, looking at the origin."""
    import math
    cams = []
    for k, (w, h) in enumerate(sizes):
        th = 2.0 * math.pi * k / len(sizes) + 0.3
        R, t = scenes.look_at((radius * math.cos(th), 0.0, radius * math.sin(th)), (0.0, 0.0, 0.0))
        cams.append(scenes.pinhole(w, h, R, t))
    return cams


@pytest.mark.parametrize("schedule", [1, 2, 3])
def test_batched_backward_matches_oracle(schedule):
    """Three cameras of different sizes in one call: the batched backward of
    the summed per-camera L1 against the oracle's per-camera backward (one
    key space: camera tile bases and camera-offset values), summed over the
    cameras, for both tile schedules."""
    sc, _ = scenes.small_clustered(2500, 27, 64, 48)
    cams = _three_cameras()
    opts = scenes.Options(schedule=schedule)
    rast, params, out = run_forward(sc, cams, opts)
    pres, refs, keys, vals, ranges = F.render_batch(sc, cams, opts)
    gimgs, ex = [], np.zeros(sc.n, bool)
    for i, (c, ref) in enumerate(zip(cams, refs)):
        img, dep, T, n = camera_numpy(out, cams, i)
        rep = parity.compare_image(img, dep, T, n, ref)
        assert rep["bad"] == 0, (i, rep)
        _, gi = OB.l1_loss(ref.image, scenes.target_image(c.width, c.height, 9 + i))
        gimgs.append(gi)
        ex |= _tie_exclusion(pres[i], ref)
    g_dev = torch.from_numpy(np.concatenate([g.astype(np.float32).reshape(-1) for g in gimgs])).cuda()
    grads = rast.backward(params, out, g_dev)
    total = None
    base = 0
    for i, c in enumerate(cams):
        g2 = OB.blend_backward(pres[i], c, opts, vals, ranges, gimgs[i], cam_index=i, tile_base=base)
        raw = OB.preprocess_backward(sc, c, opts, pres[i], g2)
        total = raw if total is None else {k: total[k] + raw[k] for k in total}
        base += pres[i].grid[0] * pres[i].grid[1]
    _assert_grads(raster.to_scene_layout({k: grads[k].cpu().numpy() for k in FIELDS}), total, ex,
                  "batched raw")


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
    _assert_grads(parity.group_2d({k: g2_gpu[i] for i, k in enumerate(names)}),
                  parity.group_2d({k: g2_ref[k] for k in names}),
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


def _oracle_bwd_work(pre, cam, opts, ref, ppt):
    """The backward blend's work counters from the oracle's walk of every
    tile list, back to front from each pixel's n_contrib: thread visits
    (every thread of a tile visits the entries before the tile's largest
    n_contrib), evaluated pairs (entry before the pixel's n_contrib, pixel in
    the rectangle), pairs with alpha >= alpha_min, and wave reductions (a
    wave and an entry that one of the wave's pairs carries).  Also the slack
    a tie-band pixel allows: its list length."""
    W, H = int(cam.width), int(cam.height)
    tw, th = int(opts.tile_w), int(opts.tile_h)
    nt = tw * th // ppt
    GX, GY = pre.grid
    amin, amax = F._f(opts.alpha_min), F._f(opts.alpha_max)
    visited = evaluated = blended = reductions = slack = 0
    for t in range(GX * GY):
        tx, ty = t % GX, t // GX
        lo, hi = ref.ranges[t]
        entries = ref.values[lo:hi].astype(np.int64)
        px, py = F.tile_pixels(tx, ty, opts, W, H)
        n = ref.n_contrib[py, px]
        maxn = int(n.max()) if n.size else 0
        visited += nt * maxn
        # wave of each pixel: thread = (row // ppt) * TW + column
        wave = (((py - ty * th) // ppt) * tw + (px - tx * tw)) // 64
        for j in range(maxn):
            g = entries[j]
            inr = ((px >= pre.rect[0, g]) & (px <= pre.rect[1, g])
                   & (py >= pre.rect[2, g]) & (py <= pre.rect[3, g]) & (j < n))
            a = F._alpha(pre, g, px - pre.u[g], py - pre.v[g], amax)
            carry = inr & (a >= amin)
            evaluated += int(inr.sum())
            blended += int(carry.sum())
            reductions += len(set(wave[carry].tolist()))
        slack += int(ref.flagged[py, px].sum()) * len(entries)
    return visited, evaluated, blended, reductions, slack


@pytest.mark.parametrize("tw,th,ppt", [(16, 16, 4), (32, 8, 2), (8, 8, 1)])
def test_backward_work_counters_match_the_oracle_walk(tw, th, ppt):
    """The counters behind the backward blend's roofline figure
    (render_blend_bwd_work) against the same events along the oracle's
    back-to-front walk, on a ragged image; the pairs that carry a gradient
    are exactly the forward's blended pairs."""
    sc, cam = scenes.small_clustered(6000, 12, 200, 136)
    opts = scenes.Options(tile_w=tw, tile_h=th, ppt_bwd=ppt)
    rast, params, out = run_forward(sc, [cam], opts)
    ref = F.render(sc, cam, opts)
    pre = F.preprocess(sc, cam, opts)
    got = rast.blend_bwd_work(params, out)
    want = _oracle_bwd_work(pre, cam, opts, ref, ppt)
    slack = want[4]
    for name, g, w in zip(("visited", "evaluated", "blended", "reductions"), got, want[:4]):
        assert abs(g - w) <= slack * (tw * th // ppt if name == "visited" else 1), (name, g, w, slack)
    assert want[2] > 0 and want[1] >= want[2] >= want[3] > 0
    assert got[2] == rast.blend_work(params)[2]
