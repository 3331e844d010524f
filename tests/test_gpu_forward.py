"""Forward parity of the HIP path against the FP64 oracle (GPU)."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from oracle import forward as F
from paper_2501_00342_amd import scenes
from tests import parity
from tests.gpu_util import camera_numpy, records_numpy, run_forward

pytestmark = pytest.mark.gpu

K_HALF_LOG2E = 0.5 / math.log(2.0)


def _check_records(rast, pre, n, cam_index=0):
    rec, ints = records_numpy(rast)
    rects = rast.tile_rects().cpu().numpy().view(np.uint64)
    keys = rast.depth_keys().cpu().numpy().view(np.uint32)
    sl = slice(cam_index * n, (cam_index + 1) * n)
    rec, ints, rects, keys = rec[sl], ints[sl], rects[sl], keys[sl]
    tx0 = (rects & 0xFFFF).astype(np.int64)
    tx1 = ((rects >> np.uint64(16)) & np.uint64(0xFFFF)).astype(np.int64)
    ty0 = ((rects >> np.uint64(32)) & np.uint64(0xFFFF)).astype(np.int64)
    ty1 = ((rects >> np.uint64(48)) & np.uint64(0xFFFF)).astype(np.int64)
    vis_gpu = tx1 >= tx0
    # integers decided on the fixed-order float64 key path: bit-exact
    assert np.array_equal(vis_gpu, pre.visible), "culling differs"
    v = pre.visible
    assert np.array_equal(keys[v], pre.depth_bits[v])
    assert np.all(keys[~v] == 0xFFFFFFFF)
    assert np.array_equal(np.stack([tx0, tx1, ty0, ty1])[:, v], pre.tile_rect[:, v])
    px0 = (ints[:, 13] & 0xFFFF).astype(np.int64)
    px1 = (ints[:, 13] >> 16).astype(np.int64)
    py0 = (ints[:, 14] & 0xFFFF).astype(np.int64)
    py1 = (ints[:, 14] >> 16).astype(np.int64)
    assert np.array_equal(np.stack([px0, px1, py0, py1])[:, v], pre.rect[:, v])
    assert np.array_equal(ints[v, 15].astype(np.int64), pre.radius[v])
    # float fields
    u = rec[v, 0].astype(np.float64) + rec[v, 2].astype(np.float64)
    vv = rec[v, 1].astype(np.float64) + rec[v, 3].astype(np.float64)
    assert np.abs(u - pre.u[v]).max() < 1e-9 * max(1.0, np.abs(pre.u[v]).max())
    assert np.abs(vv - pre.v[v]).max() < 1e-9 * max(1.0, np.abs(pre.v[v]).max())
    assert np.allclose(rec[v, 8], pre.opacity[v], rtol=1e-6, atol=1e-7)
    assert np.abs(rec[v, 9:12].T - pre.rgb[:, v]).max() < 2e-6   # float32 colour
    assert np.allclose(rec[v, 12], pre.z[v], rtol=1e-7)
    # whitening reproduces the conic: Q = (w1 w1^T + w2 w2^T) / k
    w1 = rec[v, 4:6].astype(np.float64)
    w2 = rec[v, 6:8].astype(np.float64)
    Qa = (w1[:, 0] ** 2 + w2[:, 0] ** 2) / K_HALF_LOG2E
    Qb = (w1[:, 0] * w1[:, 1] + w2[:, 0] * w2[:, 1]) / K_HALF_LOG2E
    Qc = (w1[:, 1] ** 2 + w2[:, 1] ** 2) / K_HALF_LOG2E
    scale = np.maximum(np.abs(pre.conic[0, v]), np.abs(pre.conic[2, v]))
    for got, ref in ((Qa, pre.conic[0, v]), (Qb, pre.conic[1, v]), (Qc, pre.conic[2, v])):
        assert np.all(np.abs(got - ref) <= 1e-5 * scale)


def _check_pairs(rast, ref, ntiles):
    bits, P = rast.status()
    assert bits == 0
    assert P == ref.keys.size
    keys = rast.sorted_keys(P).cpu().numpy().view(np.uint64)
    assert np.array_equal(keys, ref.keys), "sorted keys differ"
    vals = rast.pair_values(P).cpu().numpy().view(np.uint32).astype(np.uint64)
    assert np.array_equal(vals, ref.values), "sorted values differ"
    rng = rast.ranges().cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(rng, ref.ranges[:ntiles]), "tile ranges differ"


def test_config0_records_pairs_and_image():
    sc, cams, opts = scenes.workload("sg-1k-128")
    rast, params, out = run_forward(sc, cams, opts)
    pre = F.preprocess(sc, cams[0], opts)
    ref = F.render(sc, cams[0], opts)
    _check_records(rast, pre, sc.n)
    _check_pairs(rast, ref, pre.grid[0] * pre.grid[1])
    img, dep, T, n = camera_numpy(out, cams)
    rep = parity.compare_image(img, dep, T, n, ref)
    assert not rep["failures"], rep


@pytest.mark.parametrize("tw,th,batch,ppt", [(16, 16, 0, 1), (16, 16, 0, 2), (16, 16, 128, 4),
                                             (8, 8, 64, 1), (32, 8, 512, 4), (16, 8, 256, 2),
                                             (8, 16, 128, 1)])
def test_clustered_scene_tile_shapes(tw, th, batch, ppt):
    """A few thousand clustered Gaussians (SH1 + 4 lobes) over a ragged
    200x136 image: many tiles, partial edge tiles, deep lists."""
    sc, cam = scenes.small_clustered(6000, 11, 200, 136)
    opts = scenes.Options(tile_w=tw, tile_h=th, batch=batch, ppt=ppt)
    rast, params, out = run_forward(sc, [cam], opts)
    ref = F.render(sc, cam, opts)
    pre = F.preprocess(sc, cam, opts)
    _check_records(rast, pre, sc.n)
    _check_pairs(rast, ref, pre.grid[0] * pre.grid[1])
    img, dep, T, n = camera_numpy(out, [cam])
    rep = parity.compare_image(img, dep, T, n, ref)
    assert not rep["failures"], rep


def test_sh3_form_parity():
    sc = scenes.sh3_scene(4000, 12, n_clusters=20)
    cam = scenes.config1_camera(160, 120)
    opts = scenes.Options()
    rast, params, out = run_forward(sc, [cam], opts)
    ref = F.render(sc, cam, opts)
    pre = F.preprocess(sc, cam, opts)
    _check_records(rast, pre, sc.n)
    img, dep, T, n = camera_numpy(out, [cam])
    rep = parity.compare_image(img, dep, T, n, ref)
    assert not rep["failures"], rep


def test_forward_is_deterministic():
    sc, cam = scenes.small_clustered(5000, 13, 180, 120)
    opts = scenes.Options()
    rast, params, out1 = run_forward(sc, [cam], opts)
    out2 = rast.forward(params)
    for a, b in zip((out1.image, out1.depth, out1.final_T, out1.n_contrib),
                    (out2.image, out2.depth, out2.final_T, out2.n_contrib)):
        assert bool((a == b).all())


def test_empty_scene_renders_background():
    sc = scenes.config0_scene(0, 5).subset(np.arange(0))
    cam = scenes.config0_camera(40, 30)
    cam.bg = np.array([0.2, 0.4, 0.6], np.float32)
    rast, params, out = run_forward(sc, [cam], scenes.Options())
    img, dep, T, n = camera_numpy(out, [cam])
    assert np.all(img == cam.bg.astype(np.float64)[:, None, None])
    assert np.all(T == 1.0) and np.all(n == 0) and np.all(dep == 0)


def test_all_culled_and_nonfinite_inputs():
    sc = scenes.config0_scene(0, 64)
    sc.means[2, :32] = -10.0            # behind the camera
    sc.quats[0, 32:40] = np.nan          # non-finite -> culled
    sc.sg_amplitudes[0, 0, 40:48] = np.inf
    cam = scenes.config0_camera(64, 64)
    opts = scenes.Options()
    rast, params, out = run_forward(sc, [cam], opts)
    pre = F.preprocess(sc, cam, opts)
    assert not pre.visible[:48].any()
    _check_records(rast, pre, sc.n)
    ref = F.render(sc, cam, opts)
    img, dep, T, n = camera_numpy(out, [cam])
    rep = parity.compare_image(img, dep, T, n, ref)
    assert not rep["failures"], rep


def test_batched_cameras_equal_single_renders():
    sc, _ = scenes.small_clustered(3000, 14, 64, 48)
    cams = scenes.ring_cameras(5, radius=6.0, seed=3, sizes=((96, 64), (64, 80), (130, 70)))
    opts = scenes.Options()
    rast, params, out = run_forward(sc, cams, opts)
    pres, outs, keys, vals, ranges = F.render_batch(sc, cams, opts)
    bits, P = rast.status()
    assert bits == 0 and P == keys.size
    gk = rast.sorted_keys(P).cpu().numpy().view(np.uint64)
    assert np.array_equal(gk, keys)
    for k, cam in enumerate(cams):
        _check_records(rast, pres[k], sc.n, cam_index=k)
        img, dep, T, n = camera_numpy(out, cams, k)
        single_r, _, single_o = run_forward(sc, [cam], opts)
        simg, sdep, sT, sn = camera_numpy(single_o, [cam])
        assert np.array_equal(img, simg) and np.array_equal(n, sn) and np.array_equal(T, sT)
        rep = parity.compare_image(img, dep, T, n, outs[k])
        assert not rep["failures"], (k, rep)


@pytest.mark.parametrize("sched,ppt,ppt_bwd", [(2, 2, 4), (3, 2, 4), (3, 1, 2), (3, 4, 1)])
def test_queue_schedule_equals_grid_schedule(sched, ppt, ppt_bwd):
    """The heavy-first tile queue and its one-wave slice variant render the
    same pixels as one workgroup per tile (bit for bit) and the same
    gradients up to atomic summation order."""
    import torch
    sc, _ = scenes.small_clustered(20000, 41, 200, 140)
    cams = scenes.ring_cameras(3, radius=6.0, seed=8, sizes=((200, 140), (96, 64)))
    res = {}
    for sc_id in (1, sched):
        opts = scenes.Options(schedule=sc_id, ppt=ppt, ppt_bwd=ppt_bwd)
        rast, params, out = run_forward(sc, cams, opts)
        tgt = torch.from_numpy(np.concatenate(
            [scenes.target_image(c.width, c.height, 5 + i).reshape(-1) for i, c in enumerate(cams)])).cuda()
        _, gimg = rast.l1(out.image, tgt)
        grads = rast.backward(params, out, gimg)
        res[sc_id] = (out.image.clone(), out.final_T.clone(), out.n_contrib.clone(),
                      {k: v.clone() for k, v in grads.items()})
    (i1, t1, n1, g1), (i2, t2, n2, g2) = res[1], res[sched]
    assert torch.equal(i1, i2) and torch.equal(t1, t2) and torch.equal(n1, n2)
    for k in g1:
        scale = float(g1[k].abs().max()) + 1e-30
        assert float((g1[k] - g2[k]).abs().max()) <= 1e-5 * scale, k


@pytest.mark.parametrize("schedule,n_cams", [(1, 1), (2, 1), (2, 3), (3, 3)])
def test_graph_replay_matches_eager(schedule, n_cams):
    """The whole forward and backward captured in one HIP graph (one camera,
    or three of different sizes on the heavy-first queue): every replay,
    with eager work and synchronisation in between, equals the eager pass."""
    import torch
    from paper_2501_00342_amd import raster
    from tests.test_gpu_backward import _three_cameras
    sc, cam = scenes.small_clustered(5000, 31, 150, 100)
    cams = [cam] if n_cams == 1 else _three_cameras(((150, 100), (96, 128), (120, 72)))
    opts = scenes.Options(schedule=schedule)
    rast, params, out_e = run_forward(sc, cams, opts)
    tgt = torch.from_numpy(np.concatenate(
        [scenes.target_image(c.width, c.height, 4 + i).reshape(-1) for i, c in enumerate(cams)])).cuda()
    _, g_e = rast.l1(out_e.image, tgt)
    grads_e = rast.backward(params, out_e, g_e)
    grads_e = {k: v.clone() for k, v in grads_e.items()}
    img_e = out_e.image.clone()
    T_e = out_e.final_T.clone()
    n_e = out_e.n_contrib.clone()

    out = rast.new_outputs()
    gimg = torch.empty_like(out.image)
    grads = raster.new_grads(params)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):           # warm-up outside capture
        rast.forward(params, out=out, check=False)
    torch.cuda.current_stream().wait_stream(stream)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rast.forward(params, out=out, check=False)
        rast.l1(out.image, tgt, grad_out=gimg)
        rast.backward_into(params, out, gimg, grads)
    other_sc, other_cam = scenes.small_clustered(2000, 32, 64, 48)
    for rep in range(3):
        for t in (out.image, out.final_T, gimg):
            t.fill_(-7.0)
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.image, img_e) and torch.equal(out.final_T, T_e), rep
        assert torch.equal(out.n_contrib, n_e), rep
        for k in grads:
            a, b = grads[k], grads_e[k]
            assert torch.allclose(a, b, rtol=1e-5, atol=1e-7 * float(b.abs().max() + 1e-30)), (rep, k)
        run_forward(other_sc, [other_cam], opts)   # unrelated eager work between replays
        torch.cuda.synchronize()


def test_packed_and_separate_colour_layouts_agree():
    """The colour arrays as one record per Gaussian (shared stride) and as
    four packed arrays give the same image and keys bit for bit, and the same
    gradients up to the order of the backward's float atomics."""
    import torch

    from paper_2501_00342_amd import raster
    sc, cam = scenes.small_clustered(6000, 17, 160, 120)
    opts = scenes.Options()
    res = []
    for packed in (True, False):
        params = raster.params_to_device(sc, packed=packed)
        rast = raster.Rasterizer([cam], opts, sc.n, sc.sh_degree, sc.n_lobes)
        out = rast.forward(params, check=True)
        tgt = torch.from_numpy(scenes.target_image(160, 120, 2).reshape(-1)).cuda()
        _, gimg = rast.l1(out.image, tgt)
        grads = rast.backward(params, out, gimg)
        res.append((out.image.clone(), rast.depth_keys().clone(),
                    {k: v.clone() for k, v in grads.items()}))
    (i1, k1, g1), (i2, k2, g2) = res
    assert torch.equal(i1, i2) and torch.equal(k1, k2)
    for k in g1:
        scale = float(g1[k].abs().max()) + 1e-30
        assert float((g1[k] - g2[k]).abs().max()) <= 1e-5 * scale, k



def _oracle_blend_work(pre, cam, opts, ref, ppt):
    """The blend's work counters from the oracle's walk of every tile list:
    thread visits (a thread owns `ppt` rows of one column and visits an entry
    while one of its pixels still blends), evaluated (pixel, entry) pairs (the
    pixel still blends and lies in the rectangle) and blended pairs (alpha at
    least alpha_min and the pixel not stopped by the entry).  Also the slack a
    tie-band decision allows: the list length of every flagged pixel."""
    W, H = int(cam.width), int(cam.height)
    tw, th = int(opts.tile_w), int(opts.tile_h)
    GX, GY = pre.grid
    amin, amax, tmin = F._f(opts.alpha_min), F._f(opts.alpha_max), F._f(opts.t_min)
    visited = evaluated = blended = slack = 0
    for t in range(GX * GY):
        tx, ty = t % GX, t // GX
        lo, hi = ref.ranges[t]
        entries = ref.values[lo:hi].astype(np.int64)
        px, py = F.tile_pixels(tx, ty, opts, W, H)
        T = np.ones(px.size)
        done = np.zeros(px.size, bool)
        visits = np.full(px.size, len(entries), np.int64)   # entries seen while live
        for j, g in enumerate(entries):
            inr = ((px >= pre.rect[0, g]) & (px <= pre.rect[1, g])
                   & (py >= pre.rect[2, g]) & (py <= pre.rect[3, g]))
            evald = ~done & inr
            a = F._alpha(pre, g, px - pre.u[g], py - pre.v[g], amax)
            take = evald & (a >= amin)
            Tn = T * (1.0 - a)
            stop = take & (Tn < tmin)
            blend = take & ~stop
            evaluated += int(evald.sum())
            blended += int(blend.sum())
            visits[stop] = j + 1
            done |= stop
            T = np.where(blend, Tn, T)
        flagged = ref.flagged[py, px]
        slack += int(flagged.sum()) * len(entries)
        # threads: column lx, rows (r // ppt) * ppt .. + ppt - 1 of the tile
        lx = px - tx * tw
        grp = (py - ty * th) // ppt
        thread_visits = {}
        for x, r, v in zip(lx, grp, visits):
            thread_visits[(x, r)] = max(thread_visits.get((x, r), 0), int(v))
        visited += sum(thread_visits.values())
    return visited, evaluated, blended, slack


@pytest.mark.parametrize("tw,th,ppt", [(16, 16, 2), (32, 8, 4)])
def test_blend_work_counters_match_the_oracle_walk(tw, th, ppt):
    """The counters behind the forward blend's roofline figure
    (render_blend_work) against the same events counted along the oracle's
    walk of the tile lists, on a ragged image."""
    sc, cam = scenes.small_clustered(6000, 11, 200, 136)
    opts = scenes.Options(tile_w=tw, tile_h=th, ppt=ppt)
    rast, params, out = run_forward(sc, [cam], opts)
    ref = F.render(sc, cam, opts)
    pre = F.preprocess(sc, cam, opts)
    got = rast.blend_work(params)
    want = _oracle_blend_work(pre, cam, opts, ref, ppt)
    slack = want[3]
    for name, g, w in zip(("visited", "evaluated", "blended"), got, want[:3]):
        assert abs(g - w) <= slack, (name, g, w, slack)
    assert want[2] > 0 and want[1] >= want[2]


def test_binning_with_two_strip_passes_and_wide_rows():
    """Binning through two strip passes (more than 256 strips: eight cameras
    of 12 tile rows, each row of 130 8x8 tiles split into strips of 64, 64
    and 2 tiles) gives the oracle's sorted keys, values and tile ranges bit
    for bit, and every camera renders as it does alone."""
    sc, _ = scenes.small_clustered(6000, 23, 96, 64)
    cams = scenes.ring_cameras(8, radius=6.0, seed=11, sizes=((1040, 96),))
    opts = scenes.Options(tile_w=8, tile_h=8)
    rast, params, out = run_forward(sc, cams, opts)
    assert rast.n_strips() == 8 * 12 * 3 > 256
    pres = [F.preprocess(sc, c, opts) for c in cams]
    keys, vals, ntiles = F.emit_pairs(pres)
    keys, vals = F.sort_pairs(keys, vals)
    ranges = F.tile_ranges(keys, ntiles)
    bits, P = rast.status()
    assert bits == 0 and P == keys.size
    assert np.array_equal(rast.sorted_keys(P).cpu().numpy().view(np.uint64), keys)
    assert np.array_equal(rast.pair_values(P).cpu().numpy().view(np.uint32).astype(np.uint64), vals)
    rng = rast.ranges().cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(rng, ranges[:ntiles])
    for k in (0, 5):
        img, dep, T, n = camera_numpy(out, cams, k)
        _, _, single_o = run_forward(sc, [cams[k]], opts)
        simg, sdep, sT, sn = camera_numpy(single_o, [cams[k]])
        assert np.array_equal(img, simg) and np.array_equal(n, sn) and np.array_equal(T, sT)


@pytest.mark.gpu
def test_binning_chunks_past_the_stage():
    """Large splats (log-scales raised by log 8, so that most span a good
    part of a 130-tile row) give more than 8,192 pairs per 512-entry chunk
    on average, so some chunk passes through the scatter's 8,192-pair LDS
    stage in several windows.  Keys, values and tile ranges still equal the
    oracle's bit for bit."""
    sc, cam = scenes.small_clustered(20000, 29, 1040, 96)
    sc = dataclasses.replace(sc, log_scales=(sc.log_scales + np.float32(math.log(8.0))).astype(np.float32))
    opts = scenes.Options(tile_w=8, tile_h=8)
    rast, params, out = run_forward(sc, [cam], opts)
    bits, P = rast.status()
    assert bits == 0
    n_chunks = int(rast.header().cpu().numpy()[6])
    assert n_chunks > 0 and P > 8192 * n_chunks   # so the largest chunk holds more than 8,192
    pre = F.preprocess(sc, cam, opts)
    keys, vals, ntiles = F.emit_pairs([pre])
    keys, vals = F.sort_pairs(keys, vals)
    ranges = F.tile_ranges(keys, ntiles)
    assert P == keys.size
    assert np.array_equal(rast.sorted_keys(P).cpu().numpy().view(np.uint64), keys)
    assert np.array_equal(rast.pair_values(P).cpu().numpy().view(np.uint32).astype(np.uint64), vals)
    rng = rast.ranges().cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(rng, ranges[:ntiles])
