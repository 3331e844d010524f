"""The tile-parallel oracle runs are a partition of the sequential ones:
forward results bit for bit, backward sums up to float64 rounding of the
summation order (CPU)."""
import numpy as np

from oracle import backward as OB
from oracle import forward as F
from oracle import parallel as OP
from paper_2501_00342_amd import scenes


def _case():
    sc, cam = scenes.small_clustered(1500, 31, 70, 45)
    opts = scenes.Options(tile_w=16, tile_h=8)
    pre = F.preprocess(sc, cam, opts)
    keys, vals, nt = F.emit_pairs(pre)
    keys, vals = F.sort_pairs(keys, vals)
    return sc, cam, opts, pre, vals, F.tile_ranges(keys, nt)


def test_parallel_forward_equals_sequential():
    sc, cam, opts, pre, vals, ranges = _case()
    seq = F.blend_image(pre, cam, opts, vals, ranges)
    par = OP.blend_image(pre, cam, opts, vals, ranges, n_workers=3)
    for a, b in zip(seq[:5], par[:5]):
        assert np.array_equal(a, b)
    assert seq[5].keys() == par[5].keys()
    assert (seq[3] > 0).sum() > 100


def test_parallel_backward_equals_sequential():
    sc, cam, opts, pre, vals, ranges = _case()
    rng = np.random.default_rng(2)
    gimg = rng.normal(size=(3, cam.height, cam.width))
    gdep = rng.normal(size=(cam.height, cam.width))
    seq = OB.blend_backward(pre, cam, opts, vals, ranges, gimg, grad_depth=gdep)
    par = OP.blend_backward(pre, cam, opts, vals, ranges, gimg, grad_depth=gdep, n_workers=3)
    assert seq.keys() == par.keys()
    for k in seq:
        scale = np.abs(seq[k]).max()
        assert scale > 0, k
        assert np.allclose(par[k], seq[k], rtol=1e-12, atol=1e-13 * scale), k
