"""The per-tile sampling helpers agree with the oracle's full key sort."""
import numpy as np

from oracle import forward as F
from paper_2501_00342_amd import scenes
from tests.sampling import sample_tiles, tile_counts, tile_list


def test_tile_lists_and_counts_match_the_full_sort():
    sc, _ = scenes.small_clustered(3000, 51, 96, 64)
    cams = scenes.ring_cameras(3, radius=6.0, seed=4, sizes=((96, 64), (64, 48)))
    opts = scenes.Options()
    pres = [F.preprocess(sc, c, opts) for c in cams]
    keys, vals, ntiles = F.emit_pairs(pres)
    keys, vals = F.sort_pairs(keys, vals)
    ranges = F.tile_ranges(keys, ntiles)
    base = 0
    for c, pre in enumerate(pres):
        GX, GY = pre.grid
        cnt = tile_counts(pre)
        assert np.array_equal(cnt, (ranges[base:base + GX * GY, 1] - ranges[base:base + GX * GY, 0]))
        assert cnt.sum() == pre.tiles_touched.sum()
        for t in range(GX * GY):
            a, b = ranges[base + t]
            assert np.array_equal(tile_list(pre, t, c * sc.n), vals[a:b]), (c, t)
        base += GX * GY
    picked = sample_tiles(cnt, 5, np.random.default_rng(0), n_heaviest=3)
    assert int(np.argmax(cnt)) in picked and 0 in picked
