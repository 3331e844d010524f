"""Per-tile views of the oracle's binning, for checking frames too large to
sort whole on the host: the sorted list of one tile and the length of every
tile's list, both computed from the oracle's preprocess alone.

A tile's list is every visible Gaussian whose tile rectangle covers it, in
ascending (depth key, Gaussian index) order — what the stable sort of the
(tile << 32 | depth) keys gives that tile.  These helpers are checked against
the oracle's full key sort in test_oracle_sampling.py.
"""
import numpy as np


def tile_list(pre, tile_local, item_base=0):
    """Values (camera * N + g) of the sorted list of local tile `tile_local`."""
    GX, _ = pre.grid
    tx, ty = tile_local % GX, tile_local // GX
    tr = pre.tile_rect
    m = pre.visible & (tr[0] <= tx) & (tr[1] >= tx) & (tr[2] <= ty) & (tr[3] >= ty)
    g = np.nonzero(m)[0]
    order = np.lexsort((g, pre.depth_bits[g]))
    return (item_base + g[order]).astype(np.uint64)


def tile_counts(pre):
    """Length of every local tile's list (row-major), via a 2D difference
    array over the visible Gaussians' tile rectangles."""
    GX, GY = pre.grid
    v = pre.visible
    tr = pre.tile_rect[:, v].astype(np.int64)
    d = np.zeros((GY + 1, GX + 1), np.int64)
    np.add.at(d, (tr[2], tr[0]), 1)
    np.add.at(d, (tr[2], tr[1] + 1), -1)
    np.add.at(d, (tr[3] + 1, tr[0]), -1)
    np.add.at(d, (tr[3] + 1, tr[1] + 1), 1)
    return d.cumsum(0).cumsum(1)[:GY, :GX].reshape(-1)


def sample_tiles(counts, n_random, rng, n_heaviest=8):
    """The heaviest tiles, a random sample, and the first and last tile."""
    heavy = np.argsort(counts, kind="stable")[::-1][:n_heaviest]
    rand = rng.choice(counts.size, size=min(n_random, counts.size), replace=False)
    return sorted(set(heavy.tolist()) | set(rand.tolist()) | {0, counts.size - 1})
