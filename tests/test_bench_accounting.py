"""The benchmark's algorithmic-byte and lane-op accounting (CPU).

The roofline fractions the benchmark reports are only as good as these
per-stage byte counts; each is checked against the traffic of the passes as
they are built (one 3M-Gaussian frame: 646,587 visible items, 29.6M pairs,
6,700 tiles in 134 row strips holding about 4M (strip, item) entries).
"""
import math

import numpy as np

import bench

N, NVIS, P, TILES = 3_000_000, 646_587, 29_641_109, 6_700
STRIPS, E = 134, 4_000_000
FPG_SG = 51             # 11 geometry floats + SH1 (12) + 4 lobes x 7
GEOM = 11


def test_geometry_floats():
    assert bench.GEOM_FLOATS == GEOM


def test_preprocess_bytes():
    fc = FPG_SG - GEOM
    want = N * 4 * GEOM + NVIS * 4 * fc + N * 12 + NVIS * 64
    assert bench.stage_bytes("fwd.preprocess", N, N, NVIS, NVIS, P, TILES, FPG_SG, STRIPS, E, 0) == want
    # every parameter counted: the full record of every Gaussian
    assert bench.stage_bytes_all_params("fwd.preprocess", N, N, NVIS, FPG_SG) == \
        N * 4 * FPG_SG + 4 * N + 64 * NVIS


def test_depth_sort_bytes_follow_the_passes():
    # pass 0: N keys read twice (count, rank), visible (key, item) written
    p0 = 4 * N + 4 * N + 8 * NVIS
    # passes 1-2: keys read (count), (key, item) read and written
    mid = 2 * (4 * NVIS + 8 * NVIS + 8 * NVIS)
    # last: keys read, (key, item) and each item's rectangle read, then
    # item, pair count and rectangle written
    last = 4 * NVIS + 8 * NVIS + 8 * NVIS + 4 * NVIS + 4 * NVIS + 8 * NVIS
    assert bench.stage_bytes("fwd.depth_sort", N, N, NVIS, NVIS, P, TILES, FPG_SG, STRIPS, E, 0) == \
        p0 + mid + last


def test_scan_duplicate_and_tile_sort_bytes():
    # entry counts read twice, each item's rectangle once, offsets written
    assert bench.stage_bytes("fwd.pair_scan", N, N, NVIS, NVIS, P, TILES, FPG_SG, STRIPS, E, 0) == 20 * NVIS
    assert bench.stage_bytes("fwd.duplicate", N, N, NVIS, NVIS, P, TILES, FPG_SG, STRIPS, E, 0) == 16 * NVIS
    # 134 strips (one 8-bit pass, u16 strip keys): the pass reads the items
    # and writes (strip, position) = 6 B per entry; the count reads position
    # and rectangle (12 B), the scatter position, rectangle and item (16 B)
    # per entry, and every pair is written once (4 B)
    want = 16 * NVIS + 6 * E + 12 * E + 16 * E + 4 * P
    assert bench.stage_bytes("fwd.tile_sort", N, N, NVIS, NVIS, P, TILES, FPG_SG, STRIPS, E, 0) == want
    # u32 strip keys beyond 65,536 strips and three passes: each later pass
    # reads the keys, then reads and writes (key, position)
    want32 = 16 * NVIS + 8 * E + 2 * (4 + 16) * E + 12 * E + 16 * E + 4 * P
    assert bench.stage_bytes("fwd.tile_sort", N, N, NVIS, NVIS, P, 10 ** 6, FPG_SG, 100_000, E, 0) \
        == want32


def test_blends_have_no_byte_bound():
    for st in ("fwd.blend", "bwd.blend", "fwd.tile_order"):
        assert bench.stage_bytes(st, N, N, NVIS, NVIS, P, TILES, FPG_SG, STRIPS, E, 0) is None


def test_standard_binning_bytes():
    # scan 8 N, duplicate 16 N_vis + 12 P, LSD sort of 8-bit digits over the
    # low 32 + ceil(log2 tiles) key bits at 8 + 24 bytes per pair and pass,
    # range search 8 P + 8 tiles
    b, passes = bench.standard_binning_bytes(N, NVIS, P, TILES)
    assert passes == math.ceil((32 + 13) / 8) == 6
    assert b == 8 * N + 16 * NVIS + 12 * P + (8 + 24 * 6) * P + 8 * P + 8 * TILES


def test_peaks():
    assert bench.HBM_PEAK_GBS == 8000
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one non-packed lane-op per lane
    assert abs(bench.VALU_PEAK_TOPS - 256 * 4 * 16 * 2.4e9 / 1e12) < 1e-9


def test_ratio_interval_and_summary():
    """The bench's statistics: the ratio of medians with a bootstrap interval
    that contains it and shrinks with more samples; p10 <= median <= p90."""
    import bench
    rng = np.random.default_rng(4)
    den = 1.0 + 0.01 * rng.normal(size=400)
    num = 1.05 * (1.0 + 0.01 * rng.normal(size=400))
    r, (lo, hi) = bench.ratio_ci(num, den)
    assert lo <= r <= hi and 1.03 < r < 1.07
    r2, (lo2, hi2) = bench.ratio_ci(num[:50], den[:50])
    assert hi2 - lo2 > hi - lo
    s = bench.summary(den)
    assert s["p10_ms"] <= s["median_ms"] <= s["p90_ms"] and s["samples"] == 400
