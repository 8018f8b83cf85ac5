"""Host replay of the load-balanced tile pass's work layout, with bounds
checks (no GPU).

The balanced pass (transpose kernel -> plan kernel -> persistent tile-list
kernel, in csrc/mm_tile.hip) cuts every tile's records into pieces of about
`piece_records` records, lays the pieces out tile by tile (piece_first),
lists them as work items (tile, j << 16 | k), and lets a persistent grid
take items from a counter; item (t, j, k) covers bin workgroups
[num_wg * j / k, num_wg * (j + 1) / k) and writes partial block
piece_first[t] + j. The runtime sizes the item list and the partial blocks
as ceil(N / R) + ntiles (R = piece_records).

This file restates that arithmetic and checks, for the workload whose
instrumented tile-list run once printed nothing until its time limit (2^24
uniform points, 1920 x 1080, tiles of 32 pixels, pieces of 16,384 records,
per-tile counts from the oracle's projection) and for adversarial counts,
that every item, partial block, piece count and workgroup range stays
inside what the runtime allocates, and that the pieces of a tile cover its
workgroups exactly once, so the item loop ends after a finite list.
"""
import math
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def plan(totals: np.ndarray, n_points: int, num_wg: int, R: int):
    """The plan kernel's layout from the tiles' record totals; returns the
    items and piece_first, after checking them against the allocations."""
    nt = totals.size
    assert R * 65535 >= n_points, "the runtime refuses piece sizes this small"
    blocks = (n_points + R - 1) // R + nt            # items and partial blocks allocated
    pieces = (totals + R - 1) // R                   # per tile
    assert pieces.max(initial=0) <= 0xFFFF, "piece count must fit 16 bits"
    piece_first = np.zeros(nt + 1, dtype=np.int64)
    np.cumsum(pieces, out=piece_first[1:])
    n_items = int(piece_first[-1])
    assert n_items <= blocks, (n_items, blocks)
    items = []
    for t in np.flatnonzero(pieces):
        k = int(pieces[t])
        for j in range(k):
            items.append((int(t), (j << 16) | k))
    assert len(items) == n_items
    # the tile-list kernel's view of every item
    covered = {}
    for t, jk in items:
        j, k = jk >> 16, jk & 0xFFFF
        assert 0 <= j < k
        w_lo = num_wg * j // k
        w_hi = num_wg * (j + 1) // k
        assert 0 <= w_lo <= w_hi <= num_wg
        part = int(piece_first[t]) + j
        assert 0 <= part < blocks, (part, blocks)
        covered.setdefault(t, []).append((w_lo, w_hi))
    for t, ranges in covered.items():  # a tile's pieces cover [0, num_wg) once
        ranges.sort()
        assert ranges[0][0] == 0 and ranges[-1][1] == num_wg
        assert all(a[1] == b[0] for a, b in zip(ranges, ranges[1:]))
    return items, piece_first, blocks


def tile_totals(pixels: np.ndarray, width: int, height: int, side: int) -> np.ndarray:
    tiles_x = (width + side - 1) // side
    tiles_y = (height + side - 1) // side
    on = pixels[pixels >= 0]
    t = (on // width // side) * tiles_x + (on % width) // side
    return np.bincount(t, minlength=tiles_x * tiles_y).astype(np.int64)


@pytest.mark.slow
def test_replay_of_the_2p24_1080p_16384_record_case():
    n, w, h, side, R = 1 << 24, 1920, 1080, 32, 16384
    P = 1024 * 8                                     # bin workgroups of 1024 threads x 8 points
    num_wg = (n + P - 1) // P
    pts = synth.uniform_cube(n, 0)
    pix = oracle.project_many(pts, synth.orbit_camera(0, w, h), w, h)
    totals = tile_totals(pix, w, h, side)
    assert totals.sum() == np.count_nonzero(pix >= 0)
    items, piece_first, blocks = plan(totals, n, num_wg, R)
    active = int(np.count_nonzero(totals))
    # about 1,000 pieces over some 260 active tiles; the list is finite, so a
    # grid that takes items from a counter until it passes the list ends
    assert 200 <= active <= 400
    assert len(items) <= blocks <= n // R + 1 + totals.size
    # (an instrumented copy that stored 10 words per piece at g_dbg[piece * 10]
    # needed room for 10 * len(items) words; the product stores none)


@pytest.mark.parametrize("case", ["one-pixel", "one-tile-row", "uniform-screen", "4k-mixture-2p28"])
def test_replay_of_adversarial_tile_counts(case):
    rng = np.random.default_rng(3)
    if case == "one-pixel":              # every point in one tile: the most pieces per tile
        n, w, h, side, R = 1 << 24, 1920, 1080, 32, 16384
        totals = np.zeros(((w + side - 1) // side) * ((h + side - 1) // side), np.int64)
        totals[777] = n
    elif case == "one-tile-row":
        n, w, h, side, R = 1 << 22, 3840, 2160, 64, 4096
        tx = (w + side - 1) // side
        totals = np.zeros(tx * ((h + side - 1) // side), np.int64)
        totals[:tx] = np.diff(np.sort(rng.integers(0, n, tx - 1)), prepend=0, append=n)
    elif case == "uniform-screen":
        n, w, h, side, R = 1 << 26, 1920, 1080, 16, 1 << 16
        nt = ((w + side - 1) // side) * ((h + side - 1) // side)
        totals = rng.multinomial(n, np.full(nt, 1.0 / nt)).astype(np.int64)
    else:                                # the 4K balanced default: R = N / 1024
        n, w, h, side = 1 << 28, 3840, 2160, 64
        R = (n // 1024 + 1023) // 1024 * 1024
        nt = ((w + side - 1) // side) * ((h + side - 1) // side)
        weights = rng.gamma(0.3, size=nt)
        totals = rng.multinomial(n, weights / weights.sum()).astype(np.int64)
    P = 1024 * 8
    plan(totals, n, math.ceil(n / P), R)
