"""Tile binning and the per-tile depth order (Sec. 3.1 "Preprocessing"
identifies Gaussian-tile intersections; "Sorting" orders each tile's
Gaussians from the closest to the furthest).

Every visible Gaussian g yields one pair per tile of its rectangle.  A pair's
order is the lexicographic order of the integer triple
    (global tile id, bit pattern of float32 depth, record id)
where the record id of Gaussian g in view v is v*N + g, and the global tile
id is the view's tile base plus ty*grid_w + tx.  Depths are positive (they
exceed z_near), so their float32 bit patterns order like the values; the
record id breaks depth ties (a reading: the paper does not say).
"""
from __future__ import annotations

import numpy as np


def depth_bits(depth_f32: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(depth_f32, dtype=np.float32).view(np.uint32).astype(np.int64)


def enumerate_pairs(rect: np.ndarray, n_tiles: np.ndarray, grid_w: int,
                    tile_base: int = 0, id_base: int = 0):
    """All (tile, record id) pairs of one view, Gaussians in id order and
    tiles in row-major order within each rectangle."""
    vis = np.nonzero(n_tiles > 0)[0]
    counts = n_tiles[vis].astype(np.int64)
    total = int(counts.sum())
    ids = np.repeat(vis, counts)
    starts = np.repeat(np.cumsum(counts) - counts, counts)
    k = np.arange(total, dtype=np.int64) - starts
    r = rect[ids]
    w = r[:, 2] - r[:, 0]
    ty = r[:, 1] + k // w
    tx = r[:, 0] + k % w
    tiles = tile_base + ty * grid_w + tx
    return tiles.astype(np.int64), (ids + id_base).astype(np.int64)


def bin_and_sort(views, n_per_view: int):
    """``views``: list of dicts with keys rect, n_tiles, depth_f32, grid_w,
    grid_h (one per view, arrays over the view's N Gaussians).

    Returns sorted record ids, their tile ids, per-tile [start, end) ranges
    over the global tile space, and the view tile bases."""
    tiles_all, ids_all, dbits_all = [], [], []
    base = 0
    bases = []
    for v, pv in enumerate(views):
        bases.append(base)
        t, i = enumerate_pairs(pv["rect"], pv["n_tiles"], pv["grid_w"], base, v * n_per_view)
        tiles_all.append(t)
        ids_all.append(i)
        dbits_all.append(depth_bits(pv["depth_f32"])[i - v * n_per_view])
        base += pv["grid_w"] * pv["grid_h"]
    tiles = np.concatenate(tiles_all) if tiles_all else np.zeros(0, np.int64)
    ids = np.concatenate(ids_all) if ids_all else np.zeros(0, np.int64)
    dbits = np.concatenate(dbits_all) if dbits_all else np.zeros(0, np.int64)
    order = np.lexsort((ids, dbits, tiles))
    st, si = tiles[order], ids[order]
    n_total_tiles = base
    t_idx = np.arange(n_total_tiles)
    ranges = np.stack([np.searchsorted(st, t_idx, side="left"),
                       np.searchsorted(st, t_idx, side="right")], axis=1)
    ranges = np.where((ranges[:, 1] > ranges[:, 0])[:, None], ranges, 0)
    return dict(ids=si, tiles=st, ranges=ranges.astype(np.int64), tile_bases=np.array(bases),
                n_pairs=int(st.shape[0]))
