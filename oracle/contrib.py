"""Per-pixel top-k contributors, in float64 (test infrastructure: only the
tests, the smoke check and the benchmark's CPU baseline use the oracle).

Sec. 3.3 "Offline Clustering" keeps, for every pixel of a cluster's views,
the k Gaussians that contribute most to it, the contribution of Gaussian i
being T_i alpha_i (its weight in Eq. 1: the transmittance in front of it
times its alpha), with k = 32.  The blend that produces T_i alpha_i is the
plain form of Eqs. 1-2 exactly as blend.render_tiles defines it (alpha skip,
alpha clamp, termination).  Readings: ties in T_i alpha_i go to the lower
record id; only blended entries contribute (a skipped or terminating entry
has no weight in Eq. 1).

contributions() returns, per pixel, its blended entries (record id, T alpha)
in blend order and the pixel's decision margin (the smallest relative
distance of any alpha / termination decision from its threshold, as in
render_tiles), so that a test can tell which float32 decisions could
legitimately differ.  topk() ranks them.
"""
from __future__ import annotations

import numpy as np

from .blend import ALPHA_THETA, _alpha


def contributions(splats: dict, ranges: np.ndarray, sorted_ids: np.ndarray, width: int,
                  height: int, tile: int, tile_base: int = 0, alpha_min: float = ALPHA_THETA,
                  alpha_max: float = 0.99, T_min: float = 1e-4, tiles=None) -> dict:
    """{(y, x): (ids [int64], weights [float64], margin, final_T)} for every
    pixel of the given local tiles (default: all) of one view."""
    mean2d = np.asarray(splats["mean2d"], dtype=np.float64)
    conic = np.asarray(splats["conic"], dtype=np.float64)
    opac = np.asarray(splats["opacity"], dtype=np.float64)
    grid_w, grid_h = -(-width // tile), -(-height // tile)
    if tiles is None:
        tiles = range(grid_w * grid_h)
    out = {}
    for t in tiles:
        tx, ty = t % grid_w, t // grid_w
        s, e = ranges[tile_base + t]
        ids = sorted_ids[s:e]
        xs = np.arange(tx * tile, min(width, (tx + 1) * tile))
        ys = np.arange(ty * tile, min(height, (ty + 1) * tile))
        X, Y = np.meshgrid(xs, ys)
        X, Y = X.ravel(), Y.ravel()
        px, py = X + 0.5, Y + 0.5
        npx = X.shape[0]
        T = np.ones(npx)
        done = np.zeros(npx, dtype=bool)
        marg = np.full(npx, np.inf)
        got_ids = [[] for _ in range(npx)]
        got_w = [[] for _ in range(npx)]
        for g in ids:
            if done.all():
                break
            alpha, raw = _alpha(px, py, mean2d[g], conic[g], opac[g], alpha_max)
            live = ~done
            m_a = np.minimum(np.abs(alpha - alpha_min) / alpha_min,
                             np.abs(raw - alpha_max) / alpha_max)
            marg = np.where(live, np.minimum(marg, m_a), marg)
            active = live & (alpha >= alpha_min)
            Tn = T * (1.0 - alpha)
            marg = np.where(active, np.minimum(marg, np.abs(Tn - T_min) / T_min), marg)
            stop = active & (Tn < T_min)
            blend = active & ~stop
            done |= stop
            for k in np.nonzero(blend)[0]:
                got_ids[k].append(int(g))
                got_w[k].append(float(T[k] * alpha[k]))
            T = np.where(blend, Tn, T)
        for k in range(npx):
            out[(int(Y[k]), int(X[k]))] = (np.asarray(got_ids[k], dtype=np.int64),
                                           np.asarray(got_w[k], dtype=np.float64),
                                           float(marg[k]), float(T[k]))
    return out


def topk(ids: np.ndarray, w: np.ndarray, k: int) -> np.ndarray:
    """The k entries with the largest weights, equal weights toward the lower
    id, as an id array in rank order."""
    order = np.lexsort((ids, -w))
    return ids[order[:k]]


def marks_and_sums(contrib: dict, k: int, n_records: int, tie_rel: float = 0.0,
                   margin_min: float = 0.0):
    """Union of every pixel's top-k ids as a bool mask over records, and the
    per-record sum of T alpha over pixels.  With tie_rel / margin_min > 0 it
    also returns (stable, possible) masks: `stable` from pixels whose
    decisions are all at least margin_min from their thresholds and whose
    k-th and (k+1)-th weights differ by more than tie_rel relatively;
    `possible` adds, for the other pixels, every entry that could rank in
    their top k under those perturbations."""
    mark = np.zeros(n_records, dtype=bool)
    stable = np.zeros(n_records, dtype=bool)
    possible = np.zeros(n_records, dtype=bool)
    sums = np.zeros(n_records)
    for ids, w, marg, _ in contrib.values():
        if len(ids) == 0:
            continue
        np.add.at(sums, ids, w)
        top = topk(ids, w, k)
        mark[top] = True
        ws = np.sort(w)[::-1]
        tight = len(ws) > k and (ws[k - 1] - ws[k]) <= tie_rel * ws[k - 1]
        if marg >= margin_min and not tight:
            stable[top] = True
            possible[top] = True
        elif marg < margin_min:
            possible[ids] = True  # any blended entry could move into the top k
        else:
            possible[ids[w >= ws[k - 1] * (1.0 - tie_rel)]] = True
    return mark, sums, stable, possible
