"""Front-to-back alpha blending, plain and contribution-aware, in float64.

Plain form (Sec. 3.1, Eqs. 1-2): every pixel walks its tile's depth-ordered
list; for entry j with 2D mean x', conic A = Sigma'^{-1}, opacity o, colour c:
    q = max(0, d^T A d) with d = p - x' (p = pixel centre, +0.5 convention)
    alpha = min(alpha_max, o * exp(-q/2))
    alpha < alpha_theta          -> skip the entry (alpha_theta = 1/255)
    T' = T (1 - alpha) < T_min   -> stop, the entry is not blended
    otherwise C += T alpha c, T = T', last = j + 1.
Output C + T*bg, the final T and last (the 1-based list position of the last
blended entry; 0 if none).  alpha_max = 0.99 and the strict stop rule are
readings: the paper states a termination threshold only.

Contribution-aware form (Sec. 3.4, Algorithm 1): pixels form w_x x w_y groups
aligned to multiples of the group size; the leader is the group's top-left
pixel (the "first pixel" named in the evaluation setup).  For each entry the
leader's alpha is computed (whether or not the leader has stopped); if it is
below alpha_theta the whole group skips the entry, otherwise every pixel of
the group that has not stopped applies the plain per-pixel step (including
its own alpha_theta skip).  Each pixel stops on its own; the group is done
when all its pixels are.

The loops below are the per-entry recurrences, vectorised only across the
independent pixels of one tile.
"""
from __future__ import annotations

import math

import numpy as np

ALPHA_THETA = 1.0 / 255.0


def splats_from_projection(p: dict) -> dict:
    return dict(mean2d=p["mean2d"], conic=p["conic"], opacity=p["opacity"], rgb=p["rgb"])


def _alpha(px, py, mean, conic, o, alpha_max):
    dx = px - mean[0]
    dy = py - mean[1]
    q = conic[0] * dx * dx + 2.0 * conic[1] * dx * dy + conic[2] * dy * dy
    q = np.maximum(q, 0.0)
    raw = o * np.exp(-0.5 * q)
    return np.minimum(alpha_max, raw), raw


def render_tiles(splats: dict, ranges: np.ndarray, sorted_ids: np.ndarray, width: int,
                 height: int, tile: int, tile_base: int = 0, mode: str = "plain",
                 group=(2, 2), bg=(0.0, 0.0, 0.0), alpha_min: float = ALPHA_THETA,
                 alpha_max: float = 0.99, T_min: float = 1e-4, tiles=None,
                 collect_lists: bool = False) -> dict:
    """Render the given local tiles (default: all) of one view."""
    mean2d = np.asarray(splats["mean2d"], dtype=np.float64)
    conic = np.asarray(splats["conic"], dtype=np.float64)
    opac = np.asarray(splats["opacity"], dtype=np.float64)
    rgb = np.asarray(splats["rgb"], dtype=np.float64)
    bg = np.asarray(bg, dtype=np.float64)
    grid_w, grid_h = -(-width // tile), -(-height // tile)
    if tiles is None:
        tiles = range(grid_w * grid_h)
    gw, gh = (1, 1) if mode == "plain" else group
    assert tile % gw == 0 and tile % gh == 0

    image = np.zeros((3, height, width))
    final_T = np.ones((height, width))
    n_contrib = np.zeros((height, width), dtype=np.int64)
    margin = np.full((height, width), np.inf)
    lists = {} if collect_lists else None
    cnt = dict(evals=0, blends=0, leader_tests=0, leader_pass=0, pass_evals=0, pairs=0)

    for t in tiles:
        tx, ty = t % grid_w, t // grid_w
        s, e = ranges[tile_base + t]
        ids = sorted_ids[s:e]
        cnt["pairs"] += len(ids)
        xs = np.arange(tx * tile, min(width, (tx + 1) * tile))
        ys = np.arange(ty * tile, min(height, (ty + 1) * tile))
        X, Y = np.meshgrid(xs, ys)
        X, Y = X.ravel(), Y.ravel()
        px, py = X + 0.5, Y + 0.5
        # leader of each pixel's group (top-left pixel), and group labels
        LX, LY = (X // gw) * gw, (Y // gh) * gh
        lpx, lpy = LX + 0.5, LY + 0.5
        glabel = (LY * width + LX)
        _, ginv = np.unique(glabel, return_inverse=True)
        n_groups = ginv.max() + 1 if len(ginv) else 0

        npx = X.shape[0]
        T = np.ones(npx)
        C = np.zeros((npx, 3))
        last = np.zeros(npx, dtype=np.int64)
        done = np.zeros(npx, dtype=bool)
        marg = np.full(npx, np.inf)
        plist = [[] for _ in range(npx)] if collect_lists else None

        for j, g in enumerate(ids):
            if done.all():
                break
            alpha, raw = _alpha(px, py, mean2d[g], conic[g], opac[g], alpha_max)
            live = ~done
            if mode == "plain":
                take = live
                cnt["evals"] += int(live.sum())
            else:
                a0, _ = _alpha(lpx, lpy, mean2d[g], conic[g], opac[g], alpha_max)
                lead_ok = a0 >= alpha_min
                group_live = np.bincount(ginv, weights=live, minlength=n_groups) > 0
                group_ok = np.zeros(n_groups, dtype=bool)
                group_ok[ginv[lead_ok]] = True
                cnt["leader_tests"] += int(group_live.sum())
                cnt["leader_pass"] += int((group_live & group_ok).sum())
                marg = np.where(live, np.minimum(marg, np.abs(a0 - alpha_min) / alpha_min), marg)
                take = live & lead_ok
                cnt["pass_evals"] += int(take.sum())
            m_a = np.minimum(np.abs(alpha - alpha_min) / alpha_min,
                             np.abs(raw - alpha_max) / alpha_max)
            marg = np.where(take, np.minimum(marg, m_a), marg)
            active = take & (alpha >= alpha_min)
            Tn = T * (1.0 - alpha)
            marg = np.where(active, np.minimum(marg, np.abs(Tn - T_min) / T_min), marg)
            stop = active & (Tn < T_min)
            blend = active & ~stop
            done |= stop
            C[blend] += (T[blend] * alpha[blend])[:, None] * rgb[g][None, :]
            T = np.where(blend, Tn, T)
            last = np.where(blend, j + 1, last)
            cnt["blends"] += int(blend.sum())
            if collect_lists:
                for k in np.nonzero(blend)[0]:
                    plist[k].append(j)

        image[:, Y, X] = (C + T[:, None] * bg[None, :]).T
        final_T[Y, X] = T
        n_contrib[Y, X] = last
        margin[Y, X] = marg
        if collect_lists:
            for k in range(npx):
                lists[(int(Y[k]), int(X[k]))] = plist[k]

    return dict(image=image, final_T=final_T, n_contrib=n_contrib, margin=margin,
                counters=cnt, lists=lists)


def render_view(proj: dict, mode: str = "plain", group=(2, 2), bg=(0.0, 0.0, 0.0),
                alpha_min: float = ALPHA_THETA, alpha_max: float = 0.99, T_min: float = 1e-4,
                collect_lists: bool = False, tiles=None) -> dict:
    """Bin, sort and blend one projected view (float64 end to end, with the
    float32 rounding of depth that the sort key defines)."""
    from .binning import bin_and_sort

    n = proj["mean2d"].shape[0]
    b = bin_and_sort([dict(rect=proj["rect"], n_tiles=proj["n_tiles"],
                           depth_f32=proj["depth"].astype(np.float32), grid_w=proj["grid_w"],
                           grid_h=proj["grid_h"])], n)
    out = render_tiles(splats_from_projection(proj), b["ranges"], b["ids"], proj["width"],
                       proj["height"], proj["tile"], 0, mode, group, bg, alpha_min, alpha_max,
                       T_min, tiles=tiles, collect_lists=collect_lists)
    out["binning"] = b
    return out


def brute_force_view(proj: dict, bg=(0.0, 0.0, 0.0), alpha_min: float = ALPHA_THETA,
                     alpha_max: float = 0.99, T_min: float = 1e-4):
    """Per-pixel reference with pure-Python loops: each pixel gathers every
    visible Gaussian whose tile rectangle contains the pixel's tile, sorts
    them by (float32 depth, id) with Python's ``sorted`` and blends them one
    by one.  For tiny scenes only."""
    W, H, tile = proj["width"], proj["height"], proj["tile"]
    rect, vis = proj["rect"], proj["visible"]
    depth32 = proj["depth"].astype(np.float32)
    image = np.zeros((3, H, W))
    final_T = np.ones((H, W))
    n_contrib = np.zeros((H, W), dtype=np.int64)
    cand_all = [int(i) for i in np.nonzero(vis)[0]]
    for y in range(H):
        for x in range(W):
            tx, ty = x // tile, y // tile
            cand = [g for g in cand_all
                    if rect[g, 0] <= tx < rect[g, 2] and rect[g, 1] <= ty < rect[g, 3]]
            cand = sorted(cand, key=lambda g: (float(depth32[g]), g))
            T, C, last = 1.0, [0.0, 0.0, 0.0], 0
            for j, g in enumerate(cand):
                dx = x + 0.5 - proj["mean2d"][g, 0]
                dy = y + 0.5 - proj["mean2d"][g, 1]
                a, b, c = proj["conic"][g]
                q = max(0.0, a * dx * dx + 2 * b * dx * dy + c * dy * dy)
                alpha = min(alpha_max, proj["opacity"][g] * math.exp(-0.5 * q))
                if alpha < alpha_min:
                    continue
                Tn = T * (1.0 - alpha)
                if Tn < T_min:
                    break
                for ch in range(3):
                    C[ch] += T * alpha * proj["rgb"][g, ch]
                T = Tn
                last = j + 1
            for ch in range(3):
                image[ch, y, x] = C[ch] + T * bg[ch]
            final_T[y, x] = T
            n_contrib[y, x] = last
    return dict(image=image, final_T=final_T, n_contrib=n_contrib)
