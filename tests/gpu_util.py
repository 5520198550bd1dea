"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and convert its outputs to the oracle's arrays."""
from __future__ import annotations

import sys

import numpy as np
import torch

from paper_2503_05168_amd import GaussianTensors, Renderer, Settings, split_views
from oracle import binning as obin

# A decision whose float64 value lies within this relative distance of its
# threshold may legitimately come out either way in float32: the float32
# alpha carries a relative error of a few 1e-7 (FP32 quadratic form, exp2).
ALPHA_MARGIN = 1e-5
RECT_MARGIN_PX = 1e-3


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(scene, cams, settings: Settings, segments=None, capacity=1 << 20):
    g = GaussianTensors.from_arrays(scene)
    r = Renderer(settings, capacity)
    f = r.render(g, cams, segments)
    torch.cuda.synchronize()
    return f


def splats_np(f, n_tiles=True):
    s = f.splats.cpu().numpy()
    rect_x = s[:, 13].view(np.uint32)
    rect_y = s[:, 14].view(np.uint32)
    out = dict(
        mean2d=s[:, 0:2].astype(np.float64),
        chol=s[:, 2:5].astype(np.float64),
        conic=s[:, 9:12].astype(np.float64),
        opacity=s[:, 5].astype(np.float64),
        rgb=s[:, 6:9].astype(np.float64),
        depth_f32=s[:, 12].copy(),
        rect=np.stack([rect_x & 0xFFFF, rect_y & 0xFFFF, rect_x >> 16, rect_y >> 16],
                      axis=1).astype(np.int64),
    )
    if n_tiles:
        out["n_tiles"] = f.n_tiles.cpu().numpy().astype(np.int64)
    return out


def oracle_binning(sp, cams, tile, n):
    """The oracle's lexicographic order over the GPU's own rects and depths."""
    views = []
    for v, cam in enumerate(cams):
        sl = slice(v * n, (v + 1) * n)
        nt = sp["n_tiles"][sl]
        rect = np.where((nt > 0)[:, None], sp["rect"][sl], 0)
        views.append(dict(rect=rect, n_tiles=nt, depth_f32=np.where(nt > 0, sp["depth_f32"][sl], 0),
                          grid_w=-(-cam.width // tile), grid_h=-(-cam.height // tile)))
    return obin.bin_and_sort(views, n)


def outputs_np(f):
    imgs = [x.cpu().numpy().astype(np.float64) for x in split_views(f.image, f.cams, 3)]
    Ts = [x.cpu().numpy().astype(np.float64) for x in split_views(f.final_T, f.cams, 1)]
    ncs = [x.cpu().numpy().astype(np.int64) for x in split_views(f.n_contrib, f.cams, 1)]
    return imgs, Ts, ncs


def psnr(a, b):
    mse = float(np.mean((a - b) ** 2))
    return float("inf") if mse == 0 else 10 * np.log10(1.0 / mse)
