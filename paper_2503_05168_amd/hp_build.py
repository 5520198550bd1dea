"""Offline construction of the view-dependent representation (Sec. 3.3
"Offline Clustering"): sampled camera poses are clustered on (normalised
position, beta * view direction); each cluster's views are rendered and every
pixel's top-k contributors by T alpha are marked (seele_contrib_topk); the
union of all clusters' top contributors becomes the shared Gaussians, every
other Gaussian that blends in some sampled view becomes exclusive to the
cluster where its summed contribution is largest, and Gaussians that never
blend are left out of every segment.  The scene is reordered into
[shared | exclusive_0 | ... | exclusive_{K-1} | unused], the layout the
runtime selection (seele_hp_select, seele_hp_segments) reads.  This module
only orchestrates the library's kernels and host routines.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _abi as A
from .pipeline import (MAX_PAIRS, CapacityError, GaussianTensors, Settings, _need, _p, _stream,
                       seele_bin_sort, seele_contrib_topk, seele_preprocess)


@dataclass
class ViewDependentScene:
    gaussians: GaussianTensors  # reordered: [shared | excl_0 | ... | excl_{K-1} | unused]
    perm: torch.Tensor          # int64 [n]: new position -> original index
    centroids: np.ndarray       # float32 [K, 6]
    seg_begin: np.ndarray       # int64 [1 + K]: shared, then clusters 0..K-1
    seg_count: np.ndarray       # int64 [1 + K]
    pos_scale: float
    beta: float
    labels: np.ndarray          # int32 [n_poses]: cluster of each sampled pose
    # per original Gaussian (device): in some cluster's top-k set; largest
    # per-cluster summed contribution and that cluster (-1: never blended)
    shared: torch.Tensor | None = None
    best_sum: torch.Tensor | None = None
    best_cluster: torch.Tensor | None = None
    stats: dict = field(default_factory=dict)


def seele_hp_pos_scale(cams) -> float:
    """The library's default position normaliser of the pose feature."""
    v = float(A.lib().seele_hp_pos_scale(A.camera_array(cams), len(cams)))
    if not v > 0.0:
        A.check(A.SEELE_ERR_INVALID_ARG, "seele_hp_pos_scale")
    return v


def seele_hp_kmeans(cams, pos_scale: float, beta: float, K: int, iters: int = 100):
    """(centroids float32 [K, 6], labels int32 [len(cams)]); pos_scale <= 0
    lets the library take its default (seele_hp_pos_scale)."""
    cents = np.zeros((K, 6), dtype=np.float32)
    labels = np.zeros(len(cams), dtype=np.int32)
    st = A.lib().seele_hp_kmeans(A.camera_array(cams), len(cams), pos_scale, beta, K, iters,
                                 cents.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                 labels.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    A.check(st, "seele_hp_kmeans")
    return cents, labels


def seele_hp_accumulate(mark, sums, n_views: int, n: int, cluster: int, shared, best_sum,
                        best_cluster, stream=None):
    _need(mark, n_views * n, torch.uint8, "mark")
    _need(sums, n_views * n, torch.float32, "sums")
    _need(shared, n, torch.uint8, "shared")
    _need(best_sum, n, torch.float32, "best_sum")
    _need(best_cluster, n, torch.int32, "best_cluster")
    st = A.lib().seele_hp_accumulate(_p(mark), _p(sums), n_views, n, cluster, _p(shared),
                                     _p(best_sum), _p(best_cluster), _stream(stream))
    A.check(st, "seele_hp_accumulate")


def seele_hp_partition(shared: np.ndarray, best_sum: np.ndarray, best_cluster: np.ndarray,
                       K: int):
    """(perm int64 [n], layout_begin int64 [1 + K], layout_count int64 [1 + K])."""
    n = int(shared.shape[0])
    shared = np.ascontiguousarray(shared, dtype=np.uint8)
    best_sum = np.ascontiguousarray(best_sum, dtype=np.float32)
    best_cluster = np.ascontiguousarray(best_cluster, dtype=np.int32)
    perm = np.zeros(max(n, 1), dtype=np.int64)
    begin = np.zeros(K + 1, dtype=np.int64)
    count = np.zeros(K + 1, dtype=np.int64)
    i64 = ctypes.POINTER(ctypes.c_int64)
    st = A.lib().seele_hp_partition(shared.ctypes.data, best_sum.ctypes.data,
                                    best_cluster.ctypes.data, n, K, perm.ctypes.data_as(i64),
                                    begin.ctypes.data_as(i64), count.ctypes.data_as(i64))
    A.check(st, "seele_hp_partition")
    return perm[:n], begin, count


def seele_gather_gaussians(g: GaussianTensors, perm: torch.Tensor, stream=None) -> GaussianTensors:
    n_out = int(perm.numel())
    out = GaussianTensors(torch.empty((3, n_out), device=g.means.device),
                          torch.empty((3, n_out), device=g.means.device),
                          torch.empty((4, n_out), device=g.means.device),
                          torch.empty((n_out,), device=g.means.device),
                          torch.zeros((16, 3, n_out), device=g.means.device), g.sh_degree)
    dst = A.seele_gaussian_grads()
    out.check(n_out, "gathered")
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        ten = getattr(out, name)
        setattr(dst, name, ten.data_ptr() if ten.numel() else None)
    src = g.struct()
    perm = _need(perm.to(dtype=torch.int64).contiguous(), n_out, torch.int64, "perm")
    st = A.lib().seele_gather_gaussians(ctypes.byref(src), _p(perm), n_out, ctypes.byref(dst),
                                        _stream(stream))
    A.check(st, "seele_gather_gaussians")
    return out


def _sorted_lists(g: GaussianTensors, cams, settings: Settings, capacity: int, ws):
    """Projected splats and per-tile lists of the views (no blending)."""
    splats, n_tiles = seele_preprocess(g, cams, settings)
    while True:
        ids, ranges, npairs, ws = seele_bin_sort(splats, n_tiles, g.n, cams, settings.tile,
                                                 capacity, ws)
        need = int(npairs.item())
        if need <= capacity:
            return splats, ids, ranges, capacity, ws
        if need > MAX_PAIRS:
            raise CapacityError(f"{need} Gaussian-tile pairs: use fewer views per call")
        capacity = min(int(need * 1.5) + 1024, MAX_PAIRS)


def seele_spatial_order(g: GaussianTensors, workspace=None, stream=None):
    """(perm int64 [n] on the device: new position -> original index, workspace)."""
    n = g.n
    dev = g.means.device
    perm = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
    need = A.lib().seele_spatial_order_workspace_size(n)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    src = g.struct()
    st = A.lib().seele_spatial_order(ctypes.byref(src), _p(workspace), workspace.numel(),
                                     _p(perm), _stream(stream))
    A.check(st, "seele_spatial_order")
    return perm[:n], workspace


def spatially_ordered(g: GaussianTensors):
    """(the scene gathered in Morton order of its means, perm)."""
    perm, _ = seele_spatial_order(g)
    return seele_gather_gaussians(g, perm), perm


def build_view_dependent(g: GaussianTensors, poses, n_clusters: int, k: int = 32,
                         beta: float = 1.0, pos_scale: float | None = None,
                         settings: Settings | None = None, iters: int = 100,
                         views_per_call: int = 16) -> ViewDependentScene:
    """The representation of Sec. 3.3 for scene g from the sampled poses.
    pos_scale (the position normalisation) defaults to the largest distance
    of a sampled camera centre from the origin."""
    settings = settings or Settings()
    if g.n == 0:
        raise ValueError("empty scene")
    if settings.mode != "plain":
        raise ValueError("the contribution pass blends in the plain form")
    if pos_scale is None:
        pos_scale = seele_hp_pos_scale(poses)
    cents, labels = seele_hp_kmeans(poses, pos_scale, beta, n_clusters, iters)
    n = g.n
    dev = g.means.device
    shared = torch.zeros(max(n, 1), dtype=torch.uint8, device=dev)
    best_sum = torch.zeros(max(n, 1), dtype=torch.float32, device=dev)
    best_cluster = torch.full((max(n, 1),), -1, dtype=torch.int32, device=dev)
    V = max(1, min(views_per_call, len(poses)))
    mark = torch.empty(V * n, dtype=torch.uint8, device=dev)
    sums = torch.empty(V * n, dtype=torch.float32, device=dev)
    cap, ws = 1 << 22, None
    for c in range(n_clusters):
        cams = [poses[i] for i in np.nonzero(labels == c)[0]]
        if not cams:
            continue
        mark.zero_()
        sums.zero_()
        for s in range(0, len(cams), V):
            chunk = cams[s:s + V]
            splats, ids, ranges, cap, ws = _sorted_lists(g, chunk, settings, cap, ws)
            # view slot v of every chunk maps to the same records v*n + i, so
            # marks and sums accumulate over the cluster's chunks
            seele_contrib_topk(splats, ids, ranges, chunk, settings, n, k,
                               mark[:len(chunk) * n], sums[:len(chunk) * n])
        seele_hp_accumulate(mark, sums, V, n, c, shared, best_sum, best_cluster)
    perm, begin, count = seele_hp_partition(shared[:n].cpu().numpy(), best_sum[:n].cpu().numpy(),
                                            best_cluster[:n].cpu().numpy(), n_clusters)
    perm_d = torch.from_numpy(perm).to(dev)
    g2 = seele_gather_gaussians(g, perm_d)
    used = int(begin[-1] + count[-1])
    stats = dict(n=n, shared=int(count[0]), exclusive=[int(x) for x in count[1:]],
                 unused=n - used, poses=len(poses), k=k)
    return ViewDependentScene(g2, perm_d, cents, begin, count, pos_scale, beta, labels,
                              shared[:n], best_sum[:n], best_cluster[:n], stats)
