"""Scene prefetching (Sec. 3.3 "Scene Prefetching") over the view-dependent
representation: the device holds the shared segment plus a fixed number of
cluster slots; each frame's selected clusters must be resident before its
preprocessing reads them, and the clusters selected at the pose predicted by
linear extrapolation are copied ahead of time from pinned host memory on a
dedicated copy stream, overlapping the frame's rendering.  Planning
(seele_resident_plan), pose prediction (seele_pose_extrapolate) and the
copies (seele_load_segments) are library calls; this module keeps the slot
table and the stream ordering:
  - a load into a slot waits (on the copy stream) for the last frame that
    read the slot's previous cluster;
  - a frame waits (on its stream) for the loads of the slots it reads.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _abi as A
from .pipeline import (GaussianTensors, Renderer, Settings, _stream, seele_hp_select)

ROWS = 3 + 3 + 4 + 1 + 48  # means, log-scales, quaternion, opacity logit, SH (16 x 3)


@dataclass
class CameraPose:
    R: np.ndarray
    t: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int


def seele_pose_extrapolate(prev, cur, s: float = 1.0) -> CameraPose:
    out = A.seele_camera()
    st = A.lib().seele_pose_extrapolate(ctypes.byref(A.make_camera(prev)),
                                        ctypes.byref(A.make_camera(cur)), float(s),
                                        ctypes.byref(out))
    A.check(st, "seele_pose_extrapolate")
    return CameraPose(np.array(out.R[:], dtype=np.float32).reshape(3, 3),
                      np.array(out.t[:], dtype=np.float32), out.fx, out.fy, out.cx, out.cy,
                      out.width, out.height)


def seele_resident_plan(slot_cluster: np.ndarray, slot_stamp: np.ndarray,
                        cluster_count: np.ndarray, slot_cap: int, need, want, frame: int):
    """Updates slot_cluster (int32) / slot_stamp (int64) in place; returns
    (loads [(cluster, slot)], number of demand loads)."""
    S = int(slot_cluster.shape[0])
    assert slot_cluster.dtype == np.int32 and slot_stamp.dtype == np.int64
    cc = np.ascontiguousarray(cluster_count, dtype=np.int64)
    nd = np.ascontiguousarray(need, dtype=np.int32)
    wt = np.ascontiguousarray(want, dtype=np.int32)
    lc = np.zeros(S, dtype=np.int32)
    ls = np.zeros(S, dtype=np.int32)
    n_loads, n_demand = ctypes.c_int32(), ctypes.c_int32()
    st = A.lib().seele_resident_plan(slot_cluster.ctypes.data, slot_stamp.ctypes.data, S,
                                     cc.ctypes.data, int(cc.shape[0]), int(slot_cap),
                                     nd.ctypes.data if nd.size else None, int(nd.size),
                                     wt.ctypes.data if wt.size else None, int(wt.size), int(frame),
                                     lc.ctypes.data, ls.ctypes.data, ctypes.byref(n_loads),
                                     ctypes.byref(n_demand))
    A.check(st, "seele_resident_plan")
    k = n_loads.value
    return [(int(lc[i]), int(ls[i])) for i in range(k)], n_demand.value


def seele_load_segments(host: torch.Tensor, pool: torch.Tensor, src_begin, dst_begin, count,
                        stream=None):
    """Copies columns of a pinned host table [rows][n] into a device table
    [rows][n_pool] (see seele.h)."""
    assert host.dim() == 2 and pool.dim() == 2 and host.shape[0] == pool.shape[0]
    assert host.is_pinned() and host.dtype == torch.float32 and pool.dtype == torch.float32
    sb = np.ascontiguousarray(src_begin, dtype=np.int64)
    db = np.ascontiguousarray(dst_begin, dtype=np.int64)
    ct = np.ascontiguousarray(count, dtype=np.int64)
    st = A.lib().seele_load_segments(host.data_ptr(), int(host.shape[1]), pool.data_ptr(),
                                     int(pool.shape[1]), int(host.shape[0]), sb.ctypes.data,
                                     db.ctypes.data, ct.ctypes.data, int(sb.size), _stream(stream))
    A.check(st, "seele_load_segments")


def pack_rows(g: GaussianTensors, out: torch.Tensor) -> torch.Tensor:
    """The [ROWS][n] attribute table of a scene (means, log-scales,
    quaternion, opacity logit, SH rows)."""
    n = g.n
    out[0:3].copy_(g.means)
    out[3:6].copy_(g.log_scales)
    out[6:10].copy_(g.quats)
    out[10].copy_(g.opacity_logits)
    out[11:].copy_(g.sh.reshape(48, n))
    return out


def table_gaussians(table: torch.Tensor, sh_degree: int) -> GaussianTensors:
    """GaussianTensors viewing the rows of a [ROWS][n] device table."""
    n = int(table.shape[1])
    return GaussianTensors(table[0:3], table[3:6], table[6:10], table[10], table[11:].view(16, 3, n),
                           sh_degree)


class PrefetchingRenderer:
    """Renders poses of a view-dependent scene with only the shared segment
    and `n_slots` cluster slots resident, prefetching the clusters selected
    at the extrapolated pose (`lookahead` frames ahead; None disables
    prediction, leaving demand loads only).  preload=True (needs n_slots >=
    the cluster count) loads every cluster into its own slot up front: the
    all-resident configuration on the same code path."""

    def __init__(self, vd, settings: Settings | None = None, M: int = 3, n_slots: int = 8,
                 lookahead: float | None = 1.0, capacity: int = 1 << 22, lists: str = "super",
                 preload: bool = False, host: torch.Tensor | None = None):
        self.vd = vd
        self.M = int(M)
        self.lookahead = lookahead
        K = len(vd.seg_begin) - 1
        self.K = K
        self.counts = np.asarray(vd.seg_count[1:], dtype=np.int64)
        self.begins = np.asarray(vd.seg_begin[1:], dtype=np.int64)
        self.n_shared = int(vd.seg_count[0])
        assert int(vd.seg_begin[0]) == 0
        self.slot_cap = int(self.counts.max()) if K else 0
        self.S = int(n_slots)
        if self.S < 1 + self.M:
            raise ValueError("need at least 1 + M slots")
        g = vd.gaussians
        n = g.n
        dev = g.means.device
        if host is None:  # the scene's attribute table in pinned host memory
            host = torch.empty((ROWS, n), dtype=torch.float32, pin_memory=True)
            host.copy_(pack_rows(g, torch.empty((ROWS, n), dtype=torch.float32, device=dev)))
        assert host.shape == (ROWS, n) and host.is_pinned()
        self.host = host
        self.n_pool = self.n_shared + self.S * self.slot_cap
        # only loaded columns are ever read (segments cover loaded clusters)
        self.pool = torch.empty((ROWS, max(self.n_pool, 1)), dtype=torch.float32, device=dev)
        self.copy_stream = torch.cuda.Stream(device=dev)
        # the copies follow everything already queued on the caller's stream
        self.copy_stream.wait_stream(torch.cuda.current_stream(dev))
        if self.n_shared:
            seele_load_segments(self.host, self.pool, [0], [0], [self.n_shared], self.copy_stream)
        self.g = table_gaussians(self.pool, g.sh_degree)
        self.slot_cluster = np.full(self.S, -1, dtype=np.int32)
        self.slot_stamp = np.zeros(self.S, dtype=np.int64)
        if preload:
            if self.S < K:
                raise ValueError("preloading needs a slot per cluster")
            seele_load_segments(self.host, self.pool, self.begins,
                                self.n_shared + np.arange(K, dtype=np.int64) * self.slot_cap,
                                self.counts, self.copy_stream)
            self.slot_cluster[:K] = np.arange(K, dtype=np.int32)
        self.copy_stream.synchronize()
        self.ready = [None] * self.S
        self.free = [None] * self.S
        self.renderer = Renderer(settings or Settings(), capacity=capacity, lists=lists)
        self.prev = None
        self.frame = 0
        self.stats = dict(frames=0, loads=0, demand_loads=0, bytes_loaded=0)

    @property
    def resident_bytes(self) -> int:
        return ROWS * 4 * self.n_pool

    def segments(self, clusters):
        slot = {int(c): int(s) for s, c in enumerate(self.slot_cluster) if c >= 0}
        segs = [(0, self.n_shared)] if self.n_shared else []
        for c in sorted(set(int(c) for c in clusters)):
            if self.counts[c]:
                segs.append((self.n_shared + slot[c] * self.slot_cap, int(self.counts[c])))
        return sorted(segs)

    def _load(self, loads):
        for c, s in loads:
            if self.free[s] is not None:
                self.copy_stream.wait_event(self.free[s])
            seele_load_segments(self.host, self.pool, [self.begins[c]],
                                [self.n_shared + s * self.slot_cap], [self.counts[c]],
                                self.copy_stream)
            ev = torch.cuda.Event()
            ev.record(self.copy_stream)
            self.ready[s] = ev
            self.stats["bytes_loaded"] += ROWS * 4 * int(self.counts[c])
        self.stats["loads"] += len(loads)

    def render(self, cam, check: bool = True):
        """One frame: demand-load what this pose selects and is missing, render
        it, then plan and enqueue the loads for the predicted pose (the
        prediction and its copies overlap this frame's rendering)."""
        vd = self.vd
        self.frame += 1
        need = seele_hp_select(vd.centroids, cam, vd.pos_scale, vd.beta, self.M)
        loads, n_demand = seele_resident_plan(self.slot_cluster, self.slot_stamp, self.counts,
                                              self.slot_cap, need, [], self.frame)
        self._load(loads)
        self.stats["demand_loads"] += n_demand
        self.stats["frames"] += 1
        compute = torch.cuda.current_stream()
        used = sorted({int(np.nonzero(self.slot_cluster == c)[0][0]) for c in need})
        for s in used:
            if self.ready[s] is not None:
                compute.wait_event(self.ready[s])
        f = self.renderer.render(self.g, [cam], self.segments(need), check=check)
        done = torch.cuda.Event()
        done.record(compute)
        for s in used:
            self.free[s] = done
        if self.lookahead is not None and self.prev is not None:
            pred = seele_pose_extrapolate(self.prev, cam, self.lookahead)
            want = seele_hp_select(vd.centroids, pred, vd.pos_scale, vd.beta, self.M)
            loads, _ = seele_resident_plan(self.slot_cluster, self.slot_stamp, self.counts,
                                           self.slot_cap, need, want, self.frame)
            self._load(loads)
        self.prev = cam
        return f
