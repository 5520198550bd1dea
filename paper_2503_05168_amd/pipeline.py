"""Torch-facing wrappers around the C ABI.

PyTorch only provides device memory and the current HIP stream here; every
step of the hot path runs inside libseele.so.  Each ``seele_*`` function has
the name of the C entry point it calls and only marshals arguments.
``Renderer`` chains them into a frame and grows the pair buffer when the
device reports that it was too small.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import torch

from . import _abi as A

SPLAT_FLOATS = 16  # 64-byte seele_splat


@dataclass
class GaussianTensors:
    """Device SoA arrays matching ``seele_gaussians``."""
    means: torch.Tensor           # [3, N] float32
    log_scales: torch.Tensor      # [3, N]
    quats: torch.Tensor           # [4, N] (w, x, y, z)
    opacity_logits: torch.Tensor  # [N]
    sh: torch.Tensor              # [16, 3, N]
    sh_degree: int = 3

    @property
    def n(self) -> int:
        return int(self.opacity_logits.shape[0])

    @classmethod
    def from_arrays(cls, scene, device="cuda") -> "GaussianTensors":
        """From any object with numpy SoA attributes means, log_scales, quats,
        opacity_logits, sh and sh_degree."""
        t = lambda a: torch.as_tensor(a, dtype=torch.float32).contiguous().to(device)
        return cls(t(scene.means), t(scene.log_scales), t(scene.quats), t(scene.opacity_logits),
                   t(scene.sh), int(getattr(scene, "sh_degree", 3)))

    # float32 elements per Gaussian of each attribute array
    PER_GAUSSIAN = (("means", 3), ("log_scales", 3), ("quats", 4), ("opacity_logits", 1),
                    ("sh", 48))

    def check(self, n: int | None = None, name: str = "gaussians") -> "GaussianTensors":
        """Every attribute array holds at least n Gaussians (default: self.n)."""
        n = self.n if n is None else n
        for attr, k in self.PER_GAUSSIAN:
            _need(getattr(self, attr), k * n, torch.float32, f"{name}.{attr}")
        return self

    def struct(self) -> A.seele_gaussians:
        self.check()
        g = A.seele_gaussians()
        g.n = self.n
        g.sh_degree = self.sh_degree
        for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
            ten = getattr(self, name)
            setattr(g, name, ten.data_ptr() if ten.numel() else None)
        return g


@dataclass
class Settings:
    tile: int = 16
    extent: str = "3sigma"         # or "opacity" (Eq. 5)
    mode: str = "plain"            # or "contrib" (Algorithm 1)
    group: tuple = (2, 2)
    lds_batch: int = 0             # 0 = one Gaussian per tile pixel per LDS step
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    lowpass: float = 0.3
    z_near: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)

    def preprocess_opts(self, segments=None):
        o = A.seele_preprocess_opts()
        o.tile = self.tile
        o.extent = {"3sigma": A.SEELE_EXTENT_3SIGMA, "opacity": A.SEELE_EXTENT_OPACITY}[self.extent]
        o.alpha_min, o.lowpass, o.z_near = self.alpha_min, self.lowpass, self.z_near
        keep = None
        if segments:
            b = (ctypes.c_int64 * len(segments))(*[int(s[0]) for s in segments])
            c = (ctypes.c_int64 * len(segments))(*[int(s[1]) for s in segments])
            o.n_segs = len(segments)
            o.seg_begin = ctypes.cast(b, ctypes.POINTER(ctypes.c_int64))
            o.seg_count = ctypes.cast(c, ctypes.POINTER(ctypes.c_int64))
            keep = (b, c)
        else:
            o.n_segs = 0
        return o, keep

    def raster_opts(self):
        o = A.seele_raster_opts()
        o.tile = self.tile
        o.mode = {"plain": A.SEELE_RASTER_PLAIN, "contrib": A.SEELE_RASTER_CONTRIB}[self.mode]
        o.group_w, o.group_h = int(self.group[0]), int(self.group[1])
        o.lds_batch = int(self.lds_batch)
        o.alpha_min, o.alpha_max, o.T_min = self.alpha_min, self.alpha_max, self.T_min
        for i in range(3):
            o.bg[i] = float(self.bg[i])
        return o


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _p(t: torch.Tensor | None):
    return None if t is None or t.numel() == 0 else ctypes.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, numel: int, dtype, name: str) -> torch.Tensor:
    """The library sees plain pointers: check every caller-provided buffer's
    element type, layout and size before handing it over."""
    if t.dtype != dtype or not t.is_contiguous() or t.numel() < numel:
        raise ValueError(f"{name}: need a contiguous {dtype} tensor of at least {numel} elements, "
                         f"got {t.dtype} {tuple(t.shape)} (contiguous={t.is_contiguous()})")
    return t


def total_tiles(cams, tile: int) -> int:
    arr = A.camera_array(cams)
    return int(A.lib().seele_total_tiles(arr, len(cams), tile))


def pixel_count(cams) -> int:
    return sum(int(c.width) * int(c.height) for c in cams)


def seele_preprocess(g: GaussianTensors, cams, settings: Settings, segments=None,
                     splats: torch.Tensor | None = None, n_tiles: torch.Tensor | None = None,
                     stream=None):
    V, n = len(cams), g.n
    dev = g.means.device
    if splats is None:
        splats = torch.empty((V * n, SPLAT_FLOATS), dtype=torch.float32, device=dev)
    if n_tiles is None:
        n_tiles = torch.empty(V * n, dtype=torch.int32, device=dev)
    _need(splats, V * n * SPLAT_FLOATS, torch.float32, "splats")
    _need(n_tiles, V * n, torch.int32, "n_tiles")
    opts, keep = settings.preprocess_opts(segments)
    gs = g.struct()
    st = A.lib().seele_preprocess(ctypes.byref(gs), A.camera_array(cams), V, ctypes.byref(opts),
                                  _p(splats), _p(n_tiles), _stream(stream))
    del keep
    A.check(st, "seele_preprocess")
    return splats, n_tiles


def seele_preprocess_staged(g: GaussianTensors, cams, settings: Settings, capacity: int,
                            workspace: torch.Tensor, segments=None,
                            splats: torch.Tensor | None = None,
                            n_tiles: torch.Tensor | None = None, stream=None):
    """seele_preprocess that also stages the binning input in `workspace` (a
    bin-sort workspace for this capacity) for seele_bin_sort_ex(staged=True)."""
    V, n = len(cams), g.n
    dev = g.means.device
    if splats is None:
        splats = torch.empty((V * n, SPLAT_FLOATS), dtype=torch.float32, device=dev)
    if n_tiles is None:
        n_tiles = torch.empty(V * n, dtype=torch.int32, device=dev)
    ws_bytes = bin_sort_workspace_size(V * n, capacity, total_tiles(cams, settings.tile))
    _need(splats, V * n * SPLAT_FLOATS, torch.float32, "splats")
    _need(n_tiles, V * n, torch.int32, "n_tiles")
    _need(workspace, ws_bytes, torch.uint8, "workspace")
    opts, keep = settings.preprocess_opts(segments)
    gs = g.struct()
    st = A.lib().seele_preprocess_staged(ctypes.byref(gs), A.camera_array(cams), V,
                                         ctypes.byref(opts), _p(splats), _p(n_tiles),
                                         _p(workspace), workspace.numel(), capacity,
                                         _stream(stream))
    del keep
    A.check(st, "seele_preprocess_staged")
    return splats, n_tiles


def seele_bin_sort_ex(splats, n_tiles, n: int, cams, tile: int, capacity: int,
                      workspace: torch.Tensor, ids: torch.Tensor, ranges: torch.Tensor,
                      num_pairs: torch.Tensor, entry_keys: torch.Tensor | None = None,
                      super_lists: bool = False, staged: bool = False, stream=None):
    """seele_bin_sort(_super), optionally from a workspace staged by
    seele_preprocess_staged; every buffer is the caller's."""
    V = len(cams)
    TT = total_tiles(cams, tile)
    nr = total_super_tiles(cams, tile) if super_lists else TT
    _need(workspace, bin_sort_workspace_size(V * n, capacity, TT), torch.uint8, "workspace")
    _need(ids, capacity, torch.int32, "ids")
    _need(ranges, 2 * nr, torch.int32, "ranges")
    _need(num_pairs, 2 if super_lists else 1, torch.int64, "num_pairs")
    if super_lists:
        _need(entry_keys, capacity, torch.int32, "entry_keys")
    if not staged:
        _need(splats, V * n * SPLAT_FLOATS, torch.float32, "splats")
        _need(n_tiles, V * n, torch.int32, "n_tiles")
    flags = (A.SEELE_BIN_SUPER if super_lists else 0) | (A.SEELE_BIN_STAGED if staged else 0)
    st = A.lib().seele_bin_sort_ex(flags, _p(splats), _p(n_tiles), n, A.camera_array(cams), V,
                                   tile, _p(workspace), workspace.numel(),
                                   _p(entry_keys) if super_lists else None, _p(ids), capacity,
                                   _p(ranges), _p(num_pairs), _stream(stream))
    A.check(st, "seele_bin_sort_ex")
    return ids, ranges, num_pairs


def seele_bin_sort_noalloc(splats, n_tiles, n: int, cams, tile: int, capacity: int,
                           ids: torch.Tensor, ranges: torch.Tensor, num_pairs: torch.Tensor,
                           entry_keys: torch.Tensor | None = None, super_lists: bool = False,
                           stream=None):
    """seele_bin_sort(_super) on the library's own per-device scratch array
    (no workspace argument, no allocation); every output buffer is the
    caller's."""
    V = len(cams)
    TT = total_tiles(cams, tile)
    nr = total_super_tiles(cams, tile) if super_lists else TT
    _need(splats, V * n * SPLAT_FLOATS, torch.float32, "splats")
    _need(n_tiles, V * n, torch.int32, "n_tiles")
    _need(ids, capacity, torch.int32, "ids")
    _need(ranges, 2 * nr, torch.int32, "ranges")
    _need(num_pairs, 2 if super_lists else 1, torch.int64, "num_pairs")
    if super_lists:
        _need(entry_keys, capacity, torch.int32, "entry_keys")
    flags = A.SEELE_BIN_SUPER if super_lists else 0
    st = A.lib().seele_bin_sort_noalloc(flags, _p(splats), _p(n_tiles), n, A.camera_array(cams),
                                        V, tile, _p(entry_keys) if super_lists else None,
                                        _p(ids), capacity, _p(ranges), _p(num_pairs),
                                        _stream(stream))
    A.check(st, "seele_bin_sort_noalloc")
    return ids, ranges, num_pairs


def bin_sort_workspace_size(n_records: int, capacity: int, n_tiles_total: int) -> int:
    return int(A.lib().seele_bin_sort_workspace_size(n_records, capacity, n_tiles_total))


def seele_bin_sort(splats, n_tiles, n: int, cams, tile: int, capacity: int,
                   workspace: torch.Tensor | None = None, sorted_ids=None, tile_ranges=None,
                   num_pairs=None, stream=None):
    dev = splats.device
    V = len(cams)
    TT = total_tiles(cams, tile)
    ws_bytes = bin_sort_workspace_size(V * n, capacity, TT)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=dev)
    if sorted_ids is None:
        sorted_ids = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    if tile_ranges is None:
        tile_ranges = torch.empty((TT, 2), dtype=torch.int32, device=dev)
    if num_pairs is None:
        num_pairs = torch.empty(1, dtype=torch.int64, device=dev)
    _need(splats, V * n * SPLAT_FLOATS, torch.float32, "splats")
    _need(n_tiles, V * n, torch.int32, "n_tiles")
    _need(sorted_ids, capacity, torch.int32, "sorted_ids")
    _need(tile_ranges, 2 * TT, torch.int32, "tile_ranges")
    _need(num_pairs, 1, torch.int64, "num_pairs")
    _need(workspace, ws_bytes, torch.uint8, "workspace")
    st = A.lib().seele_bin_sort(_p(splats), _p(n_tiles), n, A.camera_array(cams), V, tile,
                                _p(workspace), workspace.numel(), _p(sorted_ids), capacity,
                                _p(tile_ranges), _p(num_pairs), _stream(stream))
    A.check(st, "seele_bin_sort")
    return sorted_ids, tile_ranges, num_pairs, workspace


def total_super_tiles(cams, tile: int) -> int:
    n = int(A.lib().seele_total_super_tiles(A.camera_array(cams), len(cams), tile))
    if n < 0:
        raise ValueError("bad cameras or tile size")
    return n


def seele_bin_sort_super(splats, n_tiles, n: int, cams, tile: int, capacity: int,
                         workspace: torch.Tensor | None = None, entry_keys=None, entry_ids=None,
                         st_ranges=None, num_pairs=None, stream=None):
    """Super-tile lists: (entry_keys, entry_ids, st_ranges, num_pairs, workspace);
    num_pairs holds [pairs, entries] and capacity bounds the entries."""
    dev = splats.device
    V = len(cams)
    TT = total_tiles(cams, tile)
    NS = total_super_tiles(cams, tile)
    ws_bytes = bin_sort_workspace_size(V * n, capacity, TT)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=dev)
    if entry_keys is None:
        entry_keys = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    if entry_ids is None:
        entry_ids = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    if st_ranges is None:
        st_ranges = torch.empty((NS, 2), dtype=torch.int32, device=dev)
    if num_pairs is None:
        num_pairs = torch.empty(2, dtype=torch.int64, device=dev)
    _need(splats, V * n * SPLAT_FLOATS, torch.float32, "splats")
    _need(n_tiles, V * n, torch.int32, "n_tiles")
    _need(entry_keys, capacity, torch.int32, "entry_keys")
    _need(entry_ids, capacity, torch.int32, "entry_ids")
    _need(st_ranges, 2 * NS, torch.int32, "st_ranges")
    _need(num_pairs, 2, torch.int64, "num_pairs")
    _need(workspace, ws_bytes, torch.uint8, "workspace")
    st = A.lib().seele_bin_sort_super(_p(splats), _p(n_tiles), n, A.camera_array(cams), V, tile,
                                      _p(workspace), workspace.numel(), _p(entry_keys),
                                      _p(entry_ids), capacity, _p(st_ranges), _p(num_pairs),
                                      _stream(stream))
    A.check(st, "seele_bin_sort_super")
    return entry_keys, entry_ids, st_ranges, num_pairs, workspace


def seele_rasterize_fwd_super(splats, entry_keys, entry_ids, st_ranges, cams, settings: Settings,
                              image=None, final_T=None, n_contrib=None, counters=None,
                              stream=None, last_entry=None):
    """Forward over super-tile lists; counters (device [6] int64) selects the
    instrumented kernel; last_entry (device int32, one per pixel), when
    given, receives 1 + the super-list index of each pixel's last blended
    entry (what seele_rasterize_bwd_super takes).  Returns (image, final_T,
    n_contrib)."""
    dev = st_ranges.device
    npix = pixel_count(cams)
    if image is None:
        image = torch.empty(3 * npix, dtype=torch.float32, device=dev)
    if final_T is None:
        final_T = torch.empty(npix, dtype=torch.float32, device=dev)
    if n_contrib is None:
        n_contrib = torch.empty(npix, dtype=torch.int32, device=dev)
    _need(st_ranges, 2 * total_super_tiles(cams, settings.tile), torch.int32, "st_ranges")
    _need(image, 3 * npix, torch.float32, "image")
    _need(final_T, npix, torch.float32, "final_T")
    _need(n_contrib, npix, torch.int32, "n_contrib")
    if counters is not None:
        _need(counters, 6, torch.int64, "counters")
    if last_entry is not None:
        _need(last_entry, npix, torch.int32, "last_entry")
    opts = settings.raster_opts()
    st = A.lib().seele_rasterize_fwd_super(_p(splats), _p(entry_keys), _p(entry_ids),
                                           _p(st_ranges), A.camera_array(cams), len(cams),
                                           ctypes.byref(opts), _p(image), _p(final_T),
                                           _p(n_contrib), _p(last_entry), _p(counters),
                                           _stream(stream))
    A.check(st, "seele_rasterize_fwd_super")
    return image, final_T, n_contrib


def seele_contrib_topk(splats, sorted_ids, tile_ranges, cams, settings: Settings, n: int,
                       k: int = 32, topk_mark=None, contrib_sum=None, stream=None):
    """Offline contribution pass over per-tile lists (plain blend): marks
    every record among some pixel's k largest contributions T alpha and adds
    every blend's T alpha per record.  Marks and sums accumulate into the
    given tensors (zero-initialised when not given).  Returns (mark, sum)."""
    dev = tile_ranges.device
    R = len(cams) * n
    if topk_mark is None:
        topk_mark = torch.zeros(max(R, 1), dtype=torch.uint8, device=dev)
    if contrib_sum is None:
        contrib_sum = torch.zeros(max(R, 1), dtype=torch.float32, device=dev)
    _need(tile_ranges, 2 * total_tiles(cams, settings.tile), torch.int32, "tile_ranges")
    _need(topk_mark, R, torch.uint8, "topk_mark")
    _need(contrib_sum, R, torch.float32, "contrib_sum")
    opts = settings.raster_opts()
    st = A.lib().seele_contrib_topk(_p(splats), _p(sorted_ids), _p(tile_ranges),
                                    A.camera_array(cams), len(cams), n, ctypes.byref(opts), k,
                                    _p(topk_mark), _p(contrib_sum), _stream(stream))
    A.check(st, "seele_contrib_topk")
    return topk_mark, contrib_sum


def seele_rasterize_fwd(splats, sorted_ids, tile_ranges, cams, settings: Settings, image=None,
                        final_T=None, n_contrib=None, stream=None):
    dev = tile_ranges.device
    npix = pixel_count(cams)
    if image is None:
        image = torch.empty(3 * npix, dtype=torch.float32, device=dev)
    if final_T is None:
        final_T = torch.empty(npix, dtype=torch.float32, device=dev)
    if n_contrib is None:
        n_contrib = torch.empty(npix, dtype=torch.int32, device=dev)
    _need(tile_ranges, 2 * total_tiles(cams, settings.tile), torch.int32, "tile_ranges")
    _need(image, 3 * npix, torch.float32, "image")
    _need(final_T, npix, torch.float32, "final_T")
    _need(n_contrib, npix, torch.int32, "n_contrib")
    opts = settings.raster_opts()
    st = A.lib().seele_rasterize_fwd(_p(splats), _p(sorted_ids), _p(tile_ranges),
                                     A.camera_array(cams), len(cams), ctypes.byref(opts),
                                     _p(image), _p(final_T), _p(n_contrib), _stream(stream))
    A.check(st, "seele_rasterize_fwd")
    return image, final_T, n_contrib


QUEUE_ORDERS = {"list": A.SEELE_QUEUE_LIST, "heaviest": A.SEELE_QUEUE_HEAVIEST_FIRST}


def seele_rasterize_fwd_queue(splats, sorted_ids, tile_ranges, cams, settings: Settings,
                              order: str = "heaviest", workspace=None, image=None, final_T=None,
                              n_contrib=None, stream=None):
    """Persistent (view, tile) work-queue form of the forward rasterizer."""
    dev = tile_ranges.device
    npix = pixel_count(cams)
    if image is None:
        image = torch.empty(3 * npix, dtype=torch.float32, device=dev)
    if final_T is None:
        final_T = torch.empty(npix, dtype=torch.float32, device=dev)
    if n_contrib is None:
        n_contrib = torch.empty(npix, dtype=torch.int32, device=dev)
    need = int(A.lib().seele_raster_queue_workspace_size(total_tiles(cams, settings.tile)))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    _need(tile_ranges, 2 * total_tiles(cams, settings.tile), torch.int32, "tile_ranges")
    _need(image, 3 * npix, torch.float32, "image")
    _need(final_T, npix, torch.float32, "final_T")
    _need(n_contrib, npix, torch.int32, "n_contrib")
    opts = settings.raster_opts()
    st = A.lib().seele_rasterize_fwd_queue(_p(splats), _p(sorted_ids), _p(tile_ranges),
                                           A.camera_array(cams), len(cams), ctypes.byref(opts),
                                           QUEUE_ORDERS[order], _p(workspace), workspace.numel(),
                                           _p(image), _p(final_T), _p(n_contrib), _stream(stream))
    A.check(st, "seele_rasterize_fwd_queue")
    return image, final_T, n_contrib, workspace


def seele_rasterize_fwd_counted(splats, sorted_ids, tile_ranges, cams, settings: Settings,
                                counters=None, stream=None):
    """Instrumented forward: same outputs plus the six work counters."""
    dev = tile_ranges.device
    npix = pixel_count(cams)
    image = torch.empty(3 * npix, dtype=torch.float32, device=dev)
    final_T = torch.empty(npix, dtype=torch.float32, device=dev)
    n_contrib = torch.empty(npix, dtype=torch.int32, device=dev)
    if counters is None:
        counters = torch.empty(6, dtype=torch.int64, device=dev)
    _need(counters, 6, torch.int64, "counters")
    _need(tile_ranges, 2 * total_tiles(cams, settings.tile), torch.int32, "tile_ranges")
    _need(image, 3 * npix, torch.float32, "image")
    _need(final_T, npix, torch.float32, "final_T")
    _need(n_contrib, npix, torch.int32, "n_contrib")
    opts = settings.raster_opts()
    st = A.lib().seele_rasterize_fwd_counted(_p(splats), _p(sorted_ids), _p(tile_ranges),
                                             A.camera_array(cams), len(cams), ctypes.byref(opts),
                                             _p(image), _p(final_T), _p(n_contrib), _p(counters),
                                             _stream(stream))
    A.check(st, "seele_rasterize_fwd_counted")
    return image, final_T, n_contrib, counters


def seele_hp_select(centroids, cam, pos_scale: float, beta: float, M: int):
    """Nearest view cluster + its M nearest neighbours (host-only C call)."""
    import numpy as np
    c = np.ascontiguousarray(centroids, dtype=np.float32)
    K = int(c.shape[0])
    buf = (ctypes.c_float * c.size)(*c.ravel().tolist())
    out = (ctypes.c_int32 * (1 + M))()
    cam_s = A.make_camera(cam)
    st = A.lib().seele_hp_select(buf, K, ctypes.byref(cam_s), float(pos_scale), float(beta),
                                 int(M), out)
    A.check(st, "seele_hp_select")
    return list(out)


def seele_hp_segments(layout_begin, layout_count, clusters):
    """Active (begin, count) segments: shared + the chosen clusters' (host-only C call)."""
    K = len(layout_begin) - 1
    lb = (ctypes.c_int64 * (K + 1))(*[int(x) for x in layout_begin])
    lc = (ctypes.c_int64 * (K + 1))(*[int(x) for x in layout_count])
    cl = (ctypes.c_int32 * max(1, len(clusters)))(*[int(x) for x in clusters])
    ob = (ctypes.c_int64 * (1 + len(clusters)))()
    oc = (ctypes.c_int64 * (1 + len(clusters)))()
    no = ctypes.c_int32()
    st = A.lib().seele_hp_segments(lb, lc, K, cl, len(clusters), ob, oc, ctypes.byref(no))
    A.check(st, "seele_hp_segments")
    return [(int(ob[i]), int(oc[i])) for i in range(no.value)]


def seele_rasterize_bwd(g: GaussianTensors, cams, settings: Settings, splats, n_tiles,
                        sorted_ids, tile_ranges, final_T, n_contrib, dL_dimage, segments=None,
                        grad2d=None, grads=None, stream=None, entry_keys=None, last_entry=None):
    """Backward of preprocess + rasterize: returns (grads, grad2d) where grads
    has the layout of the Gaussian arrays and grad2d holds per-record
    dL/d(mean_x, mean_y, conic a, b, c, opacity, r, g, b).  With entry_keys
    the lists are super-tile lists (sorted_ids = entry ids, tile_ranges =
    super-tile ranges) and seele_rasterize_bwd_super runs on the forward's
    last_entry (n_contrib is then not read)."""
    dev = g.means.device
    V, n = len(cams), g.n
    if grad2d is None:
        grad2d = torch.empty((V * n, 9), dtype=torch.float32, device=dev)
    if grads is None:
        grads = GaussianTensors(torch.empty_like(g.means), torch.empty_like(g.log_scales),
                                torch.empty_like(g.quats), torch.empty_like(g.opacity_logits),
                                torch.empty_like(g.sh), g.sh_degree)
    gs = A.seele_gaussian_grads()
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        t = _need(getattr(grads, name), getattr(g, name).numel(), torch.float32, f"grads.{name}")
        setattr(gs, name, t.data_ptr() if t.numel() else None)
    npix = pixel_count(cams)
    _need(splats, V * n * SPLAT_FLOATS, torch.float32, "splats")
    _need(n_tiles, V * n, torch.int32, "n_tiles")
    sup = entry_keys is not None
    if sup and last_entry is None:
        raise ValueError("the super-tile backward needs the forward's last_entry")
    nr = total_super_tiles(cams, settings.tile) if sup else total_tiles(cams, settings.tile)
    _need(tile_ranges, 2 * nr, torch.int32, "tile_ranges")
    _need(final_T, npix, torch.float32, "final_T")
    if sup:
        _need(last_entry, npix, torch.int32, "last_entry")
    else:
        _need(n_contrib, npix, torch.int32, "n_contrib")
    _need(grad2d, V * n * 9, torch.float32, "grad2d")
    popts, keep = settings.preprocess_opts(segments)
    ropts = settings.raster_opts()
    gst = g.struct()
    dL = _need(dL_dimage.contiguous(), 3 * npix, torch.float32, "dL_dimage")
    if sup:
        st = A.lib().seele_rasterize_bwd_super(
            ctypes.byref(gst), A.camera_array(cams), V, ctypes.byref(popts), ctypes.byref(ropts),
            _p(splats), _p(n_tiles), _p(entry_keys), _p(sorted_ids), _p(tile_ranges), _p(final_T),
            _p(last_entry), _p(dL), _p(grad2d), ctypes.byref(gs), _stream(stream))
    else:
        st = A.lib().seele_rasterize_bwd(ctypes.byref(gst), A.camera_array(cams), V,
                                         ctypes.byref(popts), ctypes.byref(ropts), _p(splats),
                                         _p(n_tiles), _p(sorted_ids), _p(tile_ranges),
                                         _p(final_T), _p(n_contrib), _p(dL), _p(grad2d),
                                         ctypes.byref(gs), _stream(stream))
    del keep
    A.check(st, "seele_rasterize_bwd_super" if sup else "seele_rasterize_bwd")
    return grads, grad2d


class SeeleRender(torch.autograd.Function):
    """Differentiable render of several views (fine-tuning, Sec. 3.5): the
    forward runs preprocess -> bin_sort -> rasterize, the backward the
    library's blend and preprocess backward.  Culling, order, alpha skips,
    leader tests and termination are constants of the backward."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, cams, settings, segments,
                renderer, sh_degree):
        g = GaussianTensors(means.detach().contiguous(), log_scales.detach().contiguous(),
                            quats.detach().contiguous(), opacity_logits.detach().contiguous(),
                            sh.detach().contiguous(), sh_degree)
        f = renderer.render(g, cams, segments)
        ctx.save_for_backward(f.splats, f.n_tiles, f.sorted_ids, f.tile_ranges, f.final_T,
                              f.n_contrib)
        ctx.g = g
        ctx.cams, ctx.settings, ctx.segments = cams, settings, segments
        ctx.mark_non_differentiable(f.final_T, f.n_contrib)
        return f.image, f.final_T, f.n_contrib

    @staticmethod
    def backward(ctx, d_image, d_T, d_nc):
        splats, n_tiles, ids, ranges, final_T, n_contrib = ctx.saved_tensors
        if d_image is None:
            d_image = torch.zeros(3 * final_T.numel(), dtype=torch.float32,
                                  device=final_T.device)
        grads, _ = seele_rasterize_bwd(ctx.g, ctx.cams, ctx.settings, splats, n_tiles, ids,
                                       ranges, final_T, n_contrib, d_image, ctx.segments)
        return (grads.means, grads.log_scales, grads.quats, grads.opacity_logits, grads.sh,
                None, None, None, None, None)


def render(means, log_scales, quats, opacity_logits, sh, cams, settings: Settings | None = None,
           segments=None, renderer: "Renderer | None" = None, sh_degree: int = 3):
    """Differentiable render: returns the concatenated per-view [3][H][W] images
    plus final transmittance and contributor counts."""
    settings = settings or Settings()
    renderer = renderer or Renderer(settings)
    return SeeleRender.apply(means, log_scales, quats, opacity_logits, sh, list(cams), settings,
                             segments, renderer, sh_degree)


def split_views(flat: torch.Tensor, cams, channels: int):
    """Per-view [C, H, W] (or [H, W]) views into a concatenated output buffer."""
    out, off = [], 0
    for c in cams:
        k = channels * c.width * c.height
        v = flat[off:off + k]
        out.append(v.view(channels, c.height, c.width) if channels > 1
                   else v.view(c.height, c.width))
        off += k
    return out


@dataclass
class Frame:
    image: torch.Tensor       # concatenated per-view [3][H][W]
    final_T: torch.Tensor
    n_contrib: torch.Tensor
    splats: torch.Tensor
    n_tiles: torch.Tensor
    sorted_ids: torch.Tensor
    tile_ranges: torch.Tensor
    num_pairs: torch.Tensor
    cams: list = field(default_factory=list)
    # super-tile lists (Renderer(lists="super")): sorted_ids holds the entry
    # ids, tile_ranges the super-tile ranges and entry_keys the entry keys;
    # num_entries the entries the frame needs
    entry_keys: torch.Tensor | None = None
    num_entries: torch.Tensor | None = None
    # Renderer(lists="super", last_entry=True): 1 + the super-list index of
    # each pixel's last blended entry (the input of the super-tile backward)
    last_entry: torch.Tensor | None = None

    def images(self):
        return split_views(self.image, self.cams, 3)

    def list_need(self) -> int:
        """Length of the stored lists the frame needs (entries for super-tile
        lists, pairs otherwise): at most the capacity when the frame fit."""
        t = self.num_entries if self.num_entries is not None else self.num_pairs
        return int(t.item())


MAX_PAIRS = (1 << 31) - 1  # list capacity limit of seele_bin_sort (int32 ranges)


class CapacityError(RuntimeError):
    """A frame needs longer lists (pairs, or super-tile entries) than one
    bin_sort call can hold."""


class Renderer:
    """preprocess -> bin_sort -> rasterize for a list of views, reusing buffers.

    The pair capacity grows (x1.5 of the reported need) and the sort is
    repeated when the device reports overflow; ``check=False`` skips that
    host read (the caller then checks ``num_pairs`` itself)."""

    def __init__(self, settings: Settings | None = None, capacity: int = 1 << 20,
                 schedule: str = "grid", lists: str = "tile", last_entry: bool = False):
        """schedule: "grid" (one workgroup per tile), "queue" or "queue_heavy"
        (persistent work queue in list / heaviest-first order).  lists:
        "tile" (per-tile lists) or "super" (super-tile lists, read by each
        tile directly; grid schedule only).  last_entry (super-tile lists):
        frames also carry the per-pixel last-entry indices the super-tile
        backward reads."""
        if lists not in ("tile", "super"):
            raise ValueError(f"unknown list form {lists!r}")
        if lists == "super" and schedule != "grid":
            raise ValueError("super-tile lists run with the grid schedule")
        self.settings = settings or Settings()
        self.capacity = int(capacity)
        self.schedule = schedule
        self.lists = lists
        self.last_entry = bool(last_entry) and lists == "super"
        self._ek = None
        self._ws = None
        self._qws = None

    def render(self, g: GaussianTensors, cams, segments=None, check: bool = True,
               stream=None) -> Frame:
        s = self.settings
        keys = None
        sup = self.lists == "super"
        while True:
            # preprocessing stages the binning input in the workspace, whose
            # layout depends on the capacity: both run again on regrowth
            dev = g.means.device
            V, TT = len(cams), total_tiles(cams, s.tile)
            ws_bytes = bin_sort_workspace_size(V * g.n, self.capacity, TT)
            if self._ws is None or self._ws.numel() < ws_bytes:
                self._ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=dev)
            splats, n_tiles = seele_preprocess_staged(g, cams, s, self.capacity, self._ws,
                                                      segments, stream=stream)
            cap = max(self.capacity, 1)
            keys = torch.empty(cap, dtype=torch.int32, device=dev) if sup else None
            ids = torch.empty(cap, dtype=torch.int32, device=dev)
            ranges = torch.empty((total_super_tiles(cams, s.tile) if sup else TT, 2),
                                 dtype=torch.int32, device=dev)
            npairs = torch.empty(2 if sup else 1, dtype=torch.int64, device=dev)
            seele_bin_sort_ex(splats, n_tiles, g.n, cams, s.tile, self.capacity, self._ws, ids,
                              ranges, npairs, keys, super_lists=sup, staged=True, stream=stream)
            if not check:
                break
            # super-tile lists store entries, per-tile lists pairs
            need = int(npairs[1 if sup else 0].item())
            if need <= self.capacity:
                break
            if need > MAX_PAIRS:
                what = "super-tile entries" if sup else "Gaussian-tile pairs"
                raise CapacityError(f"the frame needs {need} {what}, more than the {MAX_PAIRS} "
                                    f"one call can sort: render fewer views per call")
            self.capacity = min(int(need * 1.5) + 1024, MAX_PAIRS)
        last_e = None
        if self.lists == "super":
            if self.last_entry:
                last_e = torch.empty(pixel_count(cams), dtype=torch.int32, device=splats.device)
            image, final_T, n_contrib = seele_rasterize_fwd_super(splats, keys, ids, ranges, cams,
                                                                  s, stream=stream,
                                                                  last_entry=last_e)
        elif self.schedule == "grid":
            image, final_T, n_contrib = seele_rasterize_fwd(splats, ids, ranges, cams, s,
                                                            stream=stream)
        else:
            order = "heaviest" if self.schedule == "queue_heavy" else "list"
            image, final_T, n_contrib, self._qws = seele_rasterize_fwd_queue(
                splats, ids, ranges, cams, s, order, self._qws, stream=stream)
        return Frame(image, final_T, n_contrib, splats, n_tiles, ids, ranges, npairs[:1],
                     list(cams), keys, npairs[1:] if sup else None, last_e)
