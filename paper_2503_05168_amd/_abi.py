"""ctypes mirror of include/seele.h: structs and the raw entry points.

Argument marshalling only -- every computation happens inside libseele.so.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_float, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libseele.so")

SEELE_OK = 0
SEELE_ERR_INVALID_ARG = 1
SEELE_ERR_UNSUPPORTED = 2
SEELE_ERR_CAPACITY = 3
SEELE_ERR_HIP = 4
SEELE_EXTENT_3SIGMA = 0
SEELE_EXTENT_OPACITY = 1
SEELE_RASTER_PLAIN = 0
SEELE_RASTER_CONTRIB = 1
SEELE_BIN_SUPER = 1
SEELE_BIN_STAGED = 2
SEELE_QUEUE_LIST = 0
SEELE_QUEUE_HEAVIEST_FIRST = 1
SEELE_NOALLOC_SCRATCH_BYTES = 64 << 20


class seele_gaussians(ctypes.Structure):
    _fields_ = [("n", c_int64), ("sh_degree", c_int32), ("reserved", c_int32),
                ("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p),
                ("opacity_logits", c_void_p), ("sh", c_void_p)]


class seele_gaussian_grads(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p),
                ("opacity_logits", c_void_p), ("sh", c_void_p)]


class seele_adam_opts(ctypes.Structure):
    _fields_ = [("lr_means", c_float), ("lr_log_scales", c_float), ("lr_quats", c_float),
                ("lr_opacity", c_float), ("lr_sh_dc", c_float), ("lr_sh_rest", c_float),
                ("beta1", c_float), ("beta2", c_float), ("eps", c_float)]


class seele_camera(ctypes.Structure):
    _fields_ = [("R", c_float * 9), ("t", c_float * 3), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("width", c_int32), ("height", c_int32)]


class seele_splat(ctypes.Structure):
    _fields_ = [("mean_x", c_float), ("mean_y", c_float), ("chol_l11", c_float),
                ("chol_l21", c_float), ("chol_l22", c_float), ("opacity", c_float),
                ("r", c_float), ("g", c_float), ("b", c_float), ("conic_a", c_float),
                ("conic_b", c_float), ("conic_c", c_float), ("depth", c_float),
                ("rect_x", ctypes.c_uint32), ("rect_y", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class seele_preprocess_opts(ctypes.Structure):
    _fields_ = [("tile", c_int32), ("extent", c_int32), ("alpha_min", c_float),
                ("lowpass", c_float), ("z_near", c_float), ("n_segs", c_int32),
                ("seg_begin", POINTER(c_int64)), ("seg_count", POINTER(c_int64))]


class seele_raster_opts(ctypes.Structure):
    _fields_ = [("tile", c_int32), ("mode", c_int32), ("group_w", c_int32), ("group_h", c_int32),
                ("lds_batch", c_int32), ("alpha_min", c_float), ("alpha_max", c_float),
                ("T_min", c_float), ("bg", c_float * 3)]


SIGNATURES = {
    "seele_total_tiles": (c_int64, [POINTER(seele_camera), c_int32, c_int32]),
    "seele_preprocess": (c_int32, [POINTER(seele_gaussians), POINTER(seele_camera), c_int32,
                                   POINTER(seele_preprocess_opts), c_void_p, c_void_p, c_void_p]),
    "seele_bin_sort_workspace_size": (c_size_t, [c_int64, c_int64, c_int64]),
    "seele_bin_sort": (c_int32, [c_void_p, c_void_p, c_int64, POINTER(seele_camera), c_int32,
                                 c_int32, c_void_p, c_size_t, c_void_p, c_int64, c_void_p,
                                 c_void_p, c_void_p]),
    "seele_total_super_tiles": (c_int64, [POINTER(seele_camera), c_int32, c_int32]),
    "seele_preprocess_staged": (c_int32, [POINTER(seele_gaussians), POINTER(seele_camera),
                                          c_int32, POINTER(seele_preprocess_opts), c_void_p,
                                          c_void_p, c_void_p, c_size_t, c_int64, c_void_p]),
    "seele_bin_sort_ex": (c_int32, [c_int32, c_void_p, c_void_p, c_int64, POINTER(seele_camera),
                                    c_int32, c_int32, c_void_p, c_size_t, c_void_p, c_void_p,
                                    c_int64, c_void_p, c_void_p, c_void_p]),
    "seele_bin_sort_noalloc": (c_int32, [c_int32, c_void_p, c_void_p, c_int64,
                                         POINTER(seele_camera), c_int32, c_int32, c_void_p,
                                         c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
    "seele_bin_sort_super": (c_int32, [c_void_p, c_void_p, c_int64, POINTER(seele_camera),
                                       c_int32, c_int32, c_void_p, c_size_t, c_void_p, c_void_p,
                                       c_int64, c_void_p, c_void_p, c_void_p]),
    "seele_rasterize_fwd": (c_int32, [c_void_p, c_void_p, c_void_p, POINTER(seele_camera),
                                      c_int32, POINTER(seele_raster_opts), c_void_p, c_void_p,
                                      c_void_p, c_void_p]),
    "seele_rasterize_fwd_super": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p,
                                            POINTER(seele_camera), c_int32,
                                            POINTER(seele_raster_opts), c_void_p, c_void_p,
                                            c_void_p, c_void_p, c_void_p, c_void_p]),
    "seele_contrib_topk": (c_int32, [c_void_p, c_void_p, c_void_p, POINTER(seele_camera), c_int32,
                                     c_int64, POINTER(seele_raster_opts), c_int32, c_void_p,
                                     c_void_p, c_void_p]),
    "seele_raster_queue_workspace_size": (c_size_t, [c_int64]),
    "seele_rasterize_fwd_queue": (c_int32, [c_void_p, c_void_p, c_void_p, POINTER(seele_camera),
                                            c_int32, POINTER(seele_raster_opts), c_int32,
                                            c_void_p, c_size_t, c_void_p, c_void_p, c_void_p,
                                            c_void_p]),
    "seele_rasterize_fwd_counted": (c_int32, [c_void_p, c_void_p, c_void_p, POINTER(seele_camera),
                                              c_int32, POINTER(seele_raster_opts), c_void_p,
                                              c_void_p, c_void_p, c_void_p, c_void_p]),
    "seele_rasterize_bwd_super": (c_int32, [POINTER(seele_gaussians), POINTER(seele_camera),
                                            c_int32, POINTER(seele_preprocess_opts),
                                            POINTER(seele_raster_opts), c_void_p, c_void_p,
                                            c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                            c_void_p, c_void_p, POINTER(seele_gaussian_grads),
                                            c_void_p]),
    "seele_rasterize_bwd": (c_int32, [POINTER(seele_gaussians), POINTER(seele_camera), c_int32,
                                      POINTER(seele_preprocess_opts), POINTER(seele_raster_opts),
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p, POINTER(seele_gaussian_grads),
                                      c_void_p]),
    "seele_hp_kmeans": (c_int32, [POINTER(seele_camera), c_int32, c_float, c_float, c_int32,
                                  c_int32, POINTER(c_float), POINTER(c_int32)]),
    "seele_hp_pos_scale": (c_float, [POINTER(seele_camera), c_int32]),
    "seele_hp_accumulate": (c_int32, [c_void_p, c_void_p, c_int32, c_int64, c_int32, c_void_p,
                                      c_void_p, c_void_p, c_void_p]),
    "seele_hp_partition": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_int32,
                                     POINTER(c_int64), POINTER(c_int64), POINTER(c_int64)]),
    "seele_gather_gaussians": (c_int32, [POINTER(seele_gaussians), c_void_p, c_int64,
                                         POINTER(seele_gaussian_grads), c_void_p]),
    "seele_pose_extrapolate": (c_int32, [POINTER(seele_camera), POINTER(seele_camera), c_float,
                                         POINTER(seele_camera)]),
    "seele_resident_plan": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_int32, c_int64,
                                      c_void_p, c_int32, c_void_p, c_int32, c_int64, c_void_p,
                                      c_void_p, POINTER(c_int32), POINTER(c_int32)]),
    "seele_load_segments": (c_int32, [c_void_p, c_int64, c_void_p, c_int64, c_int32, c_void_p,
                                      c_void_p, c_void_p, c_int32, c_void_p]),
    "seele_photometric_loss_workspace_size": (c_size_t, [POINTER(seele_camera), c_int32]),
    "seele_photometric_loss": (c_int32, [c_void_p, c_void_p, POINTER(seele_camera), c_int32,
                                         c_float, c_void_p, c_size_t, c_void_p, c_void_p,
                                         c_void_p]),
    "seele_adam_step": (c_int32, [POINTER(seele_gaussian_grads), POINTER(seele_gaussian_grads),
                                  POINTER(seele_gaussian_grads), POINTER(seele_gaussian_grads),
                                  c_int64, c_int32, POINTER(seele_adam_opts), c_int64, c_void_p]),
    "seele_flip_loss_workspace_size": (c_size_t, [POINTER(seele_camera), c_int32]),
    "seele_flip_loss": (c_int32, [c_void_p, c_void_p, POINTER(seele_camera), c_int32, c_float,
                                  c_float, c_int32, c_void_p, c_size_t, c_void_p, c_void_p,
                                  c_void_p]),
    "seele_spatial_order_workspace_size": (c_size_t, [c_int64]),
    "seele_spatial_order": (c_int32, [POINTER(seele_gaussians), c_void_p, c_size_t, c_void_p,
                                      c_void_p]),
    "seele_hp_select": (c_int32, [POINTER(c_float), c_int32, POINTER(seele_camera), c_float,
                                  c_float, c_int32, POINTER(c_int32)]),
    "seele_hp_segments": (c_int32, [POINTER(c_int64), POINTER(c_int64), c_int32, POINTER(c_int32),
                                    c_int32, POINTER(c_int64), POINTER(c_int64), POINTER(c_int32)]),
    "seele_last_error": (c_char_p, []),
    "seele_status_string": (c_char_p, [c_int32]),
    "seele_abi_version": (c_int32, []),
}

_lib = None


def lib():
    """Load libseele.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2503_05168_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class SeeleError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = L.seele_last_error().decode(errors="replace")
        name = L.seele_status_string(status).decode()
        super().__init__(f"{where}: {name}: {msg}")
        self.status = status


def check(status: int, where: str):
    if status != SEELE_OK:
        raise SeeleError(status, where)


def make_camera(cam) -> seele_camera:
    """Any object with R (3x3), t (3), fx, fy, cx, cy, width, height."""
    c = seele_camera()
    R = [float(x) for row in cam.R for x in row]
    for i in range(9):
        c.R[i] = R[i]
    for i in range(3):
        c.t[i] = float(cam.t[i])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def camera_array(cams):
    arr = (seele_camera * len(cams))()
    for i, cam in enumerate(cams):
        arr[i] = make_camera(cam)
    return arr
